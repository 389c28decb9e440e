// In-block hopping terms with the block resident in LDS, shared by the
// block solvers and the block-determinant kernels.
#pragma once

#include "stencil.h"

namespace wdr {
namespace {

using namespace dev;

// loader for in-block neighbours of the opposite parity, from an LDS half
// field laid out [12][Vh]; `off` is subtracted from the local index
template <typename T> struct LdsLoader {
    const typename C2<T>::type *sh;
    int Vh, off;
    __device__ __forceinline__ void operator()(int, int nl, spinor<T> &p) const
    {
        const int i = nl - off;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) p.s[sp].c[a] = ld<T>(sh, (long)(3 * sp + a) * Vh + i);
    }
};

template <typename T>
__device__ __forceinline__ void lds_store(typename C2<T>::type *sh, int Vh, int i, const spinor<T> &p)
{
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) st<T>(sh, (long)(3 * sp + a) * Vh + i, p.s[sp].c[a]);
}

// ---------------------------------------------------------------- B^4 blocks
// A B^4 block resident in LDS: both spinor halves and the first two rows of
// U_mu(x) for every site (the third row is rebuilt as conj(row0 x row1), so
// the links must be SU(3); in-block links never carry the boundary phase,
// since a block never wraps around the lattice).  LDS: 2 x 12 x Vh spinor
// entries + 4 x 6 x Vb link entries (FP32 74 KB, FP64 147 KB for 4^4).

template <typename T, int B> struct CubeLds {
    typedef typename C2<T>::type T2;
    static constexpr int Vb = Cube<B>::Vb, Vh = Cube<B>::Vh;
    T2 she[12 * Vh];
    T2 sho[12 * Vh];
    T2 lk[4 * 6 * Vb];
    T red[3][Vb / 64 > 0 ? Vb / 64 : 1];
    T alpha[2];
};

template <typename T>
__device__ __forceinline__ void reconstruct(su3<T> &u)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int a = (c + 1) % 3, b = (c + 2) % 3;
        const cx<T> v = u.m[0][a] * u.m[1][b] - u.m[0][b] * u.m[1][a];
        u.m[2][c] = mk<T>(v.re, -v.im);
    }
}

template <typename T, int B>
__device__ __forceinline__ void lds_link(const typename C2<T>::type *lk, int mu, int l, su3<T> &u)
{
    constexpr int Vb = Cube<B>::Vb;
#pragma unroll
    for (int e = 0; e < 6; ++e) u.m[e / 3][e % 3] = ld<T>(lk, (long)(mu * 6 + e) * Vb + l);
    reconstruct(u);
}

// one direction (compile-time MU) of the in-block hop sum at site l (coords
// x): both hops that stay inside the block, neighbour spinors from the LDS
// half field sh (opposite parity, local index minus off), links from LDS;
// added to acc
template <typename T, int B, int MU>
__device__ __forceinline__ void hop_dir_lds(const typename C2<T>::type *sh, int off, const typename C2<T>::type *lk,
                                            int l, const int x[4], spinor<T> &acc)
{
    typedef Cube<B> CB;
    LdsLoader<T> ldr{sh, CB::Vh, off};
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        const bool fwd = dir == 0;
        if (fwd ? x[MU] + 1 >= B : x[MU] == 0) continue;
        int y[4] = {x[0], x[1], x[2], x[3]};
        y[MU] += fwd ? 1 : -1;
        const int nl = CB::index(y);
        spinor<T> p;
        ldr(0, nl, p);
        vec3<T> a0, a1;
        A_dn(MU, p.s[2], p.s[3], a0, a1);
        vec3<T> h0, h1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            h0.c[a] = fwd ? p.s[0].c[a] - a0.c[a] : p.s[0].c[a] + a0.c[a];
            h1.c[a] = fwd ? p.s[1].c[a] - a1.c[a] : p.s[1].c[a] + a1.c[a];
        }
        su3<T> u;
        lds_link<T, B>(lk, MU, fwd ? l : nl, u);
        const vec3<T> c0 = fwd ? mul(u, h0) : mul_dag(u, h0);
        const vec3<T> c1 = fwd ? mul(u, h1) : mul_dag(u, h1);
        vec3<T> d0, d1;
        Adag_h(MU, c0, c1, d0, d1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            acc.s[0].c[a] = acc.s[0].c[a] + c0.c[a];
            acc.s[1].c[a] = acc.s[1].c[a] + c1.c[a];
            acc.s[2].c[a] = fwd ? acc.s[2].c[a] - d0.c[a] : acc.s[2].c[a] + d0.c[a];
            acc.s[3].c[a] = fwd ? acc.s[3].c[a] - d1.c[a] : acc.s[3].c[a] + d1.c[a];
        }
    }
}

template <typename T, int B>
__device__ __forceinline__ void hop_dir_lds_rt(int mu, const typename C2<T>::type *sh, int off,
                                               const typename C2<T>::type *lk, int l, const int x[4], spinor<T> &acc)
{
    switch (mu) {
    case 0: hop_dir_lds<T, B, 0>(sh, off, lk, l, x, acc); break;
    case 1: hop_dir_lds<T, B, 1>(sh, off, lk, l, x, acc); break;
    case 2: hop_dir_lds<T, B, 2>(sh, off, lk, l, x, acc); break;
    default: hop_dir_lds<T, B, 3>(sh, off, lk, l, x, acc); break;
    }
}

// The two in-block hops of direction MU at one site with the links held in
// registers: uf = U_mu(x), ub = U_mu(x - mu) (all three rows), nf / nb the
// LDS indices (in sh, [12][Vh]) of x + mu and x - mu.  A hop that leaves the
// block comes with a zero link and a valid index, so both hops are always
// taken and no lane branches.  Their sum is written to acc.
template <typename T, int MU>
__device__ __forceinline__ void hop_dir_reg(const typename C2<T>::type *sh, int Vh, const su3<T> &uf,
                                            const su3<T> &ub, int nf, int nb, spinor<T> &acc)
{
    LdsLoader<T> ldr{sh, Vh, 0};
    vec3<T> lo0, lo1;  // spins 2, 3 of the forward hop before their sign
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        const bool fwd = dir == 0;
        const int nl = fwd ? nf : nb;
        spinor<T> p;
        ldr(0, nl, p);
        vec3<T> a0, a1;
        A_dn(MU, p.s[2], p.s[3], a0, a1);
        vec3<T> h0, h1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            h0.c[a] = fwd ? p.s[0].c[a] - a0.c[a] : p.s[0].c[a] + a0.c[a];
            h1.c[a] = fwd ? p.s[1].c[a] - a1.c[a] : p.s[1].c[a] + a1.c[a];
        }
        const vec3<T> c0 = fwd ? mul(uf, h0) : mul_dag(ub, h0);
        const vec3<T> c1 = fwd ? mul(uf, h1) : mul_dag(ub, h1);
        vec3<T> d0, d1;
        Adag_h(MU, c0, c1, d0, d1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (fwd) {
                acc.s[0].c[a] = c0.c[a];
                acc.s[1].c[a] = c1.c[a];
                lo0.c[a] = d0.c[a];
                lo1.c[a] = d1.c[a];
            } else {
                acc.s[0].c[a] = acc.s[0].c[a] + c0.c[a];
                acc.s[1].c[a] = acc.s[1].c[a] + c1.c[a];
                acc.s[2].c[a] = d0.c[a] - lo0.c[a];
                acc.s[3].c[a] = d1.c[a] - lo1.c[a];
            }
        }
    }
}

// in-block hop sum at site l over all four directions
template <typename T, int B>
__device__ __forceinline__ void hop_in_lds(const typename C2<T>::type *sh, int off, const typename C2<T>::type *lk,
                                           int l, const int x[4], spinor<T> &acc)
{
    zero(acc);
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) hop_dir_lds_rt<T, B>(mu, sh, off, lk, l, x, acc);
}

}  // namespace
}  // namespace wdr
