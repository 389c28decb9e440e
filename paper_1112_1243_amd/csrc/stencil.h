// Per-site Wilson hopping sum (device inline), shared by the global stencil
// and the LDS-resident block solvers.
//
//   H psi(x) = sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ]
//
// restricted to the hops selected by HOPS (all / inside the block / across
// a block boundary).  The neighbour spinor comes from a loader functor
// ld(slot, local_index), so the same code reads global memory or LDS.
#pragma once

#include "ops.h"

namespace wdr {
namespace dev {

__device__ __forceinline__ int lexi(const Geo &g, int x0, int x1, int x2, int x3)
{
    return x0 + g.B[0] * (x1 + g.B[1] * (x2 + g.B[2] * x3));
}

__device__ __forceinline__ void local_coords(const Geo &g, int l, int x[4])
{
    const uint32_t c = g.loc_coord[l];
    x[0] = (int)(c & 255u);
    x[1] = (int)((c >> 8) & 255u);
    x[2] = (int)((c >> 16) & 255u);
    x[3] = (int)(c >> 24);
}

template <typename T>
__device__ __forceinline__ void load_link(const typename C2<T>::type *U, int slot, int mu, int Vb, int l, su3<T> &u)
{
    const long base = ((long)slot * 4 + mu) * 9 * Vb + l;
    const auto *Ug = as_global(U);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) u.m[a][b] = ldg<T>(Ug, base + (long)(3 * a + b) * Vb);
}

template <typename T> __device__ __forceinline__ void zero(spinor<T> &p)
{
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) p.s[sp].c[a] = mk<T>(0, 0);
}

template <typename T, int HOPS, class Loader>
__device__ __forceinline__ void hop_sum(const Geo &g, const typename C2<T>::type *__restrict__ U, int slot, int l,
                                        const int x[4], Loader &&ldr, spinor<T> &acc)
{
    const int Vb = g.Vb;
    zero(acc);
    // the direction loop stays rolled: unrolled, the compiler hoists the
    // loads of all eight hops and runs out of registers
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        {   // forward: (1 - g_mu) U_mu(x) psi(x + mu)
            const bool inside = x[mu] + 1 < g.B[mu];
            if (HOPS == HOPS_ALL || (HOPS == HOPS_IN && inside) || (HOPS == HOPS_CROSS && !inside)) {
                int y[4] = {x[0], x[1], x[2], x[3]};
                y[mu] = inside ? x[mu] + 1 : 0;
                const int ns = inside ? slot : g.slot_nbr[slot * 8 + 2 * mu];
                const int nl = g.loc_index[lexi(g, y[0], y[1], y[2], y[3])];
                spinor<T> p;
                ldr(ns, nl, p);
                vec3<T> a0, a1;
                A_dn(mu, p.s[2], p.s[3], a0, a1);
                vec3<T> h0, h1;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    h0.c[a] = p.s[0].c[a] - a0.c[a];
                    h1.c[a] = p.s[1].c[a] - a1.c[a];
                }
                su3<T> u;
                load_link<T>(U, slot, mu, Vb, l, u);
                const vec3<T> c0 = mul(u, h0), c1 = mul(u, h1);
                vec3<T> d0, d1;
                Adag_h(mu, c0, c1, d0, d1);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    acc.s[0].c[a] = acc.s[0].c[a] + c0.c[a];
                    acc.s[1].c[a] = acc.s[1].c[a] + c1.c[a];
                    acc.s[2].c[a] = acc.s[2].c[a] - d0.c[a];
                    acc.s[3].c[a] = acc.s[3].c[a] - d1.c[a];
                }
            }
        }
        {   // backward: (1 + g_mu) U_mu(x - mu)^+ psi(x - mu)
            const bool inside = x[mu] > 0;
            if (HOPS == HOPS_ALL || (HOPS == HOPS_IN && inside) || (HOPS == HOPS_CROSS && !inside)) {
                int y[4] = {x[0], x[1], x[2], x[3]};
                y[mu] = inside ? x[mu] - 1 : g.B[mu] - 1;
                const int ns = inside ? slot : g.slot_nbr[slot * 8 + 2 * mu + 1];
                const int nl = g.loc_index[lexi(g, y[0], y[1], y[2], y[3])];
                spinor<T> p;
                ldr(ns, nl, p);
                vec3<T> a0, a1;
                A_dn(mu, p.s[2], p.s[3], a0, a1);
                vec3<T> h0, h1;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    h0.c[a] = p.s[0].c[a] + a0.c[a];
                    h1.c[a] = p.s[1].c[a] + a1.c[a];
                }
                su3<T> u;
                load_link<T>(U, ns, mu, Vb, nl, u);
                const vec3<T> c0 = mul_dag(u, h0), c1 = mul_dag(u, h1);
                vec3<T> d0, d1;
                Adag_h(mu, c0, c1, d0, d1);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    acc.s[0].c[a] = acc.s[0].c[a] + c0.c[a];
                    acc.s[1].c[a] = acc.s[1].c[a] + c1.c[a];
                    acc.s[2].c[a] = acc.s[2].c[a] + d0.c[a];
                    acc.s[3].c[a] = acc.s[3].c[a] + d1.c[a];
                }
            }
        }
    }
}

// ---------------------------------------------------------------- cubic blocks
// Compile-time geometry of a B^4 block (even sites first, lexicographic in
// each parity), so neighbour indices are integer arithmetic instead of
// table lookups.
template <int B> struct Cube {
    static constexpr int Vb = B * B * B * B, Vh = Vb / 2, H = B / 2;
    __device__ static __forceinline__ void coords(int l, int x[4])
    {
        const int p = l >= Vh ? 1 : 0;
        const int idx = l - p * Vh;
        int r = idx / H;
        x[1] = r % B;
        r /= B;
        x[2] = r % B;
        x[3] = r / B;
        x[0] = 2 * (idx % H) + ((p + x[1] + x[2] + x[3]) & 1);
    }
    __device__ static __forceinline__ int index(const int x[4])
    {
        const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
        return p * Vh + ((x[3] * B + x[2]) * B + x[1]) * H + (x[0] >> 1);
    }
};

// Loaders of the hop bodies below.  A spinor loader returns component c of
// site nl of slot ns; a link loader returns entry e (row-major, e < 6 suffices
// for two-row reads) of the link (slot, mu) at site l.  Offsets are 32-bit
// element indices from the system's base pointer; `pin` is added to every
// offset (see hop_sum_cube).
template <typename T, int Vb> struct SpinorLd {
    const __attribute__((address_space(1))) typename C2<T>::type *p;
    int pin;
    __device__ __forceinline__ cx<T> operator()(int ns, int c, int nl) const
    {
        return ldg<T>(p, ns * 12 * Vb + nl + pin + c * Vb);
    }
};
template <typename T, int Vb> struct LinkLd {  // [slot][mu][9][Vb]
    const __attribute__((address_space(1))) typename C2<T>::type *p;
    int pin;
    __device__ __forceinline__ cx<T> operator()(int sl, int mu, int e, int l) const
    {
        return ldg<T>(p, (sl * 4 + mu) * 9 * Vb + l + pin + e * Vb);
    }
};
template <int Vb> struct SpinorLdH {  // FP16 with a scale per slot
    const __attribute__((address_space(1))) h2 *p;
    const float *scale;
    __device__ __forceinline__ cx<float> operator()(int ns, int c, int nl) const
    {
        return ldh(p, ns * 12 * Vb + nl + c * Vb, scale[ns]);
    }
};
template <int Vb> struct LinkLdH {  // FP16, first two rows: [slot][mu][6][Vb]
    const __attribute__((address_space(1))) h2 *p;
    __device__ __forceinline__ cx<float> operator()(int sl, int mu, int e, int l) const
    {
        return ldh(p, (sl * 4 + mu) * 6 * Vb + l + e * Vb, 1.f);
    }
};

// One direction mu (compile time) of the hop sum at a site of a B^4 block:
// the forward hop (1 - g_mu) U_mu(x) psi(x + mu) and the backward hop
// (1 + g_mu) U_mu(x - mu)^+ psi(x - mu), added to acc.
//
// R2: read only the first two rows of each link and rebuild the third as the
// conjugated cross product of the first two (valid for SU(3) links), times
// the boundary sign for links that wrap around the lattice; wrap_f / wrap_b
// are that sign for the forward and the backward link of this site.
template <typename T, int HOPS, int B, int DAG, int MU, int R2, class SpL, class LkL>
__device__ __forceinline__ void hop_dir_ld(const SpL &in, const LkL &U, int slot, const int nbr[8], int l,
                                           const int x[4], spinor<T> &acc, T wrap_f, T wrap_b)
{
    typedef Cube<B> CB;
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        const bool fwd = dir == 0;
        const bool inside = fwd ? x[MU] + 1 < B : x[MU] > 0;
        if (HOPS == HOPS_IN && !inside) continue;
        if (HOPS == HOPS_CROSS && inside) continue;
        int y[4] = {x[0], x[1], x[2], x[3]};
        y[MU] = fwd ? (inside ? x[MU] + 1 : 0) : (inside ? x[MU] - 1 : B - 1);
        const int ns = inside ? slot : nbr[2 * MU + dir];
        const int nl = CB::index(y);
        spinor<T> p;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) p.s[sp].c[a] = in(ns, 3 * sp + a, nl);
        su3<T> u;
#pragma unroll
        for (int e = 0; e < (R2 ? 6 : 9); ++e) u.m[e / 3][e % 3] = U(fwd ? slot : ns, MU, e, fwd ? l : nl);
        if (R2) {
            const T sg = fwd ? wrap_f : wrap_b;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int a = (c + 1) % 3, b = (c + 2) % 3;
                const cx<T> v = u.m[0][a] * u.m[1][b] - u.m[0][b] * u.m[1][a];
                u.m[2][c] = mk<T>(sg * v.re, -sg * v.im);
            }
        }
        if (DAG) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                p.s[2].c[a] = neg(p.s[2].c[a]);
                p.s[3].c[a] = neg(p.s[3].c[a]);
            }
        }
        vec3<T> a0, a1;
        A_dn(MU, p.s[2], p.s[3], a0, a1);
        vec3<T> h0, h1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            h0.c[a] = fwd ? p.s[0].c[a] - a0.c[a] : p.s[0].c[a] + a0.c[a];
            h1.c[a] = fwd ? p.s[1].c[a] - a1.c[a] : p.s[1].c[a] + a1.c[a];
        }
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

// hop_dir_ld on fields of the internal layout (FP32 / FP64 storage)
template <typename T, int HOPS, int B, int DAG, int MU, int R2 = 0>
__device__ __forceinline__ void hop_dir_cube(const __attribute__((address_space(1))) typename C2<T>::type *U,
                                             const __attribute__((address_space(1))) typename C2<T>::type *in,
                                             int slot, const int nbr[8], int l, const int x[4], int pin,
                                             spinor<T> &acc, T wrap_f = 1, T wrap_b = 1)
{
    constexpr int Vb = Cube<B>::Vb;
    hop_dir_ld<T, HOPS, B, DAG, MU, R2>(SpinorLd<T, Vb>{in, pin}, LinkLd<T, Vb>{U, pin}, slot, nbr, l, x, acc,
                                        wrap_f, wrap_b);
}

// hop sum for B^4 blocks; nbr[8] are the neighbour slots of this block
// (uniform over the workgroup).  The direction loop stays rolled (all eight
// hops in flight need more registers than occupancy allows) and dispatches
// on the uniform direction to a compile-time specialised body, so the spin
// projections are plain register moves and each hop's spinor and link loads
// issue together.  DAG applies gamma5 to the loaded spinors (the caller
// applies it to the result).
template <typename T, int HOPS, int B, int DAG>
__device__ __forceinline__ void hop_sum_cube(const typename C2<T>::type *__restrict__ U,
                                             const typename C2<T>::type *__restrict__ in, int slot, const int nbr[8],
                                             int l, const int x[4], spinor<T> &acc)
{
    const auto *Ug = as_global(U);
    const auto *ing = as_global(in);
    zero(acc);
    // The loop stays rolled and every iteration's loads stay in it: their
    // addresses carry `pin`, a zero the compiler cannot see through, so the
    // loads of all four directions are not hoisted (and kept live) together.
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        int pin = 0;
        asm volatile("" : "+s"(pin));
        switch (mu) {
        case 0: hop_dir_cube<T, HOPS, B, DAG, 0>(Ug, ing, slot, nbr, l, x, pin, acc); break;
        case 1: hop_dir_cube<T, HOPS, B, DAG, 1>(Ug, ing, slot, nbr, l, x, pin, acc); break;
        case 2: hop_dir_cube<T, HOPS, B, DAG, 2>(Ug, ing, slot, nbr, l, x, pin, acc); break;
        default: hop_dir_cube<T, HOPS, B, DAG, 3>(Ug, ing, slot, nbr, l, x, pin, acc); break;
        }
    }
}

// loader from a global field in the internal layout
template <typename T> struct GlobalLoader {
    const typename C2<T>::type *f;
    int Vb;
    __device__ __forceinline__ void operator()(int ns, int nl, spinor<T> &p) const
    {
        const long base = (long)ns * 12 * Vb + nl;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) p.s[sp].c[a] = ld<T>(f, base + (long)(3 * sp + a) * Vb);
    }
};

template <typename T>
__device__ __forceinline__ void load_site(const typename C2<T>::type *f, int slot, int Vb, int l, spinor<T> &p)
{
    GlobalLoader<T>{f, Vb}(slot, l, p);
}
template <typename T>
__device__ __forceinline__ void store_site(typename C2<T>::type *f, int slot, int Vb, int l, const spinor<T> &p)
{
    const long base = (long)slot * 12 * Vb + l;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) st<T>(f, base + (long)(3 * sp + a) * Vb, p.s[sp].c[a]);
}

}  // namespace dev
}  // namespace wdr
