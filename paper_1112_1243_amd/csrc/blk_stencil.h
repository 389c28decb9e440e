// Device bodies of the block-staged stencil on B^4 blocks (one workgroup
// per block, the block's input staged in LDS), shared by the stencil kernels
// and the fused solver kernels.
#pragma once

#include "clover.h"
#include "stencil.h"

namespace wdr {
namespace dev {

// The two hops of direction MU at site l: in-block neighbours from the LDS
// copy sh ([12][NS], entry (c, nl - off)), the others from global memory;
// DAG applies gamma_5 to the loaded spinors (the caller to the result).
template <typename T, int B, int MU, int HOPS, int DAG, int NS>
__device__ __forceinline__ void hop_blk(const T2<T> *sh, int off, const __attribute__((address_space(1))) T2<T> *in,
                                        const __attribute__((address_space(1))) T2<T> *Ug, int slot, const int nbr[8],
                                        int l, const int x[4], int pin, spinor<T> &acc, T wrap_f, T wrap_b)
{
    typedef Cube<B> CB;
    constexpr int Vb = CB::Vb;
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        const bool fwd = dir == 0;
        const bool inside = fwd ? x[MU] + 1 < B : x[MU] > 0;
        if (HOPS == HOPS_IN && !inside) continue;
        int y[4] = {x[0], x[1], x[2], x[3]};
        y[MU] = fwd ? (inside ? x[MU] + 1 : 0) : (inside ? x[MU] - 1 : B - 1);
        const int ns = inside ? slot : nbr[2 * MU + dir];
        const int nl = CB::index(y);
        spinor<T> p;
        if (inside) {
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int a = 0; a < 3; ++a) p.s[sp].c[a] = ld<T>(sh, (3 * sp + a) * NS + nl - off);
        } else {
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int a = 0; a < 3; ++a) p.s[sp].c[a] = ldg<T>(in, ns * 12 * Vb + nl + pin + (3 * sp + a) * Vb);
        }
        su3<T> u;
        const int ls = fwd ? slot : ns, ll = fwd ? l : nl;
#pragma unroll
        for (int e = 0; e < 6; ++e) u.m[e / 3][e % 3] = ldg<T>(Ug, (ls * 4 + MU) * 9 * Vb + ll + pin + e * Vb);
        const T sg = fwd ? wrap_f : wrap_b;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int a = (c + 1) % 3, b = (c + 2) % 3;
            const cx<T> v = u.m[0][a] * u.m[1][b] - u.m[0][b] * u.m[1][a];
            u.m[2][c] = mk<T>(sg * v.re, -sg * v.im);
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

// The even-odd halves of the block-staged stencil: out = diag - kappa
// H_{par, 1-par} in on the sites of parity par, with gamma_5 on both sides
// for DAG.  One workgroup per block, one lane per output site; the block's
// input sites of the other parity are read once into LDS (sh).
// blk_eo_block is one workgroup's block (system m, slot `slot`, lane t =
// threadIdx.x); with NRM it returns the lane's |out|^2 in FP64 (0
// otherwise).  It ends with the LDS still in use: a caller that runs it
// again on the same sh synchronises the workgroup first.
template <typename T, int B, int DAG, int CL, int NRM>
__device__ __forceinline__ double blk_eo_block(const Geo &g, int m, int slot, int t, UTab<T> Utab,
                                               const double *__restrict__ kap, int kneg,
                                               const T *const *__restrict__ ctab, long n, int par,
                                               const T2<T> *__restrict__ in, const T2<T> *__restrict__ diag,
                                               T2<T> *__restrict__ out, T kappa, T2<T> (*sh)[Cube<B>::Vh])
{
    typedef Cube<B> CB;
    constexpr int Vb = CB::Vb, Vh = CB::Vh;
    if (kap) kappa = kneg ? -(T)kap[m] : (T)kap[m];
    const int off = (1 - par) * Vh;  // first local index of the input parity
    const auto *Ug = as_global(Utab[m]);
    const auto *ing = as_global(in + m * n);
    const long sbase = (long)slot * 12 * Vb;
#pragma unroll
    for (int c = 0; c < 12; ++c) st<T>(&sh[c][0], t, ldg<T>(ing, sbase + off + t + c * Vb));
    const int l = par * Vh + t;
    int x[4];
    CB::coords(l, x);
    int nbr[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) nbr[k] = g.slot_nbr[slot * 8 + k];
    const int bl = g.slot_blk[slot];
    __syncthreads();
    spinor<T> acc;
    zero(acc);
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        int pin = 0;
        asm volatile("" : "+s"(pin));
        T wf = 1, wb = 1;
        if (g.bc[mu] < 0) {
            int b2 = bl;
            for (int d = 0; d < mu; ++d) b2 /= g.NB[d];
            const int nmu = b2 % g.NB[mu];
            if (nmu == g.NB[mu] - 1 && x[mu] == B - 1) wf = -1;
            if (nmu == 0 && x[mu] == 0) wb = -1;
        }
        switch (mu) {
        case 0: hop_blk<T, B, 0, HOPS_ALL, DAG, Vh>(&sh[0][0], off, ing, Ug, slot, nbr, l, x, pin, acc, wf, wb); break;
        case 1: hop_blk<T, B, 1, HOPS_ALL, DAG, Vh>(&sh[0][0], off, ing, Ug, slot, nbr, l, x, pin, acc, wf, wb); break;
        case 2: hop_blk<T, B, 2, HOPS_ALL, DAG, Vh>(&sh[0][0], off, ing, Ug, slot, nbr, l, x, pin, acc, wf, wb); break;
        default: hop_blk<T, B, 3, HOPS_ALL, DAG, Vh>(&sh[0][0], off, ing, Ug, slot, nbr, l, x, pin, acc, wf, wb); break;
        }
    }
    const long obase = m * n + sbase + l;
    double nrm = 0;
    if (CL) {
        cx<T> v[12], dg[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            v[c] = scale(-kappa, acc.s[c / 3].c[c % 3]);
            if (DAG && c >= 6) v[c] = neg(v[c]);
            dg[c] = diag ? ld<T>(diag, obase + (long)c * Vb) : mk<T>(0, 0);
        }
        clov_site<T, CL>(ctab[m], (long)g.V, slot, Vb, l, dg, v);
#pragma unroll
        for (int c = 0; c < 12; ++c) st_nt<T>(out, obase + (long)c * Vb, v[c]);
        return nrm;
    }
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const long i = obase + (long)(3 * sp + a) * Vb;
            cx<T> v = scale(-kappa, acc.s[sp].c[a]);
            if (DAG && sp >= 2) v = neg(v);
            if (diag) v = v + ld<T>(diag, i);
            st_nt<T>(out, i, v);
            if (NRM) nrm += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
        }
    return nrm;
}


}  // namespace dev
}  // namespace wdr
