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
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) u.m[a][b] = ld<T>(U, base + (long)(3 * a + b) * Vb);
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
