// Block minimal-residual solver and Schwarz sweep for gfx950.
//
// Domain decomposition (paper Sec. 3) with the Schwarz alternating
// procedure of Luscher (hep-lat/0310048, cited in Secs. 1 and 3).  One
// workgroup owns one block of Vb <= 256 sites, one lane per site (even
// sites in the first half of the workgroup, odd sites in the second, so the
// two halves are separate wavefronts).  The even-odd reduced block system
//     (1 - kappa^2 H_eo H_oe) d_e = r_e + kappa H_eo r_o,
//     d_o = r_o + kappa H_oe d_e,                    (D_b = 1 - kappa H_b)
// is solved by MR steps with both half fields resident in LDS; only the
// links are read from global memory (they stay in L2 across the steps).
// Per-block inner products are wavefront shuffles plus an LDS tree.
#include "stencil.h"

namespace wdr {
namespace {

using namespace dev;

constexpr int MAXVB = 256;

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

// sum over the first `width` lanes (width = 16, 32 or 64: blocks smaller
// than a wavefront have a partial wavefront of a power-of-two size)
template <typename T> __device__ __forceinline__ T wave_sum(T v, int width)
{
    for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_down(v, off, width);
    return v;
}

// MODE 0: Schwarz sweep on one colour: r = eta - D x (global stencil on x),
//         MR on the block, x += d.
// MODE 1: block MR for a given right-hand side: d = MR(D_b, rhs).
template <typename T, int MODE>
__global__ __launch_bounds__(MAXVB) void k_block_mr(Geo g, const typename C2<T>::type *__restrict__ U,
                                                    const typename C2<T>::type *__restrict__ src,
                                                    typename C2<T>::type *__restrict__ dst, T kappa, int nmr,
                                                    int slot0)
{
    typedef typename C2<T>::type T2;
    __shared__ T2 she[12 * MAXVB / 2];
    __shared__ T2 sho[12 * MAXVB / 2];
    __shared__ T red[3][MAXVB / 64];
    __shared__ T alpha_sh[2];

    const int Vb = g.Vb, Vh = g.Vh;
    const int slot = slot0 + blockIdx.x;
    const int l = threadIdx.x;
    const bool even = l < Vh;
    const int hi = even ? l : l - Vh;
    const int nw = (Vb + 63) / 64;
    const int ww = Vb < 64 ? Vb : 64;
    int x[4];
    local_coords(g, l, x);

    // ---- residual of the block system at this site
    spinor<T> r, acc;
    if (MODE == 0) {
        hop_sum<T, HOPS_ALL>(g, U, slot, l, x, GlobalLoader<T>{dst, Vb}, acc);
        spinor<T> e, xs;
        load_site<T>(src, slot, Vb, l, e);
        load_site<T>(dst, slot, Vb, l, xs);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                r.s[sp].c[a] = e.s[sp].c[a] - xs.s[sp].c[a] + scale(kappa, acc.s[sp].c[a]);
    } else {
        load_site<T>(src, slot, Vb, l, r);
    }

    // ---- rhs_e = r_e + kappa H_eo r_o
    if (!even) lds_store<T>(sho, Vh, hi, r);
    __syncthreads();
    spinor<T> rho, del;
    if (even) {
        hop_sum<T, HOPS_IN>(g, U, slot, l, x, LdsLoader<T>{sho, Vh, Vh}, acc);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                rho.s[sp].c[a] = r.s[sp].c[a] + scale(kappa, acc.s[sp].c[a]);
                del.s[sp].c[a] = mk<T>(0, 0);
            }
        lds_store<T>(she, Vh, hi, rho);
    }

    // ---- MR steps on (1 - kappa^2 H_eo H_oe)
    const T k2 = kappa * kappa;
    for (int it = 0; it < nmr; ++it) {
        __syncthreads();
        if (!even) {  // t_o = H_oe rho
            hop_sum<T, HOPS_IN>(g, U, slot, l, x, LdsLoader<T>{she, Vh, 0}, acc);
            lds_store<T>(sho, Vh, hi, acc);
        }
        __syncthreads();
        T pr = 0, pi = 0, pp = 0;
        spinor<T> p;
        if (even) {  // p = rho - kappa^2 H_eo t_o
            hop_sum<T, HOPS_IN>(g, U, slot, l, x, LdsLoader<T>{sho, Vh, Vh}, acc);
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    p.s[sp].c[a] = rho.s[sp].c[a] - scale(k2, acc.s[sp].c[a]);
                    const cx<T> q = conjmul(p.s[sp].c[a], rho.s[sp].c[a]);
                    pr += q.re;
                    pi += q.im;
                    pp += p.s[sp].c[a].re * p.s[sp].c[a].re + p.s[sp].c[a].im * p.s[sp].c[a].im;
                }
        }
        pr = wave_sum(pr, ww);
        pi = wave_sum(pi, ww);
        pp = wave_sum(pp, ww);
        if ((l & 63) == 0) {
            red[0][l >> 6] = pr;
            red[1][l >> 6] = pi;
            red[2][l >> 6] = pp;
        }
        __syncthreads();
        if (l == 0) {
            T sr = 0, si = 0, sp2 = 0;
            for (int w = 0; w < nw; ++w) {
                sr += red[0][w];
                si += red[1][w];
                sp2 += red[2][w];
            }
            alpha_sh[0] = sp2 > 0 ? sr / sp2 : T(0);
            alpha_sh[1] = sp2 > 0 ? si / sp2 : T(0);
        }
        __syncthreads();
        const cx<T> al = mk<T>(alpha_sh[0], alpha_sh[1]);
        if (even) {
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    del.s[sp].c[a] = del.s[sp].c[a] + al * rho.s[sp].c[a];
                    rho.s[sp].c[a] = rho.s[sp].c[a] - al * p.s[sp].c[a];
                }
            lds_store<T>(she, Vh, hi, rho);
        }
    }

    // ---- d_o = r_o + kappa H_oe d_e
    __syncthreads();
    if (even) lds_store<T>(she, Vh, hi, del);
    __syncthreads();
    if (!even) {
        hop_sum<T, HOPS_IN>(g, U, slot, l, x, LdsLoader<T>{she, Vh, 0}, acc);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) del.s[sp].c[a] = r.s[sp].c[a] + scale(kappa, acc.s[sp].c[a]);
    }

    if (MODE == 0) {
        spinor<T> xs;
        load_site<T>(dst, slot, Vb, l, xs);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) xs.s[sp].c[a] = xs.s[sp].c[a] + del.s[sp].c[a];
        // every lane of the block has read x (neighbour reads of this block
        // only come from this workgroup) before any lane writes it
        __syncthreads();
        store_site<T>(dst, slot, Vb, l, xs);
    } else {
        store_site<T>(dst, slot, Vb, l, del);
    }
}

}  // namespace

template <typename T>
void launch_sap_colour(const Geo &g, const typename C2<T>::type *U, const typename C2<T>::type *eta,
                       typename C2<T>::type *x, T kappa, int nmr, int slot0, int nslots, hipStream_t s)
{
    if (nslots > 0) k_block_mr<T, 0><<<nslots, g.Vb, 0, s>>>(g, U, eta, x, kappa, nmr, slot0);
}

template <typename T>
void launch_block_mr(const Geo &g, const typename C2<T>::type *U, const typename C2<T>::type *r,
                     typename C2<T>::type *d, T kappa, int nmr, int slot0, int nslots, hipStream_t s)
{
    if (nslots > 0) k_block_mr<T, 1><<<nslots, g.Vb, 0, s>>>(g, U, r, d, kappa, nmr, slot0);
}

#define INST(T)                                                                                                  \
    template void launch_sap_colour<T>(const Geo &, const C2<T>::type *, const C2<T>::type *, C2<T>::type *, T,  \
                                       int, int, int, hipStream_t);                                              \
    template void launch_block_mr<T>(const Geo &, const C2<T>::type *, const C2<T>::type *, C2<T>::type *, T,    \
                                     int, int, int, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace wdr
