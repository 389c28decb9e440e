// Wilson-Dirac stencil for gfx950 (paper Sec. 5: plain Wilson-Dirac
// operator; Sec. 3: Dirichlet block operators and block-interaction hops).
//
// One lane per site.  A workgroup covers 256 consecutive sites of one block
// slot (grid.y = slot), so a wavefront reads each spinor / link component of
// 64 consecutive sites as one contiguous 512 B (FP32) or 1 KiB (FP64) run.
// Hops are spin-projected: only the 2-spin half spinor is multiplied by the
// link, and the lower two spins are reconstructed from it.
#include "stencil.h"

namespace wdr {
namespace {

using namespace dev;

// loader that applies gamma_5 (flip the sign of spins 2, 3) when dag is set
template <typename T> struct G5Loader {
    const typename C2<T>::type *f;
    int Vb, dag;
    __device__ __forceinline__ void operator()(int ns, int nl, spinor<T> &p) const
    {
        GlobalLoader<T>{f, Vb}(ns, nl, p);
        if (dag) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                p.s[2].c[a] = neg(p.s[2].c[a]);
                p.s[3].c[a] = neg(p.s[3].c[a]);
            }
        }
    }
};

template <typename T, int HOPS>
__global__ __launch_bounds__(256) void k_dslash(Geo g, int par, int dag, const typename C2<T>::type *__restrict__ U,
                                                const typename C2<T>::type *__restrict__ in,
                                                const typename C2<T>::type *__restrict__ diag,
                                                typename C2<T>::type *__restrict__ out, T kappa, int slot0)
{
    const int Vb = g.Vb;
    const int nloc = par < 0 ? Vb : g.Vh;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nloc) return;
    const int l = (par > 0 ? g.Vh : 0) + i;
    const int slot = slot0 + blockIdx.y;
    int x[4];
    local_coords(g, l, x);
    spinor<T> acc;
    hop_sum<T, HOPS>(g, U, slot, l, x, G5Loader<T>{in, Vb, dag}, acc);

    const long base = (long)slot * 12 * Vb + l;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<T> v = scale(-kappa, acc.s[sp].c[a]);
            if (dag && sp >= 2) v = neg(v);
            if (diag) v = v + ld<T>(diag, base + (long)(3 * sp + a) * Vb);
            st<T>(out, base + (long)(3 * sp + a) * Vb, v);
        }
}

// ---------------------------------------------------------------- packing

__device__ __forceinline__ long canon_index(const Geo &g, int slot, int l, int x[4])
{
    int b = g.slot_blk[slot];
    const uint32_t c = g.loc_coord[l];
    int loc[4] = {(int)(c & 255u), (int)((c >> 8) & 255u), (int)((c >> 16) & 255u), (int)(c >> 24)};
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (b % g.NB[mu]) * g.B[mu] + loc[mu];
        b /= g.NB[mu];
    }
    return x[0] + (long)g.L[0] * (x[1] + (long)g.L[1] * (x[2] + (long)g.L[2] * x[3]));
}

template <typename T>
__global__ __launch_bounds__(256) void k_pack_spinor(Geo g, const double2 *__restrict__ canon,
                                                     typename C2<T>::type *__restrict__ out)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const int slot = blockIdx.y;
    int x[4];
    const long s = canon_index(g, slot, l, x);
    const long base = (long)slot * 12 * g.Vb + l;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double2 v = canon[s * 12 + c];
        typename C2<T>::type w;
        w.x = (T)v.x;
        w.y = (T)v.y;
        out[base + (long)c * g.Vb] = w;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_unpack_spinor(Geo g, const typename C2<T>::type *__restrict__ in,
                                                       double2 *__restrict__ canon)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const int slot = blockIdx.y;
    int x[4];
    const long s = canon_index(g, slot, l, x);
    const long base = (long)slot * 12 * g.Vb + l;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        typename C2<T>::type v = in[base + (long)c * g.Vb];
        canon[s * 12 + c] = make_double2((double)v.x, (double)v.y);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_pack_gauge(Geo g, int4 bc, const double2 *__restrict__ canon,
                                                    typename C2<T>::type *__restrict__ out)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const int slot = blockIdx.y;
    int x[4];
    const long s = canon_index(g, slot, l, x);
    const int bcv[4] = {bc.x, bc.y, bc.z, bc.w};
    for (int mu = 0; mu < 4; ++mu) {
        const double f = (x[mu] == g.L[mu] - 1) ? (double)bcv[mu] : 1.0;
        const long base = ((long)slot * 4 + mu) * 9 * g.Vb + l;
        for (int e = 0; e < 9; ++e) {
            double2 v = canon[(s * 4 + mu) * 9 + e];
            typename C2<T>::type w;
            w.x = (T)(f * v.x);
            w.y = (T)(f * v.y);
            out[base + (long)e * g.Vb] = w;
        }
    }
}

__global__ __launch_bounds__(256) void k_unpack_gauge(Geo g, int4 bc, const double2 *__restrict__ in,
                                                      double2 *__restrict__ canon)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const int slot = blockIdx.y;
    int x[4];
    const long s = canon_index(g, slot, l, x);
    const int bcv[4] = {bc.x, bc.y, bc.z, bc.w};
    for (int mu = 0; mu < 4; ++mu) {
        const double f = (x[mu] == g.L[mu] - 1) ? (double)bcv[mu] : 1.0;
        const long base = ((long)slot * 4 + mu) * 9 * g.Vb + l;
        for (int e = 0; e < 9; ++e) {
            double2 v = in[base + (long)e * g.Vb];
            canon[(s * 4 + mu) * 9 + e] = make_double2(f * v.x, f * v.y);
        }
    }
}

__global__ __launch_bounds__(256) void k_convert_gauge_f32(long n, const double2 *__restrict__ in, float2 *__restrict__ out)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double2 v = in[i];
    out[i] = make_float2((float)v.x, (float)v.y);
}

template <typename T>
__global__ __launch_bounds__(256) void k_g5(Geo g, const typename C2<T>::type *__restrict__ in,
                                            typename C2<T>::type *__restrict__ out, int slot0)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const long base = (long)(slot0 + blockIdx.y) * 12 * g.Vb + l;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        typename C2<T>::type v = in[base + (long)c * g.Vb];
        if (c >= 6) {
            v.x = -v.x;
            v.y = -v.y;
        }
        out[base + (long)c * g.Vb] = v;
    }
}

}  // namespace

template <typename T>
void launch_dslash(const Geo &g, int hops, int par, int dag, const typename C2<T>::type *U,
                   const typename C2<T>::type *in, const typename C2<T>::type *diag, typename C2<T>::type *out,
                   T kappa, int slot0, int nslots, hipStream_t s)
{
    if (nslots <= 0) return;
    const int nloc = par < 0 ? g.Vb : g.Vh;
    dim3 grid((nloc + 255) / 256, nslots);
    if (hops == HOPS_ALL)
        k_dslash<T, HOPS_ALL><<<grid, 256, 0, s>>>(g, par, dag, U, in, diag, out, kappa, slot0);
    else if (hops == HOPS_IN)
        k_dslash<T, HOPS_IN><<<grid, 256, 0, s>>>(g, par, dag, U, in, diag, out, kappa, slot0);
    else
        k_dslash<T, HOPS_CROSS><<<grid, 256, 0, s>>>(g, par, dag, U, in, diag, out, kappa, slot0);
}

template <typename T> void launch_pack_spinor(const Geo &g, const double2 *canon, typename C2<T>::type *out, hipStream_t s)
{
    k_pack_spinor<T><<<dim3((g.Vb + 255) / 256, g.nblk), 256, 0, s>>>(g, canon, out);
}
template <typename T> void launch_unpack_spinor(const Geo &g, const typename C2<T>::type *in, double2 *canon, hipStream_t s)
{
    k_unpack_spinor<T><<<dim3((g.Vb + 255) / 256, g.nblk), 256, 0, s>>>(g, in, canon);
}
template <typename T>
void launch_pack_gauge(const Geo &g, const int bc[4], const double2 *canon, typename C2<T>::type *out, hipStream_t s)
{
    k_pack_gauge<T><<<dim3((g.Vb + 255) / 256, g.nblk), 256, 0, s>>>(g, make_int4(bc[0], bc[1], bc[2], bc[3]), canon,
                                                                     out);
}
void launch_unpack_gauge(const Geo &g, const int bc[4], const double2 *in, double2 *canon, hipStream_t s)
{
    k_unpack_gauge<<<dim3((g.Vb + 255) / 256, g.nblk), 256, 0, s>>>(g, make_int4(bc[0], bc[1], bc[2], bc[3]), in,
                                                                    canon);
}
void launch_convert_gauge_f32(const Geo &g, const double2 *in, float2 *out, hipStream_t s)
{
    long n = (long)g.V * 36;
    k_convert_gauge_f32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, in, out);
}
template <typename T>
void launch_g5(const Geo &g, const typename C2<T>::type *in, typename C2<T>::type *out, int slot0, int nslots,
               hipStream_t s)
{
    if (nslots <= 0) return;
    k_g5<T><<<dim3((g.Vb + 255) / 256, nslots), 256, 0, s>>>(g, in, out, slot0);
}

#define INST(T)                                                                                                  \
    template void launch_dslash<T>(const Geo &, int, int, int, const C2<T>::type *, const C2<T>::type *,         \
                                   const C2<T>::type *, C2<T>::type *, T, int, int, hipStream_t);                \
    template void launch_pack_spinor<T>(const Geo &, const double2 *, C2<T>::type *, hipStream_t);               \
    template void launch_unpack_spinor<T>(const Geo &, const C2<T>::type *, double2 *, hipStream_t);             \
    template void launch_pack_gauge<T>(const Geo &, const int *, const double2 *, C2<T>::type *, hipStream_t);   \
    template void launch_g5<T>(const Geo &, const C2<T>::type *, C2<T>::type *, int, int, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace wdr
