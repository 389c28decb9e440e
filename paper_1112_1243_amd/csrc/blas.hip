// BLAS-1 kernels and deterministic FP64 reductions over batches of fields.
//
// Reductions run in two passes with a fixed grid: workgroup (c, m) sums a
// fixed, strided share of system m's elements in FP64 (wavefront shuffles,
// then LDS across the 4 wavefronts), and one workgroup per system adds the
// partial sums in a fixed order.  Results do not depend on scheduling and
// are bit-reproducible from run to run.
#include <algorithm>

#include "ops.h"

namespace wdr {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// sums v over the workgroup into thread 0; sh: 4 doubles of LDS
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

template <typename T> __device__ __forceinline__ double2 toD(typename C2<T>::type v)
{
    return make_double2((double)v.x, (double)v.y);
}

__device__ __forceinline__ bool off(const int32_t *active, int m) { return active && !active[m]; }

// partial[(m * nv + j) * 2G + 2c + {0,1}]
template <typename T>
__global__ __launch_bounds__(NT) void k_multidot_partial(const int32_t *active, long n,
                                                         const typename C2<T>::type *const *v, int nv,
                                                         const typename C2<T>::type *__restrict__ y, double *partial)
{
    __shared__ double sh[4];
    const int G = gridDim.x, m = blockIdx.y;
    if (off(active, m)) return;
    const typename C2<T>::type *ym = y + m * n;
    for (int j = 0; j < nv; ++j) {
        const typename C2<T>::type *vj = v[j] + m * n;
        double re = 0, im = 0;
        for (long i = (long)blockIdx.x * NT + threadIdx.x; i < n; i += (long)G * NT) {
            const double2 a = toD<T>(vj[i]), b = toD<T>(ym[i]);
            re += a.x * b.x + a.y * b.y;
            im += a.x * b.y - a.y * b.x;
        }
        re = block_sum(re, sh);
        im = block_sum(im, sh);
        if (threadIdx.x == 0) {
            partial[((long)m * nv + j) * 2 * G + 2 * blockIdx.x] = re;
            partial[((long)m * nv + j) * 2 * G + 2 * blockIdx.x + 1] = im;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_dot_partial(const int32_t *active, const int32_t *list, long n, int hs,
                                                    const typename C2<T>::type *__restrict__ a,
                                                    const typename C2<T>::type *__restrict__ b, int norm,
                                                    double *partial)
{
    __shared__ double sh[4];
    const int G = gridDim.x, m = sys_at(list, blockIdx.y);
    if (off(active, m)) return;
    a += m * n;
    b += m * n;
    const long ne = hs ? n >> 1 : n;
    double re = 0, im = 0;
    for (long i = (long)blockIdx.x * NT + threadIdx.x; i < ne; i += (long)G * NT) {
        const long e = emap(i, hs);
        const double2 x = toD<T>(a[e]);
        if (norm) {
            re += x.x * x.x + x.y * x.y;
        } else {
            const double2 y = toD<T>(b[e]);
            re += x.x * y.x + x.y * y.y;
            im += x.x * y.y - x.y * y.x;
        }
    }
    re = block_sum(re, sh);
    im = block_sum(im, sh);
    if (threadIdx.x == 0) {
        partial[(long)m * 2 * G + 2 * blockIdx.x] = re;
        partial[(long)m * 2 * G + 2 * blockIdx.x + 1] = im;
    }
}

// out[m * ostride + j] = sum over the G partials, fixed order; workgroup
// (system, j) for j < nv = gridDim.y
__global__ __launch_bounds__(NT) void k_final(const int32_t *active, const int32_t *list, const double *partial,
                                              int G, double2 *out, int ostride)
{
    __shared__ double sh[4];
    const int m = sys_at(list, blockIdx.x), j = blockIdx.y, nv = gridDim.y;
    if (off(active, m)) return;
    const double *p = partial + ((long)m * nv + j) * 2 * G;
    double re = 0, im = 0;
    for (int i = threadIdx.x; i < G; i += NT) {
        re += p[2 * i];
        im += p[2 * i + 1];
    }
    re = block_sum(re, sh);
    im = block_sum(im, sh);
    if (threadIdx.x == 0) out[(long)m * ostride + j] = make_double2(re, im);
}

// Fused passes of the Krylov solvers: an elementwise update followed by the
// first pass of a reduction over its result, with the element split of
// k_dot_partial, so the sums match a separate reduction over the stored
// values.  Partials: 2G per system (k_final), 3G for k_norm_dot_partial.

// One CG step on system m with s = sc[m * sstride]: alpha = s[0].x / s[1].x
// (|r|^2 / |w|^2, 0 when |w|^2 is not positive), x += alpha w, r -= alpha q
// in T, and the partial sums of |r|^2 of the new r.
template <typename T>
__global__ __launch_bounds__(NT) void k_cg_xr_partial(const int32_t *active, const int32_t *list, long n, int hs,
                                                      const double2 *sc, int sstride,
                                                      typename C2<T>::type *__restrict__ x,
                                                      const typename C2<T>::type *__restrict__ w,
                                                      typename C2<T>::type *__restrict__ r,
                                                      const typename C2<T>::type *__restrict__ q, double *partial)
{
    __shared__ double sh[4];
    const int G = gridDim.x, m = sys_at(list, blockIdx.y);
    if (off(active, m)) return;
    const double ww = sc[(long)m * sstride + 1].x;
    const T a = (T)(ww > 0 ? sc[(long)m * sstride].x / ww : 0.0);
    x += m * n;
    w += m * n;
    r += m * n;
    q += m * n;
    const long ne = hs ? n >> 1 : n;
    double re = 0;
    for (long j = (long)blockIdx.x * NT + threadIdx.x; j < ne; j += (long)G * NT) {
        const long i = emap(j, hs);
        typename C2<T>::type xi = x[i], ri = r[i];
        const typename C2<T>::type wi = w[i], qi = q[i];
        xi.x = xi.x + a * wi.x;
        xi.y = xi.y + a * wi.y;
        ri.x = ri.x - a * qi.x;
        ri.y = ri.y - a * qi.y;
        x[i] = xi;
        r[i] = ri;
        const double2 d = toD<T>(ri);
        re += d.x * d.x + d.y * d.y;
    }
    re = block_sum(re, sh);
    if (threadIdx.x == 0) {
        partial[(long)m * 2 * G + 2 * blockIdx.x] = re;
        partial[(long)m * 2 * G + 2 * blockIdx.x + 1] = 0.0;
    }
}

// partial sums of |a|^2 and <a, b> (three per workgroup)
__global__ __launch_bounds__(NT) void k_norm_dot_partial(const int32_t *active, long n, const double2 *__restrict__ a,
                                                         const double2 *__restrict__ b, double *partial)
{
    __shared__ double sh[4];
    const int G = gridDim.x, m = blockIdx.y;
    if (off(active, m)) return;
    a += m * n;
    b += m * n;
    double nn = 0, re = 0, im = 0;
    for (long i = (long)blockIdx.x * NT + threadIdx.x; i < n; i += (long)G * NT) {
        const double2 x = a[i], y = b[i];
        nn += x.x * x.x + x.y * x.y;
        re += x.x * y.x + x.y * y.y;
        im += x.x * y.y - x.y * y.x;
    }
    nn = block_sum(nn, sh);
    re = block_sum(re, sh);
    im = block_sum(im, sh);
    if (threadIdx.x == 0) {
        double *p = partial + (long)m * 3 * G + 3 * blockIdx.x;
        p[0] = nn;
        p[1] = re;
        p[2] = im;
    }
}

// out_n[m * nstride] = (|a|^2, 0), out_d[m * dstride] = <a, b> / |a|
__global__ __launch_bounds__(NT) void k_final_norm_dot(const int32_t *active, const double *partial, int G,
                                                       double2 *out_n, int nstride, double2 *out_d, int dstride)
{
    __shared__ double sh[4];
    const int m = blockIdx.x;
    if (off(active, m)) return;
    const double *p = partial + (long)m * 3 * G;
    double nn = 0, re = 0, im = 0;
    for (int i = threadIdx.x; i < G; i += NT) {
        nn += p[3 * i];
        re += p[3 * i + 1];
        im += p[3 * i + 2];
    }
    nn = block_sum(nn, sh);
    re = block_sum(re, sh);
    im = block_sum(im, sh);
    if (threadIdx.x == 0) {
        const double f = 1.0 / sqrt(nn);
        out_n[(long)m * nstride] = make_double2(nn, 0.0);
        out_d[(long)m * dstride] = make_double2(re * f, im * f);
    }
}

// a *= 1 / sqrt(nrm[m * nstride].x), then b -= c[m * cstride] a, and the
// partial sums of |b|^2 of the new b
__global__ __launch_bounds__(NT) void k_orth_partial(const int32_t *active, long n, const double2 *nrm, int nstride,
                                                     const double2 *c, int cstride, double2 *__restrict__ a,
                                                     double2 *__restrict__ b, double *partial)
{
    __shared__ double sh[4];
    const int G = gridDim.x, m = blockIdx.y;
    if (off(active, m)) return;
    const double f = 1.0 / sqrt(nrm[(long)m * nstride].x);
    const double2 cm = c[(long)m * cstride];
    const double cr = -cm.x, ci = -cm.y;
    a += m * n;
    b += m * n;
    double s = 0;
    for (long i = (long)blockIdx.x * NT + threadIdx.x; i < n; i += (long)G * NT) {
        double2 v = a[i];
        v = make_double2(f * v.x, f * v.y);
        a[i] = v;
        double2 y = b[i];
        y.x += cr * v.x - ci * v.y;
        y.y += cr * v.y + ci * v.x;
        b[i] = y;
        s += y.x * y.x + y.y * y.y;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) {
        partial[(long)m * 2 * G + 2 * blockIdx.x] = s;
        partial[(long)m * 2 * G + 2 * blockIdx.x + 1] = 0.0;
    }
}

// One classical Gram-Schmidt update followed by the first pass of the next
// reduction: y -= sum_{j < nv} c[m * cstride + j] v_j (nv <= CGS_MAXV), then
// NORM = 0: <v_j, y> for j < nv (partials as k_multidot_partial);
// NORM = 1: |y|^2 and <y, b> (partials as k_norm_dot_partial).
constexpr int CGS_MAXV = 16;
template <int NORM>
__global__ __launch_bounds__(NT) void k_cgs_partial(const int32_t *active, long n, const double2 *c, int cstride,
                                                    const double2 *const *v, int nv, double2 *__restrict__ y,
                                                    const double2 *__restrict__ b, double *partial)
{
    __shared__ double sh[4];
    const int G = gridDim.x, m = blockIdx.y;
    if (off(active, m)) return;
    const double2 *vp[CGS_MAXV];
    double2 cm[CGS_MAXV];
#pragma unroll
    for (int j = 0; j < CGS_MAXV; ++j) {
        vp[j] = j < nv ? v[j] + m * n : nullptr;
        cm[j] = j < nv ? c[(long)m * cstride + j] : make_double2(0.0, 0.0);
    }
    y += m * n;
    if (NORM) b += m * n;
    constexpr int NA = NORM ? 3 : 2 * CGS_MAXV;
    double acc[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) acc[k] = 0;
    for (long i = (long)blockIdx.x * NT + threadIdx.x; i < n; i += (long)G * NT) {
        double2 a[CGS_MAXV];
        double2 yi = y[i];
#pragma unroll
        for (int j = 0; j < CGS_MAXV; ++j)
            if (j < nv) {
                a[j] = vp[j][i];
                const double cr = -cm[j].x, ci = -cm[j].y;
                yi.x += cr * a[j].x - ci * a[j].y;
                yi.y += cr * a[j].y + ci * a[j].x;
            }
        y[i] = yi;
        if constexpr (NORM) {
            const double2 bi = b[i];
            acc[0] += yi.x * yi.x + yi.y * yi.y;
            acc[1] += yi.x * bi.x + yi.y * bi.y;
            acc[2] += yi.x * bi.y - yi.y * bi.x;
        } else {
#pragma unroll
            for (int j = 0; j < CGS_MAXV; ++j)
                if (j < nv) {
                    acc[2 * j] += a[j].x * yi.x + a[j].y * yi.y;
                    acc[2 * j + 1] += a[j].x * yi.y - a[j].y * yi.x;
                }
        }
    }
    if constexpr (NORM) {
        const double nn = block_sum(acc[0], sh), re = block_sum(acc[1], sh), im = block_sum(acc[2], sh);
        if (threadIdx.x == 0) {
            double *p = partial + (long)m * 3 * G + 3 * blockIdx.x;
            p[0] = nn;
            p[1] = re;
            p[2] = im;
        }
    } else {
#pragma unroll
        for (int j = 0; j < CGS_MAXV; ++j)
            if (j < nv) {
                const double re = block_sum(acc[2 * j], sh), im = block_sum(acc[2 * j + 1], sh);
                if (threadIdx.x == 0) {
                    partial[((long)m * nv + j) * 2 * G + 2 * blockIdx.x] = re;
                    partial[((long)m * nv + j) * 2 * G + 2 * blockIdx.x + 1] = im;
                }
            }
    }
}

// r = b - a and the partial sums of |r|^2
__global__ __launch_bounds__(NT) void k_sub_partial(const int32_t *active, const int32_t *list, long n, int hs,
                                                    const double2 *__restrict__ b, const double2 *__restrict__ a,
                                                    double2 *__restrict__ r, double *partial)
{
    __shared__ double sh[4];
    const int G = gridDim.x, m = sys_at(list, blockIdx.y);
    if (off(active, m)) return;
    a += m * n;
    b += m * n;
    r += m * n;
    const long ne = hs ? n >> 1 : n;
    double s = 0;
    for (long j = (long)blockIdx.x * NT + threadIdx.x; j < ne; j += (long)G * NT) {
        const long i = emap(j, hs);
        const double2 u = b[i], v = a[i];
        const double2 d = make_double2(u.x - v.x, u.y - v.y);
        r[i] = d;
        s += d.x * d.x + d.y * d.y;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) {
        partial[(long)m * 2 * G + 2 * blockIdx.x] = s;
        partial[(long)m * 2 * G + 2 * blockIdx.x + 1] = 0.0;
    }
}

// workgroups per system of a reduction over msys systems of n elements: 8
// elements per thread, or down to 2 while the launch has fewer than about
// 2048 workgroups (small fields of few systems still spread over the CUs);
// at most RED_BLOCKS
int red_grid(long n, int msys)
{
    const long g8 = (n + NT * 8 - 1) / (NT * 8), g2 = (n + NT * 2 - 1) / (NT * 2);
    const long fill = (2048 + std::max(msys, 1) - 1) / std::max(msys, 1);
    long g = std::max(g8, std::min(g2, fill));
    if (g < 1) g = 1;
    if (g > RED_BLOCKS) g = RED_BLOCKS;
    return (int)g;
}

template <typename TO, typename TI>
__global__ __launch_bounds__(NT) void k_convert(const typename C2<TI>::type *__restrict__ a,
                                                typename C2<TO>::type *__restrict__ out, long total)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= total) return;
    const typename C2<TI>::type v = a[i];
    typename C2<TO>::type w;
    w.x = (TO)v.x;
    w.y = (TO)v.y;
    out[i] = w;
}

// out = (TO) a and z = 0 (the start of a Schwarz preconditioner: source
// converted, solution cleared)
template <typename TO, typename TI>
__global__ __launch_bounds__(NT) void k_convert_zero(const typename C2<TI>::type *__restrict__ a,
                                                     typename C2<TO>::type *__restrict__ out,
                                                     typename C2<TO>::type *__restrict__ z, long total)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= total) return;
    const typename C2<TI>::type v = a[i];
    typename C2<TO>::type w;
    w.x = (TO)v.x;
    w.y = (TO)v.y;
    out[i] = w;
    w.x = 0;
    w.y = 0;
    z[i] = w;
}

template <typename T> __global__ __launch_bounds__(NT) void k_zero(typename C2<T>::type *a, long total)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= total) return;
    typename C2<T>::type z;
    z.x = 0;
    z.y = 0;
    a[i] = z;
}

// zero outside [lo, hi) of every field (element index within the field)
__global__ __launch_bounds__(NT) void k_keep_range(double2 *f, long n, long total, long lo, long hi)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= total) return;
    const long e = i % n;
    if (e < lo || e >= hi) f[i] = make_double2(0.0, 0.0);
}

__global__ __launch_bounds__(NT) void k_multi_axpy(const int32_t *active, long n, long total, const double2 *c,
                                                   int cstride, double f, const double2 *const *v, int nv,
                                                   const int32_t *cnt, double2 *__restrict__ y, int acc)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= total) return;
    const int m = (int)(i / n);
    if (off(active, m)) return;
    const int k = cnt ? cnt[m] : nv;
    double2 b = acc ? y[i] : make_double2(0.0, 0.0);
    for (int j = 0; j < k; ++j) {
        const double2 cj = c[(long)m * cstride + j];
        const double cr = f * cj.x, ci = f * cj.y;
        const double2 a = v[j][i];
        b.x += cr * a.x - ci * a.y;
        b.y += cr * a.y + ci * a.x;
    }
    y[i] = b;
}

__global__ __launch_bounds__(NT) void k_sub(const int32_t *active, const int32_t *list, long n, long total,
                                            const double2 *b, const double2 *a, double2 *r)
{
    const long k = (long)blockIdx.x * NT + threadIdx.x;
    if (k >= total) return;
    int m;
    const long i = batch_index(list, n, k, m);
    if (off(active, m)) return;
    const double2 u = b[i], v = a[i];
    r[i] = make_double2(u.x - v.x, u.y - v.y);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_add_to64(const int32_t *active, const int32_t *list, long n, int hs,
                                                 long total, const typename C2<T>::type *x, double2 *y)
{
    const long k = (long)blockIdx.x * NT + threadIdx.x;
    if (k >= total) return;
    int m;
    const long i = batch_elem(list, n, hs, k, m);
    if (off(active, m)) return;
    const typename C2<T>::type u = x[i];
    const double2 v = y[i];
    y[i] = make_double2(v.x + (double)u.x, v.y + (double)u.y);
}


// per-slot squared norm, workgroup (slot, m)
__global__ __launch_bounds__(NT) void k_slot_norm2(Geo g, const int32_t *active, long n, const double2 *a,
                                                   double *out, int slot0)
{
    __shared__ double sh[4];
    const int slot = slot0 + blockIdx.x, m = blockIdx.y;
    if (off(active, m)) return;
    const long base = m * n + (long)slot * 12 * g.Vb;
    const long cnt = 12L * g.Vb;
    double s = 0;
    for (long i = threadIdx.x; i < cnt; i += NT) {
        const double2 v = a[base + i];
        s += v.x * v.x + v.y * v.y;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[(long)m * g.nblk + slot] = s;
}

// Block-solve residual, workgroup (slot0 + blockIdx.x, m) of RESID_NT threads:
// r = b - t on the slot (t NULL: r already holds the residual) and
// out[m * nblk + slot] = |r|^2 over the slot.  Other slots are not touched
// (the caller keeps them zero).
constexpr int RESID_NT = 1024;
__global__ __launch_bounds__(RESID_NT) void k_block_resid_norm(Geo g, const int32_t *active, long n,
                                                               const double2 *b, const double2 *t, double2 *r,
                                                               double *out, int slot0)
{
    __shared__ double sh[RESID_NT / 64];
    const int slot = slot0 + blockIdx.x, m = blockIdx.y;
    if (off(active, m)) return;
    const long cnt = 12L * g.Vb, base = m * n + (long)slot * cnt;
    double s = 0;
    for (long i = threadIdx.x; i < cnt; i += RESID_NT) {
        double2 v;
        if (t) {
            const double2 u = b[base + i], w = t[base + i];
            v = make_double2(u.x - w.x, u.y - w.y);
            r[base + i] = v;
        } else {
            v = r[base + i];
        }
        s += v.x * v.x + v.y * v.y;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0;
#pragma unroll
        for (int w = 0; w < RESID_NT / 64; ++w) tot += sh[w];
        out[(long)m * g.nblk + slot] = tot;
    }
}

inline unsigned nblk(long n) { return (unsigned)((n + NT - 1) / NT); }

}  // namespace

template <typename T>
void launch_multidot(const Sys &sy, const T2<T> *const *v, int nv, const T2<T> *y, double *red, double2 *out,
                     int ostride, hipStream_t s)
{
    if (nv <= 0) return;
    const int G = red_grid(sy.n, sy.M);
    k_multidot_partial<T><<<dim3(G, sy.M), NT, 0, s>>>(sy.active, sy.n, v, nv, y, red);
    k_final<<<dim3(sy.M, nv), NT, 0, s>>>(sy.active, nullptr, red, G, out, ostride);
}

template <typename T>
void launch_dot(const Sys &sy, const T2<T> *a, const T2<T> *b, double *red, double2 *out, int ostride, hipStream_t s)
{
    const int G = red_grid(sy.ne(), sy.launch_m());
    k_dot_partial<T><<<dim3(G, sy.launch_m()), NT, 0, s>>>(sy.active, sy.list, sy.n, sy.hs, a, b, 0, red);
    k_final<<<sy.launch_m(), NT, 0, s>>>(sy.active, sy.list, red, G, out, ostride);
}

template <typename T>
void launch_norm2(const Sys &sy, const T2<T> *a, double *red, double2 *out, int ostride, hipStream_t s)
{
    const int G = red_grid(sy.ne(), sy.launch_m());
    k_dot_partial<T><<<dim3(G, sy.launch_m()), NT, 0, s>>>(sy.active, sy.list, sy.n, sy.hs, a, a, 1, red);
    k_final<<<sy.launch_m(), NT, 0, s>>>(sy.active, sy.list, red, G, out, ostride);
}

template <typename T>
void launch_cg_xr_norm(const Sys &sy, const double2 *sc, int sstride, T2<T> *x, const T2<T> *w, T2<T> *r,
                       const T2<T> *q, double *red, double2 *out, int ostride, hipStream_t s)
{
    const int G = red_grid(sy.ne(), sy.launch_m());
    k_cg_xr_partial<T><<<dim3(G, sy.launch_m()), NT, 0, s>>>(sy.active, sy.list, sy.n, sy.hs, sc, sstride, x, w, r, q,
                                                              red);
    k_final<<<sy.launch_m(), NT, 0, s>>>(sy.active, sy.list, red, G, out, ostride);
}

void launch_final(const Sys &sy, const double *partial, int G, double2 *out, int ostride, hipStream_t s)
{
    k_final<<<sy.launch_m(), NT, 0, s>>>(sy.active, sy.list, partial, G, out, ostride);
}

void launch_norm_dot(const Sys &sy, const double2 *a, const double2 *b, double *red, double2 *out_n, int nstride,
                     double2 *out_d, int dstride, hipStream_t s)
{
    const int G = red_grid(sy.n, sy.M);
    k_norm_dot_partial<<<dim3(G, sy.M), NT, 0, s>>>(sy.active, sy.n, a, b, red);
    k_final_norm_dot<<<sy.M, NT, 0, s>>>(sy.active, red, G, out_n, nstride, out_d, dstride);
}

void launch_orth_norm(const Sys &sy, const double2 *nrm, int nstride, const double2 *c, int cstride, double2 *a,
                      double2 *b, double *red, double2 *out, int ostride, hipStream_t s)
{
    const int G = red_grid(sy.n, sy.M);
    k_orth_partial<<<dim3(G, sy.M), NT, 0, s>>>(sy.active, sy.n, nrm, nstride, c, cstride, a, b, red);
    k_final<<<sy.M, NT, 0, s>>>(sy.active, nullptr, red, G, out, ostride);
}

void launch_cgs_multidot(const Sys &sy, const double2 *c, int cstride, const double2 *const *v, int nv, double2 *y,
                         double *red, double2 *out, int ostride, hipStream_t s)
{
    if (nv <= 0 || nv > CGS_MAXV) return;
    const int G = red_grid(sy.n, sy.M);
    k_cgs_partial<0><<<dim3(G, sy.M), NT, 0, s>>>(sy.active, sy.n, c, cstride, v, nv, y, nullptr, red);
    k_final<<<dim3(sy.M, nv), NT, 0, s>>>(sy.active, nullptr, red, G, out, ostride);
}

void launch_cgs_norm_dot(const Sys &sy, const double2 *c, int cstride, const double2 *const *v, int nv, double2 *y,
                         const double2 *b, double *red, double2 *out_n, int nstride, double2 *out_d, int dstride,
                         hipStream_t s)
{
    if (nv <= 0 || nv > CGS_MAXV) return;
    const int G = red_grid(sy.n, sy.M);
    k_cgs_partial<1><<<dim3(G, sy.M), NT, 0, s>>>(sy.active, sy.n, c, cstride, v, nv, y, b, red);
    k_final_norm_dot<<<sy.M, NT, 0, s>>>(sy.active, red, G, out_n, nstride, out_d, dstride);
}

void launch_sub_norm(const Sys &sy, const double2 *b, const double2 *a, double2 *r, double *red, double2 *out,
                     int ostride, hipStream_t s)
{
    const int G = red_grid(sy.ne(), sy.launch_m());
    k_sub_partial<<<dim3(G, sy.launch_m()), NT, 0, s>>>(sy.active, sy.list, sy.n, sy.hs, b, a, r, red);
    k_final<<<sy.launch_m(), NT, 0, s>>>(sy.active, sy.list, red, G, out, ostride);
}

void launch_convert_zero_f32(const Sys &sy, const double2 *a, float2 *out, float2 *z, hipStream_t s)
{
    const long total = sy.n * sy.M;
    if (total > 0) k_convert_zero<float, double><<<nblk(total), NT, 0, s>>>(a, out, z, total);
}
template <typename TO, typename TI> void launch_convert(const Sys &sy, const T2<TI> *a, T2<TO> *out, hipStream_t s)
{
    const long total = sy.n * sy.M;
    if (total > 0) k_convert<TO, TI><<<nblk(total), NT, 0, s>>>(a, out, total);
}
template <typename T> void launch_zero(T2<T> *a, long n, hipStream_t s)
{
    if (n > 0) k_zero<T><<<nblk(n), NT, 0, s>>>(a, n);
}
void launch_keep_slots(const Geo &g, const Sys &sy, double2 *f, int slot0, int nslots, hipStream_t s)
{
    const long per = 12L * g.Vb, total = sy.n * sy.M;
    if (slot0 == 0 && nslots == g.nblk) return;
    k_keep_range<<<nblk(total), NT, 0, s>>>(f, sy.n, total, per * slot0, per * (slot0 + nslots));
}
void launch_block_resid_norm(const Geo &g, const Sys &sy, const double2 *b, const double2 *t, double2 *r,
                             double *out, int slot0, int nslots, hipStream_t s)
{
    if (nslots > 0) k_block_resid_norm<<<dim3(nslots, sy.M), RESID_NT, 0, s>>>(g, sy.active, sy.n, b, t, r, out, slot0);
}
void launch_multi_axpy(const Sys &sy, const double2 *c, int cstride, double f, const double2 *const *v, int nv,
                       const int32_t *cnt, double2 *y, int acc, hipStream_t s)
{
    const long total = sy.n * sy.M;
    k_multi_axpy<<<nblk(total), NT, 0, s>>>(sy.active, sy.n, total, c, cstride, f, v, nv, cnt, y, acc);
}
void launch_sub(const Sys &sy, const double2 *b, const double2 *a, double2 *r, hipStream_t s)
{
    const long total = sy.n * sy.launch_m();
    k_sub<<<nblk(total), NT, 0, s>>>(sy.active, sy.list, sy.n, total, b, a, r);
}
template <typename T> void launch_add_to64(const Sys &sy, const T2<T> *x, double2 *y, hipStream_t s)
{
    const long total = sy.ne() * sy.launch_m();
    k_add_to64<T><<<nblk(total), NT, 0, s>>>(sy.active, sy.list, sy.n, sy.hs, total, x, y);
}
void launch_slot_norm2(const Geo &g, const Sys &sy, const double2 *a, double *out, int slot0, int nslots,
                       hipStream_t s)
{
    if (nslots > 0) k_slot_norm2<<<dim3(nslots, sy.M), NT, 0, s>>>(g, sy.active, sy.n, a, out, slot0);
}

#define INST(T)                                                                                                  \
    template void launch_multidot<T>(const Sys &, const T2<T> *const *, int, const T2<T> *, double *, double2 *, \
                                     int, hipStream_t);                                                          \
    template void launch_dot<T>(const Sys &, const T2<T> *, const T2<T> *, double *, double2 *, int, hipStream_t); \
    template void launch_norm2<T>(const Sys &, const T2<T> *, double *, double2 *, int, hipStream_t);            \
    template void launch_zero<T>(T2<T> *, long, hipStream_t);                                                     \
    template void launch_add_to64<T>(const Sys &, const T2<T> *, double2 *, hipStream_t);                     \
    template void launch_cg_xr_norm<T>(const Sys &, const double2 *, int, T2<T> *, const T2<T> *, T2<T> *,       \
                                       const T2<T> *, double *, double2 *, int, hipStream_t);
INST(double)
INST(float)
#undef INST
template void launch_convert<double, float>(const Sys &, const float2 *, double2 *, hipStream_t);
template void launch_convert<float, double>(const Sys &, const double2 *, float2 *, hipStream_t);
template void launch_convert<double, double>(const Sys &, const double2 *, double2 *, hipStream_t);
template void launch_convert<float, float>(const Sys &, const float2 *, float2 *, hipStream_t);

}  // namespace wdr
