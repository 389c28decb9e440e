// BLAS-1 kernels and deterministic FP64 reductions.
//
// Reductions run in two passes with a fixed grid: every workgroup sums a
// fixed, strided share of the elements in FP64 (wavefront shuffles, then
// LDS across the 4 wavefronts), and one workgroup adds the partial sums in
// a fixed order.  The result therefore does not depend on scheduling and is
// bit-reproducible from run to run.
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

// sums v over the workgroup into lane 0 of wave 0; sh: 4 doubles of LDS
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

// partial[j * 2 * G + 2 * blk + {0,1}] = re/im of the workgroup's share of <v_j, y>
template <typename T>
__global__ __launch_bounds__(NT) void k_multidot_partial(const typename C2<T>::type *const *v, int m,
                                                         const typename C2<T>::type *__restrict__ y, long n,
                                                         double *partial)
{
    __shared__ double sh[4];
    const int G = gridDim.x;
    for (int j = 0; j < m; ++j) {
        const typename C2<T>::type *vj = v[j];
        double re = 0, im = 0;
        for (long i = (long)blockIdx.x * NT + threadIdx.x; i < n; i += (long)G * NT) {
            double2 a = toD<T>(vj[i]), b = toD<T>(y[i]);
            re += a.x * b.x + a.y * b.y;
            im += a.x * b.y - a.y * b.x;
        }
        re = block_sum(re, sh);
        im = block_sum(im, sh);
        if (threadIdx.x == 0) {
            partial[j * 2 * G + 2 * blockIdx.x] = re;
            partial[j * 2 * G + 2 * blockIdx.x + 1] = im;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_dot_partial(const typename C2<T>::type *__restrict__ a,
                                                    const typename C2<T>::type *__restrict__ b, long n, int norm,
                                                    double *partial)
{
    __shared__ double sh[4];
    const int G = gridDim.x;
    double re = 0, im = 0;
    for (long i = (long)blockIdx.x * NT + threadIdx.x; i < n; i += (long)G * NT) {
        double2 x = toD<T>(a[i]);
        if (norm) {
            re += x.x * x.x + x.y * x.y;
        } else {
            double2 y = toD<T>(b[i]);
            re += x.x * y.x + x.y * y.y;
            im += x.x * y.y - x.y * y.x;
        }
    }
    re = block_sum(re, sh);
    im = block_sum(im, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = re;
        partial[2 * blockIdx.x + 1] = im;
    }
}

// out[j] = sum over G partials, fixed order (pairwise tree over lanes)
__global__ __launch_bounds__(NT) void k_final(const double *partial, int G, int m, double2 *out)
{
    __shared__ double sh[4];
    for (int j = 0; j < m; ++j) {
        double re = 0, im = 0;
        for (int i = threadIdx.x; i < G; i += NT) {
            re += partial[j * 2 * G + 2 * i];
            im += partial[j * 2 * G + 2 * i + 1];
        }
        re = block_sum(re, sh);
        im = block_sum(im, sh);
        if (threadIdx.x == 0) out[j] = make_double2(re, im);
    }
}

int red_grid(long n)
{
    long g = (n + NT * 4 - 1) / (NT * 4);
    if (g < 1) g = 1;
    if (g > RED_BLOCKS) g = RED_BLOCKS;
    return (int)g;
}

template <typename TO, typename TI>
__global__ __launch_bounds__(NT) void k_convert(const typename C2<TI>::type *__restrict__ a,
                                                typename C2<TO>::type *__restrict__ out, long n)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    typename C2<TI>::type v = a[i];
    typename C2<TO>::type w;
    w.x = (TO)v.x;
    w.y = (TO)v.y;
    out[i] = w;
}

template <typename T> __global__ __launch_bounds__(NT) void k_zero(typename C2<T>::type *a, long n)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    typename C2<T>::type z;
    z.x = 0;
    z.y = 0;
    a[i] = z;
}

__global__ __launch_bounds__(NT) void k_axpy_dev(const double2 *c, double f, const double2 *__restrict__ x,
                                                 double2 *__restrict__ y, long n)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    const double cr = f * c->x, ci = f * c->y;
    double2 a = x[i], b = y[i];
    b.x += cr * a.x - ci * a.y;
    b.y += cr * a.y + ci * a.x;
    y[i] = b;
}

__global__ __launch_bounds__(NT) void k_multi_axpy(const double2 *c, double f, const double2 *const *v, int m,
                                                   double2 *__restrict__ y, long n, int acc)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    double2 b = acc ? y[i] : make_double2(0.0, 0.0);
    for (int j = 0; j < m; ++j) {
        const double cr = f * c[j].x, ci = f * c[j].y;
        double2 a = v[j][i];
        b.x += cr * a.x - ci * a.y;
        b.y += cr * a.y + ci * a.x;
    }
    y[i] = b;
}

__global__ __launch_bounds__(NT) void k_scale_invsqrt(const double2 *nrm, double2 *y, long n)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    const double f = 1.0 / sqrt(nrm->x);
    double2 v = y[i];
    y[i] = make_double2(f * v.x, f * v.y);
}

__global__ __launch_bounds__(NT) void k_sub(const double2 *b, const double2 *a, double2 *r, long n)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    double2 u = b[i], v = a[i];
    r[i] = make_double2(u.x - v.x, u.y - v.y);
}

__global__ __launch_bounds__(NT) void k_axpby(double a, const double2 *x, double b, double2 *y, long n)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    double2 u = x[i], v = y[i];
    y[i] = make_double2(a * u.x + b * v.x, a * u.y + b * v.y);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_add_to64(const typename C2<T>::type *x, double2 *y, long n)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    typename C2<T>::type u = x[i];
    double2 v = y[i];
    y[i] = make_double2(v.x + (double)u.x, v.y + (double)u.y);
}

// per-slot squared norm, one workgroup per slot
__global__ __launch_bounds__(NT) void k_slot_norm2(Geo g, const double2 *a, double *out, int slot0)
{
    __shared__ double sh[4];
    const int slot = slot0 + blockIdx.x;
    const long base = (long)slot * 12 * g.Vb;
    const long n = 12L * g.Vb;
    double s = 0;
    for (long i = threadIdx.x; i < n; i += NT) {
        double2 v = a[base + i];
        s += v.x * v.x + v.y * v.y;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

inline unsigned nblk(long n) { return (unsigned)((n + NT - 1) / NT); }

}  // namespace

template <typename T>
void launch_multidot(const typename C2<T>::type *const *v_dev, int m, const typename C2<T>::type *y, long n,
                     double *red, double2 *out, hipStream_t s)
{
    const int G = red_grid(n);
    k_multidot_partial<T><<<G, NT, 0, s>>>(v_dev, m, y, n, red);
    k_final<<<1, NT, 0, s>>>(red, G, m, out);
}

template <typename T>
void launch_dot(const typename C2<T>::type *a, const typename C2<T>::type *b, long n, double *red, double2 *out,
                hipStream_t s)
{
    const int G = red_grid(n);
    k_dot_partial<T><<<G, NT, 0, s>>>(a, b, n, 0, red);
    k_final<<<1, NT, 0, s>>>(red, G, 1, out);
}

template <typename T> void launch_norm2(const typename C2<T>::type *a, long n, double *red, double2 *out, hipStream_t s)
{
    const int G = red_grid(n);
    k_dot_partial<T><<<G, NT, 0, s>>>(a, a, n, 1, red);
    k_final<<<1, NT, 0, s>>>(red, G, 1, out);
}

template <typename TO, typename TI>
void launch_convert(const typename C2<TI>::type *a, typename C2<TO>::type *out, long n, hipStream_t s)
{
    if (n > 0) k_convert<TO, TI><<<nblk(n), NT, 0, s>>>(a, out, n);
}
template <typename T> void launch_zero(typename C2<T>::type *a, long n, hipStream_t s)
{
    if (n > 0) k_zero<T><<<nblk(n), NT, 0, s>>>(a, n);
}
void launch_axpy_dev(const double2 *c, double f, const double2 *x, double2 *y, long n, hipStream_t s)
{
    k_axpy_dev<<<nblk(n), NT, 0, s>>>(c, f, x, y, n);
}
void launch_multi_axpy(const double2 *c, double f, const double2 *const *v_dev, int m, double2 *y, long n, int acc,
                       hipStream_t s)
{
    k_multi_axpy<<<nblk(n), NT, 0, s>>>(c, f, v_dev, m, y, n, acc);
}
void launch_scale_invsqrt(const double2 *nrm, double2 *y, long n, hipStream_t s)
{
    k_scale_invsqrt<<<nblk(n), NT, 0, s>>>(nrm, y, n);
}
void launch_sub(const double2 *b, const double2 *a, double2 *r, long n, hipStream_t s)
{
    k_sub<<<nblk(n), NT, 0, s>>>(b, a, r, n);
}
void launch_axpby(double a, const double2 *x, double b, double2 *y, long n, hipStream_t s)
{
    k_axpby<<<nblk(n), NT, 0, s>>>(a, x, b, y, n);
}
template <typename T> void launch_add_to64(const typename C2<T>::type *x, double2 *y, long n, hipStream_t s)
{
    k_add_to64<T><<<nblk(n), NT, 0, s>>>(x, y, n);
}
void launch_slot_norm2(const Geo &g, const double2 *a, double *out, int slot0, int nslots, hipStream_t s)
{
    if (nslots > 0) k_slot_norm2<<<nslots, NT, 0, s>>>(g, a, out, slot0);
}

#define INST(T)                                                                                                  \
    template void launch_multidot<T>(const C2<T>::type *const *, int, const C2<T>::type *, long, double *,       \
                                     double2 *, hipStream_t);                                                    \
    template void launch_dot<T>(const C2<T>::type *, const C2<T>::type *, long, double *, double2 *, hipStream_t); \
    template void launch_norm2<T>(const C2<T>::type *, long, double *, double2 *, hipStream_t);                  \
    template void launch_zero<T>(C2<T>::type *, long, hipStream_t);                                              \
    template void launch_add_to64<T>(const C2<T>::type *, double2 *, long, hipStream_t);
INST(double)
INST(float)
#undef INST
template void launch_convert<double, float>(const float2 *, double2 *, long, hipStream_t);
template void launch_convert<float, double>(const double2 *, float2 *, long, hipStream_t);
template void launch_convert<double, double>(const double2 *, double2 *, long, hipStream_t);

}  // namespace wdr
