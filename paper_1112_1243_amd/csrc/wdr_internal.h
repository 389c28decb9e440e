// Internal declarations of the HIP library behind include/wdr.h.
//
// Internal layout (all device fields)
//   Sites are ordered block by block, black blocks first, then white
//   (paper Sec. 3); a block slot holds Vb = B0*B1*B2*B3 sites, its even
//   sites first, then its odd sites, each in lexicographic order of the
//   in-block coordinates.  Every block has even extents, so in-block parity
//   equals global parity.
//   spinor  [slot][12][Vb]     complex (T2), component = 3*spin + colour
//   gauge   [slot][mu][9][Vb]  complex, U_mu(x) row-major, boundary phase
//           folded into the links that wrap around the lattice
// so a wavefront of 64 consecutive sites reads 64 consecutive complex
// numbers for every component.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/wdr.h"

namespace wdr {

// ---------------------------------------------------------------- errors

void set_error(const std::string &msg);
#define WDR_HIP(call)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess) {                                                                         \
            ::wdr::set_error(std::string(#call) + ": " + hipGetErrorString(e_));                        \
            return WDR_EDEVICE;                                                                         \
        }                                                                                               \
    } while (0)

// ---------------------------------------------------------------- geometry

struct Geo {
    int L[4], B[4], NB[4], bc[4];
    int V, Vb, Vh, nblk, nblack;
    int colourable;               // L/B even in every direction
    const uint32_t *loc_coord;    // [Vb]  in-block coords of local index, 8 bits each
    const uint16_t *loc_index;    // [Vb]  local index of lexicographic in-block coords
    const int32_t *slot_nbr;      // [nblk*8] neighbour slot, entry 2*mu (+mu) / 2*mu+1 (-mu)
    const int32_t *slot_blk;      // [nblk] lexicographic block id of each slot
    // workgroup -> slot schedules for launches over the black slots, the
    // white slots and all slots (index 0, 1, 2): spatially contiguous runs
    // of blocks are dealt to the same XCD (workgroup i runs on XCD i % 8)
    const int32_t *sched[3];
    int stencil;  // wdr_stencil choice for D and D_b on 4^4 blocks
    int mr_form;  // wdr_mr_form choice for the FP32 / FP16 block MR of block solves
    int cg_form;  // wdr_cg_form choice for the steps of the FP32 / FP64 even-odd CGNE
};

// which schedule covers the slot range [slot0, slot0 + n), or -1
inline int sched_index(const Geo &g, int slot0, int n)
{
    if (slot0 == 0 && n == g.nblk) return 2;
    if (slot0 == 0 && n == g.nblack) return 0;
    if (slot0 == g.nblack && n == g.nblk - g.nblack) return 1;
    return -1;
}

// complex types
template <typename T> struct C2;
template <> struct C2<double> { typedef double2 type; };
template <> struct C2<float> { typedef float2 type; };

// FP16 storage of a complex number (two IEEE binary16 values); arithmetic on
// such data is done in FP32
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

// system of launch index j (a compacted launch maps its j-th system through list)
__device__ __forceinline__ int sys_at(const int32_t *list, int j) { return list ? list[j] : j; }
// element index in the whole batch of launch element k of an elementwise
// launch over n-element fields (a compacted launch covers the systems of list
// back to back); m receives the system
__device__ __forceinline__ long batch_index(const int32_t *list, long n, long k, int &m)
{
    const int j = (int)(k / n);
    m = sys_at(list, j);
    return k + (long)(m - j) * n;
}

// field element visited by index i of an elementwise pass: every element
// (hs = 0), or with hs = log2(Vh) the even-site half of every (slot,
// component) run of Vb = 2 Vh entries
__device__ __forceinline__ long emap(long i, int hs) { return hs ? i + ((i >> hs) << hs) : i; }
// element of the whole batch for launch element k of an elementwise launch
// that visits ne = n or n / 2 (hs > 0) elements per system (a compacted
// launch covers the systems of list back to back); m receives the system
__device__ __forceinline__ long batch_elem(const int32_t *list, long n, int hs, long k, int &m)
{
    const long ne = hs ? n >> 1 : n;
    const int j = (int)(k / ne);
    m = sys_at(list, j);
    return (long)m * n + emap(k - (long)j * ne, hs);
}

template <typename T> struct Field {  // one spinor field in the internal layout
    typename C2<T>::type *p;
};

}  // namespace wdr

// ---------------------------------------------------------------- device math

namespace wdr {
namespace dev {

template <typename T> struct cx {
    T re, im;
};

template <typename T> __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cx<T> conjmul(cx<T> a, cx<T> b)  // conj(a) * b
{
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T> __device__ __forceinline__ cx<T> scale(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.im, a.re}; }
template <typename T> __device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.im, -a.re}; }
template <typename T> __device__ __forceinline__ cx<T> neg(cx<T> a) { return {-a.re, -a.im}; }

template <typename T> __device__ __forceinline__ cx<T> ld(const typename C2<T>::type *p, long i)
{
    typename C2<T>::type v = p[i];
    return {v.x, v.y};
}
// a pointer read from a device table is generic to the compiler; kernels
// cast it so its loads are global loads rather than flat loads
template <typename P> __device__ __forceinline__ const __attribute__((address_space(1))) P *as_global(const P *p)
{
    return (const __attribute__((address_space(1))) P *)p;
}
template <typename T> __device__ __forceinline__ cx<T> ldg(const __attribute__((address_space(1))) typename C2<T>::type *p, long i)
{
    const __attribute__((address_space(1))) T *q = (const __attribute__((address_space(1))) T *)p;
    return {q[2 * i], q[2 * i + 1]};
}
// streaming store: the stencil output is not read again by the launch, so it
// is written non-temporally
template <typename T> __device__ __forceinline__ void st_nt(typename C2<T>::type *p, long i, cx<T> a)
{
    typedef T v2 __attribute__((ext_vector_type(2)));
    v2 v;
    v.x = a.re;
    v.y = a.im;
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) v2 *)p + i);
}
template <typename T> __device__ __forceinline__ void st(typename C2<T>::type *p, long i, cx<T> a)
{
    typename C2<T>::type v;
    v.x = a.re;
    v.y = a.im;
    p[i] = v;
}

// A colour 3-vector and a half spinor (2 spins x 3 colours)
template <typename T> struct vec3 {
    cx<T> c[3];
};
template <typename T> struct half {
    vec3<T> s[2];
};
template <typename T> struct spinor {
    vec3<T> s[4];
};
template <typename T> struct su3 {
    cx<T> m[3][3];
};

template <typename T> __device__ __forceinline__ vec3<T> mul(const su3<T> &u, const vec3<T> &v)
{
    vec3<T> r;
#pragma unroll
    for (int a = 0; a < 3; ++a) r.c[a] = u.m[a][0] * v.c[0] + u.m[a][1] * v.c[1] + u.m[a][2] * v.c[2];
    return r;
}
template <typename T> __device__ __forceinline__ vec3<T> mul_dag(const su3<T> &u, const vec3<T> &v)
{
    vec3<T> r;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        r.c[a] = conjmul(u.m[0][a], v.c[0]) + conjmul(u.m[1][a], v.c[1]) + conjmul(u.m[2][a], v.c[2]);
    return r;
}

// Spin projection in the chiral basis: g_mu = [[0, A_mu], [A_mu^+, 0]] with
// A_1 = -i s_1, A_2 = -i s_2, A_3 = -i s_3, A_4 = 1, so
//   (1 - g_mu) psi = (h, -A^+ h),  h = psi_up - A psi_dn
//   (1 + g_mu) psi = (h,  A^+ h),  h = psi_up + A psi_dn
// A psi_dn for psi_dn = (d0, d1):
//   mu=0: (-i d1, -i d0)  mu=1: (-d1, d0)  mu=2: (-i d0, i d1)  mu=3: (d0, d1)
// A^+ h for h = (h0, h1):
//   mu=0: (i h1, i h0)    mu=1: (h1, -h0)  mu=2: (i h0, -i h1)  mu=3: (h0, h1)
template <typename T> __device__ __forceinline__ vec3<T> vmap(const vec3<T> &v, int op)
{
    // op: 0 identity, 1 negate, 2 times i, 3 times -i
    vec3<T> r;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<T> x = v.c[a];
        r.c[a] = op == 0 ? x : op == 1 ? neg(x) : op == 2 ? mul_i(x) : mul_mi(x);
    }
    return r;
}
template <typename T> __device__ __forceinline__ vec3<T> vadd(const vec3<T> &a, const vec3<T> &b)
{
    vec3<T> r;
#pragma unroll
    for (int i = 0; i < 3; ++i) r.c[i] = a.c[i] + b.c[i];
    return r;
}

// A psi_dn: returns (first, second) spin components
template <typename T> __device__ __forceinline__ void A_dn(int mu, const vec3<T> &d0, const vec3<T> &d1, vec3<T> &o0,
                                                           vec3<T> &o1)
{
    switch (mu) {
    case 0: o0 = vmap(d1, 3); o1 = vmap(d0, 3); break;
    case 1: o0 = vmap(d1, 1); o1 = d0; break;
    case 2: o0 = vmap(d0, 3); o1 = vmap(d1, 2); break;
    default: o0 = d0; o1 = d1; break;
    }
}
// A^+ h
template <typename T> __device__ __forceinline__ void Adag_h(int mu, const vec3<T> &h0, const vec3<T> &h1, vec3<T> &o0,
                                                             vec3<T> &o1)
{
    switch (mu) {
    case 0: o0 = vmap(h1, 2); o1 = vmap(h0, 2); break;
    case 1: o0 = h1; o1 = vmap(h0, 1); break;
    case 2: o0 = vmap(h0, 2); o1 = vmap(h1, 3); break;
    default: o0 = h0; o1 = h1; break;
    }
}

// FP16 element i of a global field, times the block scale s
__device__ __forceinline__ cx<float> ldh(const __attribute__((address_space(1))) h2 *p, long i, float s)
{
    const h2 v = p[i];
    return {(float)v.x * s, (float)v.y * s};
}
// a / s rounded to FP16 (round to nearest even); inv = 1 / s is a power of two
__device__ __forceinline__ h2 to_h2(cx<float> a, float inv)
{
    h2 r;
    r.x = (_Float16)(a.re * inv);
    r.y = (_Float16)(a.im * inv);
    return r;
}
// the power of two 2^ceil(log2 mx) (1 for an all-zero block)
__device__ __forceinline__ float pow2_at_least(float mx)
{
    if (!(mx > 0.f)) return 1.f;
    int e;
    const float f = frexpf(mx, &e);  // mx = f 2^e, f in [0.5, 1)
    return ldexpf(1.f, f == 0.5f ? e - 1 : e);
}

}  // namespace dev
}  // namespace wdr
