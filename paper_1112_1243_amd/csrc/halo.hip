// Halo of a lattice cut along t (x3) into slabs of whole blocks, one slab
// per GPU: the sharding of a lattice too large for one GPU.  By eq. domdec
// of the paper (Sec. 3) D is its block-diagonal part plus the hops between
// blocks; a slab is a union of blocks, so the hops between two slabs are
// block-interaction hops across the cut, and everything else is the slab's
// own D with an open t boundary.  Each slab sends its neighbours the
// spin-projected half spinors they need (the hop's projector applied, and
// for the slab above the link as well, since that link lives here) and adds
// the hops across its faces from what they send back.  Face buffers are
// component-major: [6][F] complex, F = L0 L1 L2 sites of one t slice in
// lexicographic order x0 + L0 (x1 + L1 x2), components (h0, h1) of the half
// spinor, colour fastest.
#include "stencil.h"

namespace wdr {
namespace {

using namespace dev;

// the full link U_mu(site) from canonical FP64 links [site][mu][3][3]
template <typename T>
__device__ __forceinline__ void link_canon(const double2 *__restrict__ U, long site, int mu, su3<T> &u)
{
    const double2 *p = U + (site * 4 + mu) * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) u.m[e / 3][e % 3] = mk<T>((T)p[e].x, (T)p[e].y);
}

// one lane per site (slot, l); the lanes of the first and last t slice work
template <typename T>
__global__ __launch_bounds__(256) void k_halo_pack(Geo g, const double2 *__restrict__ U,
                                                  const T2<T> *__restrict__ in, T2<T> *__restrict__ lo,
                                                  T2<T> *__restrict__ hi)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const int slot = blockIdx.y;
    int x[4];
    const long site = canon_index(g, slot, l, x);
    const bool bot = x[3] == 0, top = x[3] == g.L[3] - 1;
    if (!bot && !top) return;
    const long F = (long)g.L[0] * g.L[1] * g.L[2], f = x[0] + (long)g.L[0] * (x[1] + (long)g.L[1] * x[2]);
    spinor<T> p;
    load_site<T>(in, slot, g.Vb, l, p);
    vec3<T> a0, a1;
    A_dn(3, p.s[2], p.s[3], a0, a1);
    if (bot) {  // (1 - g_t) psi: the forward hop of the slab below
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            st<T>(lo, a * F + f, p.s[0].c[a] - a0.c[a]);
            st<T>(lo, (3 + a) * F + f, p.s[1].c[a] - a1.c[a]);
        }
    }
    if (top) {  // (1 + g_t) U_t^+ psi: the backward hop of the slab above
        vec3<T> h0, h1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            h0.c[a] = p.s[0].c[a] + a0.c[a];
            h1.c[a] = p.s[1].c[a] + a1.c[a];
        }
        su3<T> u;
        link_canon<T>(U, site, 3, u);
        const vec3<T> c0 = mul_dag(u, h0), c1 = mul_dag(u, h1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            st<T>(hi, a * F + f, c0.c[a]);
            st<T>(hi, (3 + a) * F + f, c1.c[a]);
        }
    }
}

// out -= kappa (hops across the two t faces) on the first and last t slice
template <typename T>
__global__ __launch_bounds__(256) void k_halo_unpack(Geo g, const double2 *__restrict__ U, T kappa,
                                                    const T2<T> *__restrict__ lo, const T2<T> *__restrict__ hi,
                                                    T slo, T shi, T2<T> *__restrict__ out)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const int slot = blockIdx.y;
    int x[4];
    const long site = canon_index(g, slot, l, x);
    const bool bot = x[3] == 0, top = x[3] == g.L[3] - 1;
    if (!bot && !top) return;
    const long F = (long)g.L[0] * g.L[1] * g.L[2], f = x[0] + (long)g.L[0] * (x[1] + (long)g.L[1] * x[2]);
    spinor<T> acc;
    zero(acc);
    if (top) {  // (1 - g_t) U_t(x) psi(x + t), psi projected by the slab above
        vec3<T> h0, h1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            h0.c[a] = scale(shi, ld<T>(hi, a * F + f));
            h1.c[a] = scale(shi, ld<T>(hi, (3 + a) * F + f));
        }
        su3<T> u;
        link_canon<T>(U, site, 3, u);
        const vec3<T> c0 = mul(u, h0), c1 = mul(u, h1);
        vec3<T> d0, d1;
        Adag_h(3, c0, c1, d0, d1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            acc.s[0].c[a] = acc.s[0].c[a] + c0.c[a];
            acc.s[1].c[a] = acc.s[1].c[a] + c1.c[a];
            acc.s[2].c[a] = acc.s[2].c[a] - d0.c[a];
            acc.s[3].c[a] = acc.s[3].c[a] - d1.c[a];
        }
    }
    if (bot) {  // (1 + g_t) U_t(x - t)^+ psi(x - t), formed by the slab below
        vec3<T> c0, c1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            c0.c[a] = scale(slo, ld<T>(lo, a * F + f));
            c1.c[a] = scale(slo, ld<T>(lo, (3 + a) * F + f));
        }
        vec3<T> d0, d1;
        Adag_h(3, c0, c1, d0, d1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            acc.s[0].c[a] = acc.s[0].c[a] + c0.c[a];
            acc.s[1].c[a] = acc.s[1].c[a] + c1.c[a];
            acc.s[2].c[a] = acc.s[2].c[a] + d0.c[a];
            acc.s[3].c[a] = acc.s[3].c[a] + d1.c[a];
        }
    }
    const long base = (long)slot * 12 * g.Vb + l;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const long i = base + (long)(3 * sp + a) * g.Vb;
            st<T>(out, i, ld<T>(out, i) - scale(kappa, acc.s[sp].c[a]));
        }
}

}  // namespace

template <typename T>
void launch_halo_pack(const Geo &g, const double2 *U, const T2<T> *in, T2<T> *lo, T2<T> *hi, hipStream_t s)
{
    k_halo_pack<T><<<dim3((g.Vb + 255) / 256, g.nblk), 256, 0, s>>>(g, U, in, lo, hi);
}
template <typename T>
void launch_halo_unpack(const Geo &g, const double2 *U, T kappa, const T2<T> *lo, const T2<T> *hi, T slo, T shi,
                        T2<T> *out, hipStream_t s)
{
    k_halo_unpack<T><<<dim3((g.Vb + 255) / 256, g.nblk), 256, 0, s>>>(g, U, kappa, lo, hi, slo, shi, out);
}
template void launch_halo_pack<double>(const Geo &, const double2 *, const double2 *, double2 *, double2 *,
                                       hipStream_t);
template void launch_halo_pack<float>(const Geo &, const double2 *, const float2 *, float2 *, float2 *, hipStream_t);
template void launch_halo_unpack<double>(const Geo &, const double2 *, double, const double2 *, const double2 *,
                                         double, double, double2 *, hipStream_t);
template void launch_halo_unpack<float>(const Geo &, const double2 *, float, const float2 *, const float2 *, float,
                                        float, float2 *, hipStream_t);

}  // namespace wdr
