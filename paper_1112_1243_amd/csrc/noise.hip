// Noise vectors, geometry maps, active-link masks and the per-block
// reduction of the stochastic sample.
//
// Noise (paper Sec. 4: a complex Gaussian vector, fresh for every factor of
// eq. param): Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
// counter (canonical site, path step, sample, j) and key (seed, 3).
#include "philox.h"
#include "stencil.h"

namespace wdr {
namespace {

using namespace dev;

__device__ __forceinline__ long canon_of(const Geo &g, int slot, int l, int x[4])
{
    int b = g.slot_blk[slot];
    int loc[4];
    local_coords(g, l, loc);
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (b % g.NB[mu]) * g.B[mu] + loc[mu];
        b /= g.NB[mu];
    }
    return x[0] + (long)g.L[0] * (x[1] + (long)g.L[1] * (x[2] + (long)g.L[2] * x[3]));
}

// writes the internal-layout FP64 noise field
__global__ __launch_bounds__(256) void k_noise(Geo g, long n, int kind, uint64_t seed, const uint64_t *seeds,
                                               const int32_t *steps, const int32_t *ks, int black_only,
                                               double2 *__restrict__ out)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const int slot = blockIdx.y, m = blockIdx.z;
    const uint32_t step = (uint32_t)steps[m], k = (uint32_t)ks[m];
    if (seeds) seed = seeds[m];
    const long base = m * n + (long)slot * 12 * g.Vb + l;
    if (black_only && slot >= g.nblack) {
        for (int c = 0; c < 12; ++c) out[base + (long)c * g.Vb] = make_double2(0.0, 0.0);
        return;
    }
    int x[4];
    const uint64_t site = (uint64_t)canon_of(g, slot, l, x);
    if (kind == WDR_NOISE_Z2) {
        uint64_t c[4] = {site, step, k, 0};
        philox4x64_10(c, seed, 3);
        for (int a = 0; a < 12; ++a)
            out[base + (long)a * g.Vb] = make_double2(1.0 - 2.0 * (double)((c[0] >> a) & 1ull), 0.0);
        return;
    }
    for (int j = 0; j < 6; ++j) {
        uint64_t c[4] = {site, step, k, (uint64_t)j};
        philox4x64_10(c, seed, 3);
        for (int h = 0; h < 2; ++h) {
            const double u1 = ((double)(c[2 * h] >> 11) + 0.5) * 0x1p-53;
            const double u2 = ((double)(c[2 * h + 1] >> 11) + 0.5) * 0x1p-53;
            const double rad = sqrt(-log(u1));
            double sn, cs;
            sincos(2.0 * M_PI * u2, &sn, &cs);
            out[base + (long)(2 * j + h) * g.Vb] = make_double2(rad * cs, rad * sn);
        }
    }
}

__global__ __launch_bounds__(256) void k_site_maps(Geo g, int32_t *bid, int32_t *col, int32_t *par, int32_t *pos)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const int slot = blockIdx.y;
    int x[4];
    const long s = canon_of(g, slot, l, x);
    if (bid) bid[s] = g.slot_blk[slot];
    if (col) col[s] = slot >= g.nblack;
    if (par) par[s] = (x[0] + x[1] + x[2] + x[3]) & 1;
    if (pos) pos[s] = slot * g.Vb + l;
}

// link (x, mu) active: both ends in the region [lo, hi]^4 of in-block
// coordinates, at most one end on its boundary (paper Sec. 3)
__global__ __launch_bounds__(256) void k_active(Geo g, int lo, int hi, uint8_t *mask)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const int slot = blockIdx.y;
    int x[4];
    const long s = canon_of(g, slot, l, x);
    int r[4];
    local_coords(g, l, r);
    for (int mu = 0; mu < 4; ++mu) {
        bool ok = r[mu] >= lo && r[mu] + 1 <= hi;
        for (int nu = 0; nu < 4; ++nu)
            if (nu != mu) ok = ok && r[nu] > lo && r[nu] < hi;
        mask[s * 4 + mu] = ok ? 1 : 0;
    }
}

// per-slot sum of |eta|^2 - |z|^2 - 2 Re(conj(w) r); one workgroup per slot
__global__ __launch_bounds__(256) void k_sample_terms(Geo g, const int32_t *active, long n, const double2 *eta,
                                                      const double2 *z, const double2 *w, const double2 *r,
                                                      double *out)
{
    __shared__ double sh[4];
    const int slot = blockIdx.x, m = blockIdx.y;
    if (active && !active[m]) return;
    const long base = m * n + (long)slot * 12 * g.Vb;
    const long cnt = 12L * g.Vb;
    double acc = 0;
    for (long i = threadIdx.x; i < cnt; i += 256) {
        double2 e = eta[base + i];
        double v = e.x * e.x + e.y * e.y;
        if (z) {
            double2 a = z[base + i];
            v -= a.x * a.x + a.y * a.y;
        }
        if (w && r) {
            double2 a = w[base + i], b = r[base + i];
            v -= 2.0 * (a.x * b.x + a.y * b.y);
        }
        acc += v;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[(long)m * g.nblk + slot] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

}  // namespace

void launch_noise(const Geo &g, const Sys &sy, int kind, uint64_t seed, const uint64_t *seeds, const int32_t *steps,
                  const int32_t *ks, int black_only, double2 *out, hipStream_t s)
{
    k_noise<<<dim3((g.Vb + 255) / 256, g.nblk, sy.M), 256, 0, s>>>(g, sy.n, kind, seed, seeds, steps, ks, black_only,
                                                                    out);
}
void launch_site_maps(const Geo &g, int32_t *bid, int32_t *col, int32_t *par, int32_t *pos, hipStream_t s)
{
    k_site_maps<<<dim3((g.Vb + 255) / 256, g.nblk), 256, 0, s>>>(g, bid, col, par, pos);
}
void launch_active_links(const Geo &g, int lo, int hi, uint8_t *mask, hipStream_t s)
{
    k_active<<<dim3((g.Vb + 255) / 256, g.nblk), 256, 0, s>>>(g, lo, hi, mask);
}
void launch_sample_terms(const Geo &g, const Sys &sy, const double2 *eta, const double2 *z, const double2 *w,
                         const double2 *r, double *per_slot, hipStream_t s)
{
    k_sample_terms<<<dim3(g.nblk, sy.M), 256, 0, s>>>(g, sy.active, sy.n, eta, z, w, r, per_slot);
}

}  // namespace wdr
