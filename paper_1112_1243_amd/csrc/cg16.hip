// FP16 storage for the even-odd CG of the global solves (the inversion that
// paper Sec. 4 needs once for each factor of eq. param), 4^4 blocks, SU(3)
// links.
//
// Layouts (internal to the CG; the FP16 fields of the C ABI keep theirs):
//   E16 field  [system][slot][Vh][12] FP16 complex: one parity of every
//              block, site-major, so the 12 values of a site are 48
//              contiguous bytes (three 16-byte loads per lane); one
//              power-of-two scale per (system, slot): stored value v / s,
//              s = 2^ceil(log2 max |component|) over the block's half.
//   E16 links  [slot][parity][mu] chunks of Vh links, each chunk the first
//              four entries of rows 0-1 (16 bytes per link, Vh of them) then
//              the last two (8 bytes per link): U_mu(x) of the sites of that
//              parity, boundary phase folded in, third row rebuilt.
// The hops of the stencil (spin projection, third link row, link times half
// spinor) run in packed FP16 on the stored values, whose magnitude is at
// most 1 (one v_pk_fma_f16 handles a complex pair; the kernel was bound by
// its FP32 instruction issue); everything else is FP32, and norms are summed
// in FP64.
#include "clover.h"
#include "half2.h"
#include "stencil.h"

namespace wdr {
namespace {

using namespace dev;

constexpr int B4 = 4, VB4 = 256, VH4 = 128;

typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef uint32_t v2u __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) v4u *G4;  // 16-byte words in global memory
union Q16 {
    v4u u;
    h2 h[4];
};
union D16 {
    v2u u;
    h2 h[2];
};

template <typename P> __device__ __forceinline__ const __attribute__((address_space(1))) P *glob(const P *p)
{
    return (const __attribute__((address_space(1))) P *)p;
}
__device__ __forceinline__ G4 g4(const uint4 *p) { return (G4)p; }

// the 12 values of site `site` (index in units of sites) times scale s
__device__ __forceinline__ void ld_site(G4 f, long site, float s, cx<float> v[12])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        Q16 q;
        q.u = f[site * 3 + k];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[4 * k + j] = mk<float>((float)q.h[j].x * s, (float)q.h[j].y * s);
    }
}
__device__ __forceinline__ void st_site(uint4 *f, long site, const cx<float> v[12], float inv)
{
    __attribute__((address_space(1))) v4u *o = (__attribute__((address_space(1))) v4u *)f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        Q16 q;
#pragma unroll
        for (int j = 0; j < 4; ++j) q.h[j] = to_h2(v[4 * k + j], inv);
        o[site * 3 + k] = q.u;
    }
}
// |v|^2 of the values as stored (rounded to FP16, times the scale)
__device__ __forceinline__ double stored_norm2(const cx<float> v[12], float s, float inv)
{
    double n = 0;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const h2 h = to_h2(v[c], inv);
        const double re = (double)((float)h.x * s), im = (double)((float)h.y * s);
        n += re * re + im * im;
    }
    return n;
}

// link chunk (slot, parity, mu): entries 0..3 for Vh sites, then 4..5
__device__ __forceinline__ void ld_link(const __attribute__((address_space(1))) h2 *L, int chunk, int i, float sg,
                                        su3<float> &u)
{
    const auto *base = L + (long)chunk * VH4 * 6;
    Q16 a;
    D16 b;
    a.u = ((G4)base)[i];
    b.u = ((const __attribute__((address_space(1))) v2u *)(base + VH4 * 4))[i];
    u.m[0][0] = mk<float>((float)a.h[0].x, (float)a.h[0].y);
    u.m[0][1] = mk<float>((float)a.h[1].x, (float)a.h[1].y);
    u.m[0][2] = mk<float>((float)a.h[2].x, (float)a.h[2].y);
    u.m[1][0] = mk<float>((float)a.h[3].x, (float)a.h[3].y);
    u.m[1][1] = mk<float>((float)b.h[0].x, (float)b.h[0].y);
    u.m[1][2] = mk<float>((float)b.h[1].x, (float)b.h[1].y);
    // third row conj(row0 x row1), times the boundary sign that the stored
    // rows carry when the link wraps around the lattice
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int p = (c + 1) % 3, q = (c + 2) % 3;
        const cx<float> v = u.m[0][p] * u.m[1][q] - u.m[0][q] * u.m[1][p];
        u.m[2][c] = mk<float>(sg * v.re, -sg * v.im);
    }
}

// largest |component| over the workgroup of NT threads; sh: NT / 64 floats
template <int NT> __device__ __forceinline__ float block_max(float v, float *sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    float r = sh[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) r = fmaxf(r, sh[w]);
    return r;
}
template <int NT> __device__ __forceinline__ double block_sum(double v, double *sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) r += sh[w];
    return r;
}

// the block's power-of-two scale of v (all threads), rounded store, and the
// norm of the stored values into partial (2 doubles per (system, slot), the
// layout of the deterministic reduction's first pass) when asked
__device__ __forceinline__ void store_block(const cx<float> v[12], uint4 *outv, float *outs, long site, long blk,
                                            double *partial, long pidx)
{
    __shared__ float redf[VH4 / 64];
    __shared__ double redd[VH4 / 64];
    float mx = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) mx = fmaxf(mx, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
    const float s = pow2_at_least(block_max<VH4>(mx, redf)), inv = 1.f / s;
    st_site(outv, site, v, inv);
    if (threadIdx.x == 0) outs[blk] = s;
    if (partial) {
        const double n = block_sum<VH4>(stored_norm2(v, s, inv), redd);
        if (threadIdx.x == 0) {
            partial[2 * pidx] = n;
            partial[2 * pidx + 1] = 0.0;
        }
    }
}

// LDS copy of FP16 sites: 12 complex FP16 per site, 48 bytes, read as three
// 16-byte words
struct Site16 {
    v4u q[3];
};
__device__ __forceinline__ void ld_site_lds(const Site16 *sh, int i, float s, spinor<float> &p)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        Q16 q;
        q.u = sh[i].q[k];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = 4 * k + j;
            p.s[c / 3].c[c % 3] = mk<float>((float)q.h[j].x * s, (float)q.h[j].y * s);
        }
    }
}
// a link's two rows as loaded (16 + 8 bytes), unpacked later
struct Link16 {
    Q16 a;
    D16 b;
};
__device__ __forceinline__ void ld_link_raw(const __attribute__((address_space(1))) h2 *L, int chunk, int i,
                                            Link16 &k)
{
    const auto *base = L + (long)chunk * VH4 * 6;
    k.a.u = ((G4)base)[i];
    k.b.u = ((const __attribute__((address_space(1))) v2u *)(base + VH4 * 4))[i];
}
__device__ __forceinline__ void unpack_link(const Link16 &k, float sg, su3<float> &u)
{
    u.m[0][0] = mk<float>((float)k.a.h[0].x, (float)k.a.h[0].y);
    u.m[0][1] = mk<float>((float)k.a.h[1].x, (float)k.a.h[1].y);
    u.m[0][2] = mk<float>((float)k.a.h[2].x, (float)k.a.h[2].y);
    u.m[1][0] = mk<float>((float)k.a.h[3].x, (float)k.a.h[3].y);
    u.m[1][1] = mk<float>((float)k.b.h[0].x, (float)k.b.h[0].y);
    u.m[1][2] = mk<float>((float)k.b.h[1].x, (float)k.b.h[1].y);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int p = (c + 1) % 3, q = (c + 2) % 3;
        const cx<float> v = u.m[0][p] * u.m[1][q] - u.m[0][q] * u.m[1][p];
        u.m[2][c] = mk<float>(sg * v.re, -sg * v.im);
    }
}

// Halo of one block half: the sites of parity q in the boundary layer of the
// neighbour block across face f = 2 mu + d (d = 0: +mu, layer x_mu = 0 of
// that block; d = 1: -mu, layer x_mu = B - 1), 32 per face for 4^4 blocks.
// Entry k of a face: the three other coordinates (increasing direction) are
// (u, v, w) with w = k >> 3, v = (k >> 1) & 3 and u the value of parity q in
// {2 (k & 1), 2 (k & 1) + 1}.
__device__ __forceinline__ void halo_site(int f, int k, int q, int y[4])
{
    const int mu = f >> 1;
    y[mu] = (f & 1) ? B4 - 1 : 0;
    int o[3], n = 0;
#pragma unroll
    for (int d = 0; d < 4; ++d)
        if (d != mu) o[n++] = d;
    const int w = k >> 3, v = (k >> 1) & 3;
    y[o[2]] = w;
    y[o[1]] = v;
    y[o[0]] = 2 * (k & 1) + ((q + y[mu] + v + w) & 1);
}
template <int MU> __device__ __forceinline__ int halo_entry(const int y[4])
{
    constexpr int o0 = MU == 0 ? 1 : 0, o1 = MU <= 1 ? 2 : 1, o2 = MU <= 2 ? 3 : 2;
    return (y[o2] << 3) | (y[o1] << 1) | (y[o0] >> 1);
}

// The two hops of direction MU at output site x (parity par): neighbours from
// the block's LDS copy (own) or the LDS halo (across a face, with that
// neighbour block's scale), links from the prefetched registers.  The spin
// projection, the third link row and the link times half spinor run in
// packed FP16 on the stored values (at most 1 in magnitude, the block scale
// divided out); each hop's half spinor is then scaled and accumulated in
// FP32.  DAG applies gamma_5 to the loaded spinors (the caller to the
// result).
template <int MU, int DAG>
__device__ __forceinline__ void hop16(const Site16 *own, const Site16 *halo, float s_own, const float *s_face, int par,
                                      const int x[4], const Link16 &lf, const Link16 &lb, float wrap_f, float wrap_b,
                                      spinor<float> &acc)
{
    typedef Cube<B4> CB;
    // A psi_dn for psi_dn = (d0, d1): (o0, o1) = (map(d_i0), map(d_i1))
    constexpr int i0 = MU == 0 ? 1 : MU == 1 ? 1 : 0, i1 = MU == 0 ? 0 : MU == 1 ? 0 : 1;
    constexpr int m0 = MU == 0 ? 3 : MU == 1 ? 1 : MU == 2 ? 3 : 0, m1 = MU == 0 ? 3 : MU == 1 ? 0 : MU == 2 ? 2 : 0;
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        const bool fwd = dir == 0;
        const bool inside = fwd ? x[MU] + 1 < B4 : x[MU] > 0;
        int y[4] = {x[0], x[1], x[2], x[3]};
        y[MU] = fwd ? (inside ? x[MU] + 1 : 0) : (inside ? x[MU] - 1 : B4 - 1);
        const int e = inside ? CB::index(y) - (1 - par) * VH4 : (2 * MU + dir) * 32 + halo_entry<MU>(y);
        const Site16 &st = inside ? own[e] : halo[e];
        const float s = inside ? s_own : s_face[2 * MU + dir];
        h2 p[12];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Q16 q;
            q.u = st.q[k];
#pragma unroll
            for (int j = 0; j < 4; ++j) p[4 * k + j] = q.h[j];
        }
        // h = psi_up -+ A psi_dn (forward -, backward +; gamma_5 flips psi_dn)
        const bool minus = fwd != (DAG != 0);
        h2 h0[3], h1[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const h2 o0 = hmap(p[6 + 3 * i0 + a], m0), o1 = hmap(p[6 + 3 * i1 + a], m1);
            h0[a] = minus ? p[a] - o0 : p[a] + o0;
            h1[a] = minus ? p[3 + a] - o1 : p[3 + a] + o1;
        }
        // the link: rows 0 and 1 as stored, row 2 = sg conj(row0 x row1)
        const Link16 &lk = fwd ? lf : lb;
        const float sg = fwd ? wrap_f : wrap_b;
        h2 u[3][3];
        u[0][0] = lk.a.h[0];
        u[0][1] = lk.a.h[1];
        u[0][2] = lk.a.h[2];
        u[1][0] = lk.a.h[3];
        u[1][1] = lk.b.h[0];
        u[1][2] = lk.b.h[1];
        const h2 sgc = (h2){(_Float16)sg, (_Float16)(-sg)};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int pp = (c + 1) % 3, qq = (c + 2) % 3;
            const h2 v = hcfma(u[0][qq], -u[1][pp], hcfma(u[0][pp], u[1][qq], (h2){0, 0}));
            u[2][c] = v * sgc;
        }
        // c = U h (forward) or U^+ h (backward)
        h2 c0[3], c1[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            h2 r0 = (h2){0, 0}, r1 = (h2){0, 0};
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if (fwd) {
                    r0 = hcfma(u[a][b], h0[b], r0);
                    r1 = hcfma(u[a][b], h1[b], r1);
                } else {
                    r0 = hcjfma(u[b][a], h0[b], r0);
                    r1 = hcjfma(u[b][a], h1[b], r1);
                }
            }
            c0[a] = r0;
            c1[a] = r1;
        }
        // scaled to FP32, spins 2 and 3 rebuilt as -+ A^+ c
        vec3<float> f0, f1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            f0.c[a] = mk<float>(s * (float)c0[a].x, s * (float)c0[a].y);
            f1.c[a] = mk<float>(s * (float)c1[a].x, s * (float)c1[a].y);
        }
        vec3<float> d0, d1;
        Adag_h(MU, f0, f1, d0, d1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            acc.s[0].c[a] = acc.s[0].c[a] + f0.c[a];
            acc.s[1].c[a] = acc.s[1].c[a] + f1.c[a];
            acc.s[2].c[a] = fwd ? acc.s[2].c[a] - d0.c[a] : acc.s[2].c[a] + d0.c[a];
            acc.s[3].c[a] = fwd ? acc.s[3].c[a] - d1.c[a] : acc.s[3].c[a] + d1.c[a];
        }
    }
}

// out = diag + f H_{par, 1-par} in on the sites of parity par (gamma_5 on
// both sides of H for DAG), f = fs kappa_m (or fk without a kappa table);
// FP16 E16 fields in and out, diag optional.  One workgroup per block and
// system, one lane per output site.  Every global load is issued up front:
// the block's input half and its halo (the 256 face sites of the neighbour
// blocks, two per lane) go to LDS as FP16, the eight links of the lane's
// hops to registers; the hops then read LDS and registers only.
// partial (optional): |out|^2 of the stored values per block.  CL: with the
// clover term (ctab: the FP32 A and A^-1 of clover.h per system) the output
// is A diag + f H in (CLOV_DIAG) or A^-1 (diag + f H in) (CLOV_INV), in FP32
// before the rounded store.
template <int DAG, int CL>
__global__ __launch_bounds__(VH4) void k_eo16(Geo g, const int32_t *__restrict__ active,
                                              const int32_t *__restrict__ list, const h2 *const *__restrict__ ltab,
                                              const double *__restrict__ kap, float fs, float fk, int par,
                                              const int32_t *__restrict__ sched, const uint4 *__restrict__ inv,
                                              const float *__restrict__ ins, const uint4 *__restrict__ dgv,
                                              const float *__restrict__ dgs, uint4 *__restrict__ outv,
                                              float *__restrict__ outs, double *__restrict__ partial,
                                              const float *const *__restrict__ ctab)
{
    typedef Cube<B4> CB;
    __shared__ Site16 own[VH4];       // the block's input half
    __shared__ Site16 halo[8 * 32];   // face sites of the neighbour blocks
    const int m = sys_at(list, blockIdx.y);
    if (active && !active[m]) return;
    const float f = kap ? fs * (float)kap[m] : fk;
    const int slot = sched[blockIdx.x];
    const int t = threadIdx.x, q = 1 - par;
    const long fbase = (long)m * g.nblk;
    const G4 inf = g4(inv);
    int nbr[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) nbr[k] = g.slot_nbr[slot * 8 + k];
    // input half and halo to LDS (raw FP16 words)
    {
        const long si = ((fbase + slot) * VH4 + t) * 3;
        own[t].q[0] = inf[si];
        own[t].q[1] = inf[si + 1];
        own[t].q[2] = inf[si + 2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int e = t + r * VH4, fc = e >> 5;
            int y[4];
            halo_site(fc, e & 31, q, y);
            const long hi = ((fbase + nbr[fc]) * VH4 + CB::index(y) - q * VH4) * 3;
            halo[e].q[0] = inf[hi];
            halo[e].q[1] = inf[hi + 1];
            halo[e].q[2] = inf[hi + 2];
        }
    }
    int x[4];
    CB::coords(par * VH4 + t, x);
    // the eight links of this lane's hops: U_mu(x) and U_mu(x - mu)
    const auto *L = glob(ltab[m]);
    Link16 lf[4], lb[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        ld_link_raw(L, (slot * 2 + par) * 4 + mu, t, lf[mu]);
        int y[4] = {x[0], x[1], x[2], x[3]};
        const bool inside = x[mu] > 0;
        y[mu] = inside ? x[mu] - 1 : B4 - 1;
        ld_link_raw(L, ((inside ? slot : nbr[2 * mu + 1]) * 2 + q) * 4 + mu, CB::index(y) - q * VH4, lb[mu]);
    }
    const float s_own = ins[fbase + slot];
    float s_face[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) s_face[k] = ins[fbase + nbr[k]];
    // boundary signs of the links that wrap around the lattice (their stored
    // rows carry bc; the rebuilt third row needs it once more)
    float wf[4], wb[4];
    const int bl = g.slot_blk[slot];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        wf[mu] = wb[mu] = 1.f;
        if (g.bc[mu] < 0) {
            int b2 = bl;
            for (int d = 0; d < mu; ++d) b2 /= g.NB[d];
            const int nmu = b2 % g.NB[mu];
            if (nmu == g.NB[mu] - 1 && x[mu] == B4 - 1) wf[mu] = -1.f;
            if (nmu == 0 && x[mu] == 0) wb[mu] = -1.f;
        }
    }
    __syncthreads();
    spinor<float> acc;
    zero(acc);
    hop16<0, DAG>(own, halo, s_own, s_face, par, x, lf[0], lb[0], wf[0], wb[0], acc);
    hop16<1, DAG>(own, halo, s_own, s_face, par, x, lf[1], lb[1], wf[1], wb[1], acc);
    hop16<2, DAG>(own, halo, s_own, s_face, par, x, lf[2], lb[2], wf[2], wb[2], acc);
    hop16<3, DAG>(own, halo, s_own, s_face, par, x, lf[3], lb[3], wf[3], wb[3], acc);
    const long site = (fbase + slot) * VH4 + t;
    cx<float> dg[12];
    if (dgv) ld_site(g4(dgv), site, dgs[fbase + slot], dg);
    cx<float> res[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        cx<float> v = scale(f, acc.s[c / 3].c[c % 3]);
        if (DAG && c >= 6) v = neg(v);
        res[c] = dgv && !CL ? v + dg[c] : v;
    }
    if (CL) {  // A diag + hops, or A^-1 (diag + hops)
        if (!dgv)
#pragma unroll
            for (int c = 0; c < 12; ++c) dg[c] = mk<float>(0.f, 0.f);
        clov_site<float, CL>(ctab[m], (long)g.V, slot, 2 * VH4, par * VH4 + t, dg, res);
    }
    store_block(res, outv, outs, site, fbase + slot, partial, fbase + slot);
}

// one CG step on the FP16 vectors of system m, alpha = sc[8m].x / sc[8m+1].x:
// x += alpha w (x FP32, the internal component-major layout, even sites;
// XUPD = 0: x is left alone and alpha is stored in alpha[m] for a later
// k_x16_flush), r -= alpha q (FP16, fresh block scales), partial sums of
// |r|^2
template <int XUPD>
__global__ __launch_bounds__(VH4) void k_xr16(Geo g, const int32_t *__restrict__ active,
                                              const int32_t *__restrict__ list, const double2 *__restrict__ sc,
                                              float2 *__restrict__ x, float *__restrict__ alpha,
                                              const uint4 *__restrict__ wv, const float *__restrict__ ws,
                                              const uint4 *__restrict__ qv, const float *__restrict__ qs,
                                              uint4 *__restrict__ rv, float *__restrict__ rs,
                                              double *__restrict__ partial)
{
    const int m = sys_at(list, blockIdx.y);
    if (active && !active[m]) return;
    const int slot = blockIdx.x, t = threadIdx.x;
    const double ww = sc[8L * m + 1].x;
    const float a = (float)(ww > 0 ? sc[8L * m].x / ww : 0.0);
    if (!XUPD && slot == 0 && t == 0) alpha[m] = a;
    const long blk = (long)m * g.nblk + slot, site = blk * VH4 + t;
    cx<float> q[12], r[12];
    ld_site(g4(qv), site, qs[blk], q);
    ld_site(g4(rv), site, rs[blk], r);
    if (XUPD) {
        cx<float> w[12];
        ld_site(g4(wv), site, ws[blk], w);
        float2 *xs = x + blk * 12 * VB4 + t;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            float2 xv = xs[c * VB4];
            xv.x += a * w[c].re;
            xv.y += a * w[c].im;
            xs[c * VB4] = xv;
        }
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) r[c] = r[c] - scale(a, q[c]);
    __syncthreads();  // every lane has read its r before the block's scale is rewritten
    store_block(r, rv, rs, site, blk, partial, blk);
}

// x += alpha_j w_j for the NK steps since the last flush, in step order and
// with the rounding of the step-by-step update (x FP32 as in k_xr16; alpha_j
// of system m at alpha[j * M + m], w_j in the E16 layout)
struct W16Set {
    const uint4 *v[4];
    const float *s[4];
};
template <int NK>
__global__ __launch_bounds__(VH4) void k_x16_flush(Geo g, const int32_t *__restrict__ active,
                                                   const int32_t *__restrict__ list, const float *__restrict__ alpha,
                                                   int M, W16Set w, float2 *__restrict__ x)
{
    const int m = sys_at(list, blockIdx.y);
    if (active && !active[m]) return;
    const int slot = blockIdx.x, t = threadIdx.x;
    const long blk = (long)m * g.nblk + slot, site = blk * VH4 + t;
    float2 *xs = x + blk * 12 * VB4 + t;
    float2 xv[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) xv[c] = xs[c * VB4];
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const float a = alpha[(long)j * M + m];
        cx<float> wj[12];
        ld_site(g4(w.v[j]), site, w.s[j][blk], wj);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            xv[c].x += a * wj[c].re;
            xv[c].y += a * wj[c].im;
        }
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) xs[c * VB4] = xv[c];
}

// p = r + beta p (beta = sc[8m + 4].x), or p = r with copy
__global__ __launch_bounds__(VH4) void k_p16(Geo g, const int32_t *__restrict__ active,
                                             const int32_t *__restrict__ list, const double2 *__restrict__ sc,
                                             int copy, const uint4 *__restrict__ rv, const float *__restrict__ rs,
                                             uint4 *__restrict__ pv, float *__restrict__ ps)
{
    const int m = sys_at(list, blockIdx.y);
    if (active && !active[m]) return;
    const int slot = blockIdx.x, t = threadIdx.x;
    const long blk = (long)m * g.nblk + slot, site = blk * VH4 + t;
    cx<float> r[12], p[12];
    ld_site(g4(rv), site, rs[blk], r);
    if (!copy) {
        const float b = (float)sc[8L * m + 4].x;
        ld_site(g4(pv), site, ps[blk], p);
#pragma unroll
        for (int c = 0; c < 12; ++c) r[c] = r[c] + scale(b, p[c]);
    }
    __syncthreads();
    store_block(r, pv, ps, site, blk, nullptr, 0);
}

// the middle level's residual: r = bh - d on even sites (FP32, component-major)
// into the FP16 iterated residual, and the partial sums of |r|^2 of the FP32
// values
__global__ __launch_bounds__(VH4) void k_r16_from32(Geo g, const int32_t *__restrict__ active,
                                                    const int32_t *__restrict__ list, const float2 *__restrict__ bh,
                                                    const float2 *__restrict__ d, uint4 *__restrict__ rv,
                                                    float *__restrict__ rs, double *__restrict__ partial)
{
    __shared__ double redd[VH4 / 64];
    const int m = sys_at(list, blockIdx.y);
    if (active && !active[m]) return;
    const int slot = blockIdx.x, t = threadIdx.x;
    const long blk = (long)m * g.nblk + slot, site = blk * VH4 + t;
    const long e0 = blk * 12 * VB4 + t;
    cx<float> r[12];
    double n = 0;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const float2 a = bh[e0 + c * VB4], b = d[e0 + c * VB4];
        r[c] = mk<float>(a.x - b.x, a.y - b.y);
        n += (double)r[c].re * r[c].re + (double)r[c].im * r[c].im;
    }
    n = block_sum<VH4>(n, redd);
    if (t == 0) {
        partial[2 * blk] = n;
        partial[2 * blk + 1] = 0.0;
    }
    store_block(r, rv, rs, site, blk, nullptr, 0);
}

// the outer level's reliable update (after x64 += x32 and r64 = bh - Dhat
// x64): the middle system restarts from r64, bh32 = (float) r64, x32 = 0,
// and the FP16 iterated residual r = r64
__global__ __launch_bounds__(VH4) void k_r16_from64(Geo g, const int32_t *__restrict__ active,
                                                    const int32_t *__restrict__ list, const double2 *__restrict__ r64,
                                                    float2 *__restrict__ bh, float2 *__restrict__ x,
                                                    uint4 *__restrict__ rv, float *__restrict__ rs)
{
    const int m = sys_at(list, blockIdx.y);
    if (active && !active[m]) return;
    const int slot = blockIdx.x, t = threadIdx.x;
    const long blk = (long)m * g.nblk + slot, site = blk * VH4 + t;
    const long e0 = blk * 12 * VB4 + t;
    cx<float> r[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const double2 v = r64[e0 + c * VB4];
        r[c] = mk<float>((float)v.x, (float)v.y);
        bh[e0 + c * VB4] = make_float2(r[c].re, r[c].im);
        x[e0 + c * VB4] = make_float2(0.f, 0.f);
    }
    store_block(r, rv, rs, site, blk, nullptr, 0);
}

// the sites of parity par of an internal FP64 field (component-major) into
// an E16 field with fresh scales, or back (the other parity's sites of the
// FP64 field set to zero)
__global__ __launch_bounds__(VH4) void k_e16_from64(Geo g, int par, const double2 *__restrict__ in,
                                                    uint4 *__restrict__ ov, float *__restrict__ os)
{
    const int slot = blockIdx.x, m = blockIdx.y, t = threadIdx.x;
    const long blk = (long)m * g.nblk + slot, e0 = blk * 12 * VB4 + par * VH4 + t;
    cx<float> v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const double2 d = in[e0 + c * VB4];
        v[c] = mk<float>((float)d.x, (float)d.y);
    }
    store_block(v, ov, os, blk * VH4 + t, blk, nullptr, 0);
}
__global__ __launch_bounds__(VH4) void k_e16_to64(Geo g, int par, const uint4 *__restrict__ iv,
                                                  const float *__restrict__ is, double2 *__restrict__ out)
{
    const int slot = blockIdx.x, m = blockIdx.y, t = threadIdx.x;
    const long blk = (long)m * g.nblk + slot, e0 = blk * 12 * VB4 + t;
    cx<float> v[12];
    ld_site(g4(iv), blk * VH4 + t, is[blk], v);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        out[e0 + c * VB4 + par * VH4] = make_double2((double)v[c].re, (double)v[c].im);
        out[e0 + c * VB4 + (1 - par) * VH4] = make_double2(0.0, 0.0);
    }
}

// E16 links from the internal FP64 links ([slot][mu][9][Vb], boundary phase
// folded in), rounded through FP32 like every FP16 copy of the library
__global__ __launch_bounds__(256) void k_pack_links_e16(long total, const double2 *__restrict__ u64,
                                                        h2 *__restrict__ out)
{
    const long k = (long)blockIdx.x * 256 + threadIdx.x;  // (slot, mu, l)
    if (k >= total) return;
    const int l = (int)(k % VB4);
    const long sm = k / VB4;
    const int mu = (int)(sm % 4);
    const long slot = sm / 4;
    const int par = l >= VH4 ? 1 : 0, i = l - par * VH4;
    const double2 *src = u64 + sm * 9 * VB4 + l;
    h2 *chunk = out + ((slot * 2 + par) * 4 + mu) * VH4 * 6;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const double2 v = src[(long)e * VB4];
        h2 h;
        h.x = (_Float16)(float)v.x;
        h.y = (_Float16)(float)v.y;
        if (e < 4)
            chunk[i * 4 + e] = h;
        else
            chunk[VH4 * 4 + i * 2 + (e - 4)] = h;
    }
}

}  // namespace

bool e16_geometry(const Geo &g)
{
    return g.B[0] == B4 && g.B[1] == B4 && g.B[2] == B4 && g.B[3] == B4 && g.colourable;
}

size_t e16_field_bytes(const Geo &g, int M) { return (size_t)M * g.nblk * (VH4 * 48 + sizeof(float)); }

E16 e16_field(const Geo &g, int M, void *p)
{
    uint4 *v = static_cast<uint4 *>(p);
    return E16{v, reinterpret_cast<float *>(v + (size_t)M * g.nblk * VH4 * 3)};
}

void launch_pack_links_e16(const Geo &g, const double2 *u64, h2 *e16, hipStream_t s)
{
    const long total = (long)g.nblk * 4 * VB4;
    k_pack_links_e16<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(total, u64, e16);
}

void launch_eo16(const Geo &g, const Sys &sy, Links16 U, float fs, float fk, int par, int dag, E16c in, E16c diag,
                 E16 out, double *partial, hipStream_t s, const float *const *ctab, int cmode)
{
    const int si = sched_index(g, 0, g.nblk);
    const dim3 grid(g.nblk, sy.launch_m());
    const int cl = ctab ? cmode : CLOV_NONE;
#define WDR_EO16(D, C)                                                                                         \
    k_eo16<D, C><<<grid, VH4, 0, s>>>(g, sy.active, sy.list, U.tab, U.kap, fs, fk, par, g.sched[si], in.v, in.s, \
                                      diag.v, diag.s, out.v, out.s, partial, ctab)
    if (dag) {
        if (cl == CLOV_DIAG) WDR_EO16(1, CLOV_DIAG);
        else if (cl == CLOV_INV) WDR_EO16(1, CLOV_INV);
        else WDR_EO16(1, CLOV_NONE);
    } else {
        if (cl == CLOV_DIAG) WDR_EO16(0, CLOV_DIAG);
        else if (cl == CLOV_INV) WDR_EO16(0, CLOV_INV);
        else WDR_EO16(0, CLOV_NONE);
    }
#undef WDR_EO16
}

void launch_e16_from64(const Geo &g, int M, int par, const double2 *in, E16 out, hipStream_t s)
{
    k_e16_from64<<<dim3(g.nblk, M), VH4, 0, s>>>(g, par, in, out.v, out.s);
}

void launch_e16_to64(const Geo &g, int M, int par, E16c in, double2 *out, hipStream_t s)
{
    k_e16_to64<<<dim3(g.nblk, M), VH4, 0, s>>>(g, par, in.v, in.s, out);
}

void launch_xr16(const Geo &g, const Sys &sy, const double2 *sc, float2 *x, float *alpha, E16c w, E16c q, E16 r,
                 double *partial, hipStream_t s)
{
    const dim3 gr(g.nblk, sy.launch_m());
    if (x)
        k_xr16<1><<<gr, VH4, 0, s>>>(g, sy.active, sy.list, sc, x, alpha, w.v, w.s, q.v, q.s, r.v, r.s, partial);
    else
        k_xr16<0><<<gr, VH4, 0, s>>>(g, sy.active, sy.list, sc, x, alpha, w.v, w.s, q.v, q.s, r.v, r.s, partial);
}

void launch_x16_flush(const Geo &g, const Sys &sy, const float *alpha, int M, const E16c *w, int nk, float2 *x,
                      hipStream_t s)
{
    W16Set ws{};
    for (int j = 0; j < nk && j < 4; ++j) {
        ws.v[j] = w[j].v;
        ws.s[j] = w[j].s;
    }
    const dim3 gr(g.nblk, sy.launch_m());
    switch (nk) {
    case 1: k_x16_flush<1><<<gr, VH4, 0, s>>>(g, sy.active, sy.list, alpha, M, ws, x); break;
    case 2: k_x16_flush<2><<<gr, VH4, 0, s>>>(g, sy.active, sy.list, alpha, M, ws, x); break;
    case 3: k_x16_flush<3><<<gr, VH4, 0, s>>>(g, sy.active, sy.list, alpha, M, ws, x); break;
    default: k_x16_flush<4><<<gr, VH4, 0, s>>>(g, sy.active, sy.list, alpha, M, ws, x); break;
    }
}

void launch_p16(const Geo &g, const Sys &sy, const double2 *sc, int copy, E16c r, E16 p, hipStream_t s)
{
    k_p16<<<dim3(g.nblk, sy.launch_m()), VH4, 0, s>>>(g, sy.active, sy.list, sc, copy, r.v, r.s, p.v, p.s);
}

void launch_r16_from32(const Geo &g, const Sys &sy, const float2 *bh, const float2 *d, E16 r, double *partial,
                       hipStream_t s)
{
    k_r16_from32<<<dim3(g.nblk, sy.launch_m()), VH4, 0, s>>>(g, sy.active, sy.list, bh, d, r.v, r.s, partial);
}

void launch_r16_from64(const Geo &g, const Sys &sy, const double2 *r64, float2 *bh, float2 *x, E16 r, hipStream_t s)
{
    k_r16_from64<<<dim3(g.nblk, sy.launch_m()), VH4, 0, s>>>(g, sy.active, sy.list, r64, bh, x, r.v, r.s);
}

}  // namespace wdr
