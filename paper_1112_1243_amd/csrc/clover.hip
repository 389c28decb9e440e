// Clover term: construction of A = 1 + T and A^-1 from the links, the
// site-local products A psi and A^-1 psi, and the canonical export (the term
// and its storage are described in clover.h; paper Sec. 3 defines the active
// links for Wilson fermions with clover term, Sec. 7 names the clover
// action).
//
// Construction, in FP64:
//   k_clover_planes  one lane per (site, plane mu < nu): Q_{mu nu}, the four
//                    plaquettes of the plane that begin and end at the site,
//                    all run mu-side first, and Fhat_{mu nu} = (Q - Q^+) / 8
//                    into a work field [plane][9][V]
//   k_clover_blocks  one lane per (site, chirality): the block of A from the
//                    six Fhat, its LDL^H factorisation and A^-1.
// In the chiral basis sigma_{mu nu} restricted to one chirality is a Pauli
// matrix: sigma_{jk} = -eps_{jkl} s_l for spatial j, k (both chiralities)
// and sigma_{k4} = +s_k / -s_k (chirality 0 / 1), so with c = c_sw kappa
//   T_chi = i c sum_k s_k (x) G_k = i c [[G_3, G_1 - i G_2], [G_1 + i G_2, -G_3]],
//   G_1 = -F_23 + e F_14,  G_2 = F_13 + e F_24,  G_3 = -F_12 + e F_34
// (continuum labels 1..4 = lattice directions 0..3, e = +1 / -1 for
// chirality 0 / 1).  The links carry the boundary phases folded in; around a
// closed loop they cancel (every phase enters once as U and once as U^+).
#include <algorithm>

#include "clover.h"
#include "stencil.h"

namespace wdr {
namespace {

using namespace dev;

typedef su3<double> M3;

__device__ __forceinline__ M3 mm(const M3 &a, const M3 &b)  // a b
{
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[i][0] * b.m[0][j] + a.m[i][1] * b.m[1][j] + a.m[i][2] * b.m[2][j];
    return r;
}
__device__ __forceinline__ M3 mmd(const M3 &a, const M3 &b)  // a b^+
{
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r.m[i][j] = conjmul(b.m[j][0], a.m[i][0]) + conjmul(b.m[j][1], a.m[i][1]) + conjmul(b.m[j][2], a.m[i][2]);
    return r;
}
__device__ __forceinline__ M3 mdm(const M3 &a, const M3 &b)  // a^+ b
{
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r.m[i][j] = conjmul(a.m[0][i], b.m[0][j]) + conjmul(a.m[1][i], b.m[1][j]) + conjmul(a.m[2][i], b.m[2][j]);
    return r;
}

// a site as (slot, in-block coordinates); one step in direction mu crosses
// into the neighbour slot at a block face (the slot table wraps the lattice)
struct Pos {
    int slot;
    int x[4];
};
__device__ __forceinline__ Pos moved(const Geo &g, Pos p, int mu, int d)
{
    p.x[mu] += d;
    if (p.x[mu] == g.B[mu]) {
        p.x[mu] = 0;
        p.slot = g.slot_nbr[p.slot * 8 + 2 * mu];
    } else if (p.x[mu] < 0) {
        p.x[mu] = g.B[mu] - 1;
        p.slot = g.slot_nbr[p.slot * 8 + 2 * mu + 1];
    }
    return p;
}
__device__ __forceinline__ M3 link(const Geo &g, const double2 *U, const Pos &p, int mu)
{
    M3 u;
    load_link<double>(U, p.slot, mu, g.Vb, g.loc_index[lexi(g, p.x[0], p.x[1], p.x[2], p.x[3])], u);
    return u;
}

// planes 0..5 = (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
__global__ __launch_bounds__(256) void k_clover_planes(Geo g, const double2 *__restrict__ U, double2 *__restrict__ F)
{
    const long V = g.V;
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= 6 * V) return;
    const int p = (int)(t / V);
    const long site = t - p * V;  // internal order: slot * Vb + l
    const int mu = p < 3 ? 0 : p < 5 ? 1 : 2;
    const int nu = p < 3 ? p + 1 : p < 5 ? p - 1 : 3;
    Pos x;
    x.slot = (int)(site / g.Vb);
    local_coords(g, (int)(site % g.Vb), x.x);
    const Pos xm = moved(g, x, mu, 1), xn = moved(g, x, nu, 1), xbm = moved(g, x, mu, -1), xbn = moved(g, x, nu, -1);
    const Pos xbm_n = moved(g, xbm, nu, 1), xbm_bn = moved(g, xbm, nu, -1), xm_bn = moved(g, xm, nu, -1);
    // x -> x+mu -> x+mu+nu -> x+nu -> x
    M3 Q = mmd(mmd(mm(link(g, U, x, mu), link(g, U, xm, nu)), link(g, U, xn, mu)), link(g, U, x, nu));
    // x -> x+nu -> x-mu+nu -> x-mu -> x
    const M3 q2 = mm(mmd(mmd(link(g, U, x, nu), link(g, U, xbm_n, mu)), link(g, U, xbm, nu)), link(g, U, xbm, mu));
    // x -> x-mu -> x-mu-nu -> x-nu -> x
    const M3 q3 = mm(mdm(mm(link(g, U, xbm_bn, nu), link(g, U, xbm, mu)), link(g, U, xbm_bn, mu)),
                     link(g, U, xbn, nu));
    // x -> x-nu -> x+mu-nu -> x+mu -> x
    const M3 q4 = mmd(mm(mdm(link(g, U, xbn, nu), link(g, U, xbn, mu)), link(g, U, xm_bn, nu)), link(g, U, x, mu));
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Q.m[i][j] = Q.m[i][j] + q2.m[i][j] + q3.m[i][j] + q4.m[i][j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const cx<double> f = scale(0.125, Q.m[i][j] - mk(Q.m[j][i].re, -Q.m[j][i].im));
            st<double>(F, (long)(p * 9 + 3 * i + j) * V + site, f);
        }
}

// the block of A for one (site, chirality), its LDL^H factorisation (no
// pivoting: A is hermitian and close to 1) and A^-1; worst[t] = the largest
// 1 / |pivot| of the factorisation
__global__ __launch_bounds__(256) void k_clover_blocks(Geo g, const double2 *__restrict__ F, double c,
                                                       double *__restrict__ A, double *__restrict__ worst)
{
    const long V = g.V;
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= 2 * V) return;
    const int chi = (int)(t / V);
    const long site = t - chi * V;
    const int slot = (int)(site / g.Vb), l = (int)(site % g.Vb), Vb = g.Vb;
    const double e = chi ? -1.0 : 1.0;
    auto f = [&](int p, int k) { return ld<double>(F, (long)(p * 9 + k) * V + site); };
    cx<double> M[6][6];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int k = 3 * a + b;
            const cx<double> G1 = scale(-1.0, f(3, k)) + scale(e, f(2, k));
            const cx<double> G2 = f(1, k) + scale(e, f(4, k));
            const cx<double> G3 = scale(-1.0, f(0, k)) + scale(e, f(5, k));
            const cx<double> t3 = mul_i(scale(c, G3));
            const double one = a == b ? 1.0 : 0.0;
            M[a][b] = mk(one, 0.0) + t3;
            M[3 + a][3 + b] = mk(one, 0.0) - t3;
            M[a][3 + b] = mul_i(scale(c, G1)) + scale(c, G2);
        }
    double *out = A + ((long)slot * 2 + chi) * 36 * Vb + l;
#pragma unroll
    for (int i = 0; i < 6; ++i) out[(long)i * Vb] = M[i][i].re;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i + 1; j < 6; ++j) {
            const int k = herm_k(i, j);
            out[(long)(6 + 2 * k) * Vb] = M[i][j].re;
            out[(long)(7 + 2 * k) * Vb] = M[i][j].im;
        }
    // A = L D L^+ with L unit lower triangular (stored below the diagonal of M)
    double d[6], bad = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double dj = M[j][j].re;
#pragma unroll
        for (int k = 0; k < j; ++k) dj -= (M[j][k].re * M[j][k].re + M[j][k].im * M[j][k].im) * d[k];
        d[j] = dj;
        const double inv = 1.0 / fabs(dj);
        bad = (inv > bad || inv != inv) ? inv : bad;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            cx<double> s = mk(M[j][i].re, -M[j][i].im);  // A_ij = conj(A_ji)
#pragma unroll
            for (int k = 0; k < j; ++k) s = s - scale(d[k], M[i][k] * mk(M[j][k].re, -M[j][k].im));
            M[i][j] = scale(1.0 / dj, s);
        }
    }
    worst[t] = bad;
    // W = L^-1 (unit lower triangular), then A^-1 = W^+ D^-1 W
    cx<double> W[6][6];
#pragma unroll
    for (int j = 0; j < 6; ++j)
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            cx<double> s = M[i][j];
#pragma unroll
            for (int k = j + 1; k < i; ++k) s = s + M[i][k] * W[k][j];
            W[i][j] = scale(-1.0, s);
        }
    double *oinv = out + 72 * V;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i; j < 6; ++j) {
            cx<double> s = mk(0.0, 0.0);
#pragma unroll
            for (int k = j; k < 6; ++k) {
                const cx<double> wki = k == i ? mk(1.0, 0.0) : W[k][i];
                const cx<double> wkj = k == j ? mk(1.0, 0.0) : W[k][j];
                s = s + scale(1.0 / d[k], conjmul(wki, wkj));
            }
            if (i == j) {
                oinv[(long)i * Vb] = s.re;
            } else {
                const int k = herm_k(i, j);
                oinv[(long)(6 + 2 * k) * Vb] = s.re;
                oinv[(long)(7 + 2 * k) * Vb] = s.im;
            }
        }
}

// out[blockIdx.x] = max over a grid-strided share of in[0 .. n) (a nan wins)
__global__ __launch_bounds__(256) void k_maxred(long n, const double *__restrict__ in, double *__restrict__ out)
{
    __shared__ double sh[256];
    double m = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const double v = in[i];
        m = (v > m || v != v) ? v : m;
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double v = sh[threadIdx.x + w], a = sh[threadIdx.x];
            sh[threadIdx.x] = (v > a || v != v) ? v : a;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_to_f32(long n, const double *__restrict__ in, float *__restrict__ out)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

template <typename T>
__global__ __launch_bounds__(256) void k_clover_mul(Geo g, const int32_t *__restrict__ active,
                                                    const int32_t *__restrict__ list, const T *const *__restrict__ ctab,
                                                    long n, int inv, int par, const T2<T> *__restrict__ in,
                                                    T2<T> *__restrict__ out)
{
    const int m = sys_at(list, blockIdx.z);
    if (active && !active[m]) return;
    const int Vb = g.Vb;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= (par < 0 ? Vb : g.Vh)) return;
    const int l = (par > 0 ? g.Vh : 0) + i, slot = blockIdx.y;
    const long base = m * n + (long)slot * 12 * Vb + l;
#pragma unroll
    for (int chi = 0; chi < 2; ++chi) {
        cx<T> x[6], y[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) x[k] = ld<T>(in, base + (long)(6 * chi + k) * Vb);
        clov_mul6<T>(clov_at<T>(ctab[m], (long)g.V, inv, slot, chi, Vb, l), Vb, x, y);
#pragma unroll
        for (int k = 0; k < 6; ++k) st<T>(out, base + (long)(6 * chi + k) * Vb, y[k]);
    }
}

__global__ __launch_bounds__(256) void k_clover_canon(Geo g, const double *__restrict__ c64, int inv,
                                                      double2 *__restrict__ canon)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const int slot = blockIdx.y;
    int x[4];
    double2 *o = canon + canon_index(g, slot, l, x) * 144;
    for (int k = 0; k < 144; ++k) o[k] = make_double2(0.0, 0.0);
    for (int chi = 0; chi < 2; ++chi) {
        const auto *p = clov_at<double>(c64, (long)g.V, inv, slot, chi, g.Vb, l);
        for (int i = 0; i < 6; ++i) {
            const int r = 6 * chi + i;
            o[r * 12 + r] = make_double2(p[(long)i * g.Vb], 0.0);
            for (int j = i + 1; j < 6; ++j) {
                const int k = herm_k(i, j), q = 6 * chi + j;
                const double re = p[(long)(6 + 2 * k) * g.Vb], im = p[(long)(7 + 2 * k) * g.Vb];
                o[r * 12 + q] = make_double2(re, im);
                o[q * 12 + r] = make_double2(re, -im);
            }
        }
    }
}

unsigned nb256(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

size_t clover_work_bytes(const Geo &g)
{
    return (size_t)g.V * 54 * sizeof(double2) + (size_t)g.V * 2 * sizeof(double) + 256 * sizeof(double);
}

void launch_clover_build(const Geo &g, const double2 *U, double csw, double kappa, void *work, double *c64, float *c32,
                         double *worst, hipStream_t s)
{
    const long V = g.V;
    double2 *F = static_cast<double2 *>(work);
    double *w = reinterpret_cast<double *>(F + 54 * V), *part = w + 2 * V;
    k_clover_planes<<<nb256(6 * V), 256, 0, s>>>(g, U, F);
    k_clover_blocks<<<nb256(2 * V), 256, 0, s>>>(g, F, csw * kappa, c64, w);
    const int nbr = (int)std::min<long>(256, nb256(2 * V));
    k_maxred<<<nbr, 256, 0, s>>>(2 * V, w, part);
    k_maxred<<<1, 256, 0, s>>>(nbr, part, worst);
    if (c32) k_to_f32<<<nb256(144 * V), 256, 0, s>>>(144 * V, c64, c32);
}

template <typename T>
void launch_clover_mul(const Geo &g, const Sys &sy, const T *const *ctab, int inv, int par, const T2<T> *in,
                       T2<T> *out, hipStream_t s)
{
    if (sy.M <= 0) return;
    const int nloc = par < 0 ? g.Vb : g.Vh;
    k_clover_mul<T><<<dim3((nloc + 255) / 256, g.nblk, sy.launch_m()), 256, 0, s>>>(g, sy.active, sy.list, ctab, sy.n,
                                                                                    inv, par, in, out);
}
template void launch_clover_mul<double>(const Geo &, const Sys &, const double *const *, int, int, const double2 *,
                                        double2 *, hipStream_t);
template void launch_clover_mul<float>(const Geo &, const Sys &, const float *const *, int, int, const float2 *,
                                       float2 *, hipStream_t);

void launch_clover_canon(const Geo &g, const double *c64, int inv, double2 *canon, hipStream_t s)
{
    k_clover_canon<<<dim3((g.Vb + 255) / 256, g.nblk), 256, 0, s>>>(g, c64, inv, canon);
}

}  // namespace wdr
