// Exact block determinants for gfx950 (paper Sec. 3, eq. ddfactor: the
// block factors det D_b; their ratios between U' and U decide the first
// acceptance step of eq. 4step, where blocks are small enough for an exact
// factorisation).
//
// With the even-odd reduction inside a Dirichlet block, det D_b = det Dhat_b,
// Dhat_b = 1 - k^2 H_eo H_oe (in-block hops only); with a clover term
// det D_b = det A_oo det Dhat_b, Dhat_b = A_ee - k^2 H_eo A_oo^-1 H_oe, and
// log det A_oo (the odd sites' 6 x 6 blocks) is added separately.  The
// normal matrix
//     A_b = Dhat_b^+ Dhat_b = g5 Dhat_b g5 Dhat_b        (n = 6 Vb rows)
// is Hermitian positive definite, so
//     log det(D_b^+ D_b) = log det A_b = 2 sum_i log L_ii,   A_b = L L^+.
// The Cholesky factorisation needs no pivoting and half the flops of an LU
// of Dhat_b.
//
//  1. k_normal: a workgroup (one lane per site) per block and range of
//     columns; column (j, c) of A_b is g5 Dhat g5 Dhat e_(j,c), applied in
//     LDS, where each stage only computes the sites that the unit vector
//     can reach by then.  A_b is Hermitian, so the column is stored
//     conjugated as a row.  Rows and columns are padded to a multiple of 64
//     with the identity (k_pad), which leaves the determinant unchanged.
//  2. Right-looking blocked Cholesky with 64-wide panels, batched over
//     blocks: k_potrf_tile factors the diagonal tile in LDS and builds
//     W = L_pp^-1 with the same elimination steps; k_tile_gemm<0> forms the
//     panel L_Ip = A_Ip W^+; k_tile_gemm<1> the updates A_IJ -= L_Ip L_Jp^+
//     (I >= J), on FP64 MFMA 16x16x4 with four real products per complex
//     one.  Panels come in groups of GROUP: after each panel only the rest
//     of its group is updated, and the tiles right of the group take one
//     update with k = 64 GROUP, so the trailing matrix is read and written
//     once per group instead of once per panel.  Only the lower triangle is
//     ever read.
#include <algorithm>
#include <cmath>

#include "clover.h"
#include "lds_stencil.h"
#include "runtime.h"

namespace wdr {
namespace {

using namespace dev;

constexpr int TW = 64;   // tile and panel width
constexpr int KC = 16;   // k-chunk staged in LDS by the tile GEMM
constexpr int GROUP = 4; // panels per trailing update
constexpr int MAX_VH = 128;

__device__ __forceinline__ void unpack_coords(uint32_t v, int x[4])
{
    x[0] = v & 255;
    x[1] = (v >> 8) & 255;
    x[2] = (v >> 16) & 255;
    x[3] = v >> 24;
}

// Matrix q of a launch is (field q / nblk, slot q % nblk) with global index
// q0 + blockIdx.y; its rows start at A + blockIdx.y * np * np.  C0 / C1:
// the fields' clover terms (A, then A^-1; NULL without one).
__global__ __launch_bounds__(256) void k_normal(Geo g, const double2 *__restrict__ U0, const double2 *__restrict__ U1,
                                                const double *__restrict__ C0, const double *__restrict__ C1,
                                                int q0, int cols, double kappa, long np, double2 *__restrict__ A)
{
    __shared__ double2 she[12 * MAX_VH], sho[12 * MAX_VH];
    const int q = q0 + blockIdx.y, slot = q % g.nblk;
    const double2 *U = q / g.nblk ? U1 : U0;
    const double *C = q / g.nblk ? C1 : C0;
    double2 *Aq = A + (long)blockIdx.y * np * np;
    const int Vh = g.Vh, n = 6 * g.Vb, l = threadIdx.x;
    const bool even = l < Vh;
    const double k2 = kappa * kappa;
    int x[4];
    unpack_coords(g.loc_coord[l], x);
    const LdsLoader<double> from_e{she, Vh, 0}, from_o{sho, Vh, Vh};
    const int c0 = blockIdx.x * cols, c1 = min(n, c0 + cols);
    for (int col = c0; col < c1; ++col) {
        const int j = col / 12, cc = col % 12;
        int xj[4];
        unpack_coords(g.loc_coord[j], xj);
        const int dist = abs(x[0] - xj[0]) + abs(x[1] - xj[1]) + abs(x[2] - xj[2]) + abs(x[3] - xj[3]);
        spinor<double> acc;
        if (even)
            for (int k = 0; k < 12; ++k) she[k * Vh + l] = make_double2(l == j && k == cc ? 1.0 : 0.0, 0.0);
        __syncthreads();
        // odd sites: H_oe e (reaches distance 1), then H_oe of the even
        // stage-2 field (distance 3)
        // even sites: g5 (x - k^2 H_eo t) (distance 2, then 4)
        for (int stage = 1; stage <= 4; ++stage) {
            const bool odd_stage = stage & 1;
            if (odd_stage && !even) {
                zero(acc);
                if (dist <= stage) {
                    hop_sum<double, HOPS_IN>(g, U, slot, l, x, from_e, acc);
                    if (C) clov_spinor<double>(C, g.V, 1, slot, g.Vb, l, acc);  // A_oo^-1 H_oe
                }
#pragma unroll
                for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                    for (int a = 0; a < 3; ++a) st<double>(sho, (long)(3 * sp + a) * Vh + l - Vh, acc.s[sp].c[a]);
            } else if (!odd_stage && even) {
                zero(acc);
                if (dist <= stage) hop_sum<double, HOPS_IN>(g, U, slot, l, x, from_o, acc);
                // the diagonal term: the input, or A_ee times it (the input
                // reaches distance 0 at stage 2, 2 at stage 4)
                spinor<double> dg;
                LdsLoader<double>{she, Vh, 0}(0, l, dg);
                if (C && dist <= stage - 2) clov_spinor<double>(C, g.V, 0, slot, g.Vb, l, dg);
#pragma unroll
                for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const long i = (long)(3 * sp + a) * Vh + l;
                        cx<double> v = dg.s[sp].c[a] - scale(k2, acc.s[sp].c[a]);
                        if (sp >= 2) v = neg(v);
                        if (stage == 2) {
                            st<double>(she, i, v);
                        } else {
                            // column col of A is row col conjugated
                            Aq[(long)col * np + 12 * l + 3 * sp + a] = make_double2(v.re, -v.im);
                        }
                    }
            }
            __syncthreads();
        }
    }
}

// The same for B^4 blocks of SU(3) links, with the links staged in LDS and
// the geometry known at compile time.  Every stage keeps all four
// wavefronts busy: for output site t of the stage's parity, lane t of the
// first half (t < Vh) sums the hops in directions 0 and 1 and lane Vh + t
// those in directions 2 and 3.  The two partial sums meet in the half field
// that the stage does not read: the output half of an odd stage, the input
// half of an even stage once both partial sums are done.
template <int B>
__global__ __launch_bounds__(Cube<B>::Vb) void k_normal_cube(int nblk, const double2 *__restrict__ U0,
                                                             const double2 *__restrict__ U1, int q0, int cols,
                                                             double kappa, long np, double2 *__restrict__ A)
{
    typedef Cube<B> CB;
    constexpr int Vb = CB::Vb, Vh = CB::Vh, n = 6 * Vb;
    __shared__ CubeLds<double, B> S;
    const int q = q0 + blockIdx.y, slot = q % nblk;
    const auto *Ug = as_global(q / nblk ? U1 : U0);
    double2 *Aq = A + (long)blockIdx.y * np * np;
    const int tid = threadIdx.x, t = tid % Vh, mu0 = tid < Vh ? 0 : 2;
    const bool first = tid < Vh;
    const double k2 = kappa * kappa;
    // output sites of this lane: even site t and odd site Vh + t
    int xe[4], xo[4];
    CB::coords(t, xe);
    CB::coords(Vh + t, xo);
    {
        const long base = (long)slot * 4 * 9 * Vb + tid;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int e = 0; e < 6; ++e)
                st<double>(S.lk, (mu * 6 + e) * Vb + tid, ldg<double>(Ug, base + (long)(mu * 9 + e) * Vb));
    }
    const int c0 = blockIdx.x * cols, c1 = min(n, c0 + cols);
    for (int col = c0; col < c1; ++col) {
        const int j = col / 12, cc = col % 12;
        int xj[4];
        CB::coords(j, xj);
        int de = 0, dn = 0;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            de += abs(xe[mu] - xj[mu]);
            dn += abs(xo[mu] - xj[mu]);
        }
        spinor<double> acc;
        if (first)
            for (int k = 0; k < 12; ++k) S.she[k * Vh + t] = make_double2(t == j && k == cc ? 1.0 : 0.0, 0.0);
        __syncthreads();
        for (int stage = 1; stage <= 4; ++stage) {
            zero(acc);
            if (stage & 1) {
                // odd sites: H_oe of the even half (reaches distance 1, then 3)
                if (dn <= stage)
                    for (int mu = mu0; mu < mu0 + 2; ++mu) hop_dir_lds_rt<double, B>(mu, S.she, 0, S.lk, Vh + t, xo, acc);
                if (first) lds_store<double>(S.sho, Vh, t, acc);
                __syncthreads();
                if (!first) {
#pragma unroll
                    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            const long i = (long)(3 * sp + a) * Vh + t;
                            st<double>(S.sho, i, ld<double>(S.sho, i) + acc.s[sp].c[a]);
                        }
                }
            } else {
                // even sites: g5 (x - k^2 H_eo t) (distance 2, then 4)
                if (de <= stage)
                    for (int mu = mu0; mu < mu0 + 2; ++mu) hop_dir_lds_rt<double, B>(mu, S.sho, Vh, S.lk, t, xe, acc);
                __syncthreads();
                if (!first) lds_store<double>(S.sho, Vh, t, acc);
                __syncthreads();
                if (first) {
#pragma unroll
                    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            const long i = (long)(3 * sp + a) * Vh + t;
                            cx<double> v = ld<double>(S.she, i) - scale(k2, acc.s[sp].c[a] + ld<double>(S.sho, i));
                            if (sp >= 2) v = neg(v);
                            if (stage == 2) st<double>(S.she, i, v);
                            else Aq[(long)col * np + 12 * t + 3 * sp + a] = make_double2(v.re, -v.im);
                        }
                }
            }
            __syncthreads();
        }
    }
}

// out[f * nblk + slot] = sum over the block's odd sites of log |det A(x)|
// (both 6 x 6 blocks), field f = blockIdx.y (C0, C1); elimination without
// pivoting on the Hermitian block (its pivots are real)
__global__ __launch_bounds__(256) void k_clover_logdet_odd(Geo g, const double *__restrict__ C0,
                                                           const double *__restrict__ C1, double *__restrict__ out)
{
    __shared__ double red[4];
    const int slot = blockIdx.x, f = blockIdx.y;
    const double *C = f ? C1 : C0;
    double s = 0;
    for (int i = threadIdx.x; i < 2 * g.Vh; i += 256) {
        const int l = g.Vh + i / 2, chi = i % 2;
        const auto *p = clov_at<double>(C, (long)g.V, 0, slot, chi, g.Vb, l);
        cx<double> a[6][6];
#pragma unroll
        for (int r = 0; r < 6; ++r) a[r][r] = mk<double>(p[(long)r * g.Vb], 0.0);
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = r + 1; c < 6; ++c) {
                const int k = herm_k(r, c);
                a[r][c] = mk<double>(p[(long)(6 + 2 * k) * g.Vb], p[(long)(7 + 2 * k) * g.Vb]);
                a[c][r] = mk<double>(a[r][c].re, -a[r][c].im);
            }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double d = a[k][k].re;
            s += log(fabs(d));
#pragma unroll
            for (int r = k + 1; r < 6; ++r) {
                const cx<double> m = scale(1.0 / d, a[r][k]);
#pragma unroll
                for (int c = k + 1; c < 6; ++c) a[r][c] = a[r][c] - m * a[k][c];
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[(long)f * g.nblk + slot] = (red[0] + red[1]) + (red[2] + red[3]);
}

// rows n .. np-1 of every matrix: the identity
__global__ __launch_bounds__(256) void k_pad(long n, long np, double2 *__restrict__ A)
{
    double2 *Aq = A + (long)blockIdx.y * np * np;
    const long total = (np - n) * np;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
        const long r = n + i / np, c = i % np;
        Aq[r * np + c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
    }
}

__global__ void k_fill_ld(int nm, double *ld, int32_t *bad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nm) {
        ld[i] = 0.0;
        bad[i] = 0;
    }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmul_conj(double2 a, double2 b)  // a * conj(b)
{
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// Cholesky of the diagonal tile p of every matrix.  Lane (u, v) = (tid / 16,
// tid % 16) keeps entries (u + 16 a, v + 16 b), a, b < 4, of the tile and of
// W in registers.  Step k: the owner of entry (k, k) publishes d = L_kk; the
// owners of column k publish L_ik = A_ik / d and those of row k of W scale
// it by 1 / d and publish it; then every lane updates its entries,
// A_ij -= L_ik conj(L_jk) and W_ic -= L_ik W_kc (i, j > k), so that W ends
// as L^-1.  Adds 2 sum_k log L_kk to ld[q]; sets bad[q] on a pivot that is
// not positive.
__global__ __launch_bounds__(256) void k_potrf_tile(double2 *__restrict__ A, long np, int p, int q0,
                                                    double2 *__restrict__ W, double *__restrict__ ld,
                                                    int32_t *__restrict__ bad)
{
    __shared__ double2 colk[TW], rowk[TW];
    __shared__ double dsh, lsh[16];
    __shared__ int badsh;
    const int tid = threadIdx.x, u = tid >> 4, v = tid & 15;
    const double2 *T = A + (long)blockIdx.x * np * np + (long)TW * p * np + TW * p;
    double2 a[4][4], w[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int r = u + 16 * x, c = v + 16 * y;
            a[x][y] = c <= r ? T[(long)r * np + c] : make_double2(0.0, 0.0);
            w[x][y] = make_double2(r == c ? 1.0 : 0.0, 0.0);
        }
    if (tid == 0) badsh = 0;
    double lsum = 0.0;
    // k = 16 kx + ku; with kx known at compile time the register arrays are
    // indexed statically and the entries that no longer change are skipped:
    // rows and columns of A below 16 kx + ku are final, and row k of W has
    // nothing right of column k
#pragma unroll
    for (int kx = 0; kx < 4; ++kx) {
        for (int ku = 0; ku < 16; ++ku) {
            const int k = 16 * kx + ku;
            if (u == ku && v == ku) {
                const double akk = a[kx][kx].x;
                if (!(akk > 0.0)) badsh = 1;  // also for NaN
                const double d = sqrt(fmax(akk, 1e-300));
                dsh = d;
                lsum += log(d);
            }
            __syncthreads();
            const double inv = 1.0 / dsh;
            if (v == ku) {  // column k of the tile: rows u + 16 x
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const int r = u + 16 * x;
                    colk[r] = r > k ? make_double2(a[x][kx].x * inv, a[x][kx].y * inv) : make_double2(0.0, 0.0);
                }
            }
            if (u == ku) {  // row k of W: columns v + 16 y, scaled in place
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    w[kx][y].x *= inv;
                    w[kx][y].y *= inv;
                    rowk[v + 16 * y] = w[kx][y];
                }
            }
            __syncthreads();
            double2 cr[4], cc[4], rw[4];
#pragma unroll
            for (int x = kx; x < 4; ++x) {
                cr[x] = colk[u + 16 * x];
                cc[x] = colk[v + 16 * x];
            }
#pragma unroll
            for (int y = 0; y <= kx; ++y) rw[y] = rowk[v + 16 * y];
            // colk is 0 at rows <= k, so only entries below row k change
#pragma unroll
            for (int x = kx; x < 4; ++x) {
#pragma unroll
                for (int y = kx; y < 4; ++y) {
                    const double2 t1 = cmul_conj(cr[x], cc[y]);
                    a[x][y].x -= t1.x;
                    a[x][y].y -= t1.y;
                }
#pragma unroll
                for (int y = 0; y <= kx; ++y) {
                    const double2 t2 = cmul(cr[x], rw[y]);
                    w[x][y].x -= t2.x;
                    w[x][y].y -= t2.y;
                }
            }
        }
    }
    double2 *Wq = W + (long)blockIdx.x * TW * TW;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) Wq[(u + 16 * x) * TW + v + 16 * y] = w[x][y];
    if (u == v) lsh[u] = lsum;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int i = 0; i < 16; ++i) t += lsh[i];
        ld[q0 + blockIdx.x] += 2.0 * t;
        if (badsh) bad[q0 + blockIdx.x] = 1;
    }
}

typedef double d4 __attribute__((ext_vector_type(4)));

// C = X Y^+ for 64 x 64 complex tiles, X and Y the tiles of rows I and J
// over columns [kbeg, kbeg + klen):
//   MODE 0: X = A_Ip, Y = W (L_pp^-1, klen 64), C = A_Ip in place (panel
//           solve); I = j0 + blockIdx.x
//   MODE 1: C = A_IJ - X Y^+ for the tile pairs I >= J: with nj > 0 the
//           rectangle I = i0 + x / nj, J = j0 + x % nj (pairs with I < J
//           exit), with nj = 0 the triangle I >= J >= j0 numbered row by row.
// Four wavefronts each own a 32 x 32 quadrant as 2 x 2 MFMA tiles.  MFMA
// 16x16x4 f64 operands: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16];
// element r of its accumulator is D[l / 16 + 4 r][l % 16].  Here
// B[k][n] = conj(Y[n][k]), and each complex product takes three real ones
// (the 3M form): P1 = Xr Yr, P2 = Xi Yi, P3 = (Xr + Xi)(Yr - Yi), so that
// re C = P1 + P2 and im C = P3 - P1 + P2.
template <int MODE>
__global__ __launch_bounds__(256) void k_tile_gemm(double2 *__restrict__ A, long np, int i0, int j0, int nj,
                                                   int kbeg, int klen, const double2 *__restrict__ W)
{
    __shared__ double xr[TW][KC + 1], xi[TW][KC + 1], yr[TW][KC + 1], yi[TW][KC + 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double2 *Aq = A + (long)blockIdx.y * np * np;
    int I, J;
    if (MODE == 0) {
        I = j0 + blockIdx.x;
        J = kbeg / TW;
    } else if (nj > 0) {
        I = i0 + blockIdx.x / nj;
        J = j0 + blockIdx.x % nj;
        if (I < J) return;
    } else {
        const int x = blockIdx.x;
        int ii = (int)((sqrt(8.0 * x + 1.0) - 1.0) * 0.5);
        while ((ii + 1) * (ii + 2) / 2 <= x) ++ii;
        while (ii * (ii + 1) / 2 > x) --ii;
        I = j0 + ii;
        J = j0 + (x - ii * (ii + 1) / 2);
    }
    const double2 *X = Aq + (long)TW * I * np + kbeg;
    const double2 *Y = MODE == 0 ? W + (long)blockIdx.y * TW * TW : Aq + (long)TW * J * np + kbeg;
    const long ys = MODE == 0 ? TW : np;
    const int r0 = 32 * (wv >> 1), c0 = 32 * (wv & 1), m = lane & 15, kl = lane >> 4;
    d4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) p1[a][b] = p2[a][b] = p3[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    // the next k-chunk is loaded into registers while this one is computed
    constexpr int PER = TW * KC / 256;
    double2 nx[PER], ny[PER];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = tid + 256 * q, r = i / KC, k = i % KC;
            nx[q] = X[(long)r * np + kc + k];
            ny[q] = Y[(long)r * ys + kc + k];
        }
    };
    fetch(0);
    for (int kc = 0; kc < klen; kc += KC) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = tid + 256 * q, r = i / KC, k = i % KC;
            xr[r][k] = nx[q].x;
            xi[r][k] = nx[q].y;
            yr[r][k] = ny[q].x;
            yi[r][k] = ny[q].y;
        }
        __syncthreads();
        if (kc + KC < klen) fetch(kc + KC);
#pragma unroll 2
        for (int k = 0; k < KC; k += 4) {
            double ar[2], ai[2], br[2], bi[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                ar[t] = xr[r0 + 16 * t + m][k + kl];
                ai[t] = xi[r0 + 16 * t + m][k + kl];
                br[t] = yr[c0 + 16 * t + m][k + kl];
                bi[t] = yi[c0 + 16 * t + m][k + kl];
            }
            double as[2], bd[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                as[t] = ar[t] + ai[t];
                bd[t] = br[t] - bi[t];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    p1[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], p1[a][b], 0, 0, 0);
                    p2[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], bi[b], p2[a][b], 0, 0, 0);
                    p3[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[a], bd[b], p3[a][b], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    double2 *C = Aq + (long)TW * I * np + TW * J;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long idx = (long)(r0 + 16 * a + kl + 4 * r) * np + c0 + 16 * b + m;
                const double re = p1[a][b][r] + p2[a][b][r], im = p3[a][b][r] - p1[a][b][r] + p2[a][b][r];
                if (MODE == 0) {
                    C[idx] = make_double2(re, im);
                } else {
                    const double2 o = C[idx];
                    C[idx] = make_double2(o.x - re, o.y - im);
                }
            }
}

}  // namespace

// FP64 workspace for the normal matrices of one pass (the batch of blocks is
// cut into passes of at most this size)
constexpr size_t BLOCKDET_WORKSPACE = 8ull << 30;

wdr_status block_logdet(wdr_ctx *c, const wdr_gauge *U0, const wdr_gauge *U1, double kappa, int max_blocks,
                        double *out, hipStream_t s)
{
    const Geo &g = c->g;
    const int nf = U1 ? 2 : 1, nm = nf * g.nblk;
    const long n = 6L * g.Vb, np = (n + TW - 1) / TW * TW, T = np / TW;
    const size_t mat_bytes = (size_t)np * np * sizeof(double2);
    size_t fit = std::max<size_t>(1, std::min<size_t>(nm, BLOCKDET_WORKSPACE / mat_bytes));
    if (max_blocks > 0) fit = std::min<size_t>(fit, max_blocks);
    const int per_pass = (int)fit;
    Work aw(c, mat_bytes * per_pass), ww(c, sizeof(double2) * TW * TW * per_pass), lw(c, sizeof(double) * nm),
        bw(c, sizeof(int32_t) * nm);
    if (!aw.ok() || !ww.ok() || !lw.ok() || !bw.ok()) return WDR_ENOMEM;
    double2 *A = aw.as<double2>(), *W = ww.as<double2>();
    double *ld = lw.as<double>();
    int32_t *bad = bw.as<int32_t>();
    k_fill_ld<<<(nm + 255) / 256, 256, 0, s>>>(nm, ld, bad);
    // about 2048 workgroups per pass for the normal-matrix columns
    const int cols = (int)std::max<long>(12, (n * per_pass + 2047) / 2048);
    const int ncg = (int)((n + cols - 1) / cols);
    // SU(3) links of 4^4 blocks: links in LDS, compile-time geometry
    // (the clover operator takes the general form)
    const bool clov = U0->c64 != nullptr;
    const bool cube4 = g.B[0] == 4 && g.B[1] == 4 && g.B[2] == 4 && g.B[3] == 4 && U0->su3 && (!U1 || U1->su3) && !clov;
    const double *C0 = U0->c64, *C1 = U1 ? U1->c64 : U0->c64;
    for (int q0 = 0; q0 < nm; q0 += per_pass) {
        const int m = std::min(per_pass, nm - q0);
        if (cube4)
            k_normal_cube<4><<<dim3(ncg, m), 256, 0, s>>>(g.nblk, U0->u64, U1 ? U1->u64 : U0->u64, q0, cols, kappa,
                                                          np, A);
        else
            k_normal<<<dim3(ncg, m), g.Vb, 0, s>>>(g, U0->u64, U1 ? U1->u64 : U0->u64, C0, C1, q0, cols, kappa, np, A);
        if (np > n) k_pad<<<dim3((unsigned)std::min<long>(64, ((np - n) * np + 255) / 256), m), 256, 0, s>>>(n, np, A);
        // panels in groups of GROUP: each panel updates only the rest of its
        // group; the tiles right of the group get one update per group
        for (int g0 = 0; g0 < T; g0 += GROUP) {
            const int g1 = (int)std::min<long>(T, g0 + GROUP);
            for (int p = g0; p < g1; ++p) {
                k_potrf_tile<<<m, 256, 0, s>>>(A, np, p, q0, W, ld, bad);
                if (p + 1 < T) k_tile_gemm<0><<<dim3((unsigned)(T - 1 - p), m), 256, 0, s>>>(A, np, 0, p + 1, 0, TW * p, TW, W);
                if (p + 1 < g1) {
                    const int nj = g1 - p - 1;
                    k_tile_gemm<1><<<dim3((unsigned)((T - p - 1) * nj), m), 256, 0, s>>>(A, np, p + 1, p + 1, nj, TW * p,
                                                                                         TW, W);
                }
            }
            const int rest = (int)(T - g1);
            if (rest > 0)
                k_tile_gemm<1><<<dim3(rest * (rest + 1) / 2, m), 256, 0, s>>>(A, np, g1, g1, 0, TW * g0,
                                                                               TW * (g1 - g0), W);
        }
    }
    WDR_HIP(hipGetLastError());
    std::vector<double> hl(nm), hc(nm, 0.0);
    std::vector<int32_t> hb(nm);
    if (clov) {  // log |det A_oo| per block: det D_b = det A_oo det Dhat_b
        Work cw(c, sizeof(double) * nm);
        if (!cw.ok()) return WDR_ENOMEM;
        k_clover_logdet_odd<<<dim3(g.nblk, nf), 256, 0, s>>>(g, C0, C1, cw.as<double>());
        WDR_HIP(hipMemcpyAsync(hc.data(), cw.as<double>(), sizeof(double) * nm, hipMemcpyDeviceToHost, s));
        WDR_HIP(hipStreamSynchronize(s));
    }
    WDR_HIP(hipMemcpyAsync(hl.data(), ld, sizeof(double) * nm, hipMemcpyDeviceToHost, s));
    WDR_HIP(hipMemcpyAsync(hb.data(), bad, sizeof(int32_t) * nm, hipMemcpyDeviceToHost, s));
    WDR_HIP(hipStreamSynchronize(s));
    int nbad = 0;
    for (int f = 0; f < nf; ++f)
        for (int b = 0; b < g.nblk; ++b) {
            const int q = f * g.nblk + c->slot_of_block[b];
            out[f * g.nblk + b] = hb[q] ? NAN : hl[q] + 2.0 * hc[q];
            nbad += hb[q] != 0;
        }
    if (nbad) {
        set_error(std::to_string(nbad) + " block normal matrices met a non-positive Cholesky pivot in FP64");
        return WDR_ENOCONV;
    }
    return WDR_OK;
}

}  // namespace wdr
