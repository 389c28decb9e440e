// Exact block determinants for gfx950 (paper Sec. 3, eq. ddfactor: the
// block factors det D_b; their ratios between U' and U decide the first
// acceptance step of eq. 4step, where blocks are small enough for an exact
// factorisation).
//
// With the even-odd reduction inside a Dirichlet block, det D_b = det Dhat_b,
// Dhat_b = 1 - k^2 H_eo H_oe (in-block hops only), and the normal matrix
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
//     panel L_Ip = A_Ip W^+; k_tile_gemm<1> the trailing update
//     A_IJ -= L_Ip L_Jp^+ (I >= J), on FP64 MFMA 16x16x4 with four real
//     products per complex one.  Only the lower triangle is ever read.
#include <algorithm>
#include <cmath>

#include "runtime.h"
#include "stencil.h"

namespace wdr {
namespace {

using namespace dev;

constexpr int TW = 64;   // tile and panel width
constexpr int KC = 32;   // k-chunk staged in LDS by the tile GEMM
constexpr int MAX_VH = 128;

// in-block neighbours from an LDS half field [12][Vh]; `off` is subtracted
// from the local index (0 for even sites, Vh for odd ones)
struct HalfLd {
    const double2 *sh;
    int Vh, off;
    __device__ __forceinline__ void operator()(int, int nl, spinor<double> &p) const
    {
        const int i = nl - off;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) p.s[sp].c[a] = ld<double>(sh, (long)(3 * sp + a) * Vh + i);
    }
};

__device__ __forceinline__ void unpack_coords(uint32_t v, int x[4])
{
    x[0] = v & 255;
    x[1] = (v >> 8) & 255;
    x[2] = (v >> 16) & 255;
    x[3] = v >> 24;
}

// Matrix q of a launch is (field q / nblk, slot q % nblk) with global index
// q0 + blockIdx.y; its rows start at A + blockIdx.y * np * np.
__global__ __launch_bounds__(256) void k_normal(Geo g, const double2 *__restrict__ U0, const double2 *__restrict__ U1,
                                                int q0, int cols, double kappa, long np, double2 *__restrict__ A)
{
    __shared__ double2 she[12 * MAX_VH], sho[12 * MAX_VH];
    const int q = q0 + blockIdx.y, slot = q % g.nblk;
    const double2 *U = q / g.nblk ? U1 : U0;
    double2 *Aq = A + (long)blockIdx.y * np * np;
    const int Vh = g.Vh, n = 6 * g.Vb, l = threadIdx.x;
    const bool even = l < Vh;
    const double k2 = kappa * kappa;
    int x[4];
    unpack_coords(g.loc_coord[l], x);
    const HalfLd from_e{she, Vh, 0}, from_o{sho, Vh, Vh};
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
                if (dist <= stage) hop_sum<double, HOPS_IN>(g, U, slot, l, x, from_e, acc);
#pragma unroll
                for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                    for (int a = 0; a < 3; ++a) st<double>(sho, (long)(3 * sp + a) * Vh + l - Vh, acc.s[sp].c[a]);
            } else if (!odd_stage && even) {
                zero(acc);
                if (dist <= stage) hop_sum<double, HOPS_IN>(g, U, slot, l, x, from_o, acc);
#pragma unroll
                for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const long i = (long)(3 * sp + a) * Vh + l;
                        cx<double> v = ld<double>(she, i) - scale(k2, acc.s[sp].c[a]);
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

// Cholesky of the diagonal tile p of every matrix, in LDS.  Step k scales
// column k by 1 / L_kk and updates the trailing lower triangle; the same
// row operations turn W = 1 into L^-1.  Adds 2 sum_k log L_kk to ld[q] and
// sets bad[q] on a pivot that is not positive.
__global__ __launch_bounds__(256) void k_potrf_tile(double2 *__restrict__ A, long np, int p, int q0,
                                                    double2 *__restrict__ W, double *__restrict__ ld,
                                                    int32_t *__restrict__ bad)
{
    __shared__ double2 a[TW][TW + 1], w[TW][TW + 1];
    const int tid = threadIdx.x;
    const double2 *T = A + (long)blockIdx.x * np * np + (long)TW * p * np + TW * p;
    for (int i = tid; i < TW * TW; i += 256) {
        const int r = i / TW, c = i % TW;
        a[r][c] = c <= r ? T[(long)r * np + c] : make_double2(0.0, 0.0);
        w[r][c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    double lsum = 0.0;
    int ok = 1;
    for (int k = 0; k < TW; ++k) {
        const double akk = a[k][k].x;
        ok &= akk > 0.0;  // also false for NaN
        const double d = sqrt(fmax(akk, 1e-300)), inv = 1.0 / d;
        lsum += log(d);
        __syncthreads();
        if (tid < TW) {
            if (tid > k) {
                a[tid][k].x *= inv;
                a[tid][k].y *= inv;
            } else {
                if (tid == k) a[k][k] = make_double2(d, 0.0);
                w[k][tid].x *= inv;
                w[k][tid].y *= inv;
            }
        }
        __syncthreads();
        const int m = TW - 1 - k;
        for (int i = tid; i < m * m; i += 256) {
            const int r = k + 1 + i / m, c = k + 1 + i % m;
            if (c <= r) {
                const double2 t = cmul_conj(a[r][k], a[c][k]);
                a[r][c].x -= t.x;
                a[r][c].y -= t.y;
            }
        }
        for (int i = tid; i < m * (k + 1); i += 256) {
            const int r = k + 1 + i / (k + 1), c = i % (k + 1);
            const double2 t = cmul(a[r][k], w[k][c]);
            w[r][c].x -= t.x;
            w[r][c].y -= t.y;
        }
        __syncthreads();
    }
    double2 *Wq = W + (long)blockIdx.x * TW * TW;
    for (int i = tid; i < TW * TW; i += 256) Wq[i] = w[i / TW][i % TW];
    if (tid == 0) {
        ld[q0 + blockIdx.x] += 2.0 * lsum;
        if (!ok) bad[q0 + blockIdx.x] = 1;
    }
}

typedef double d4 __attribute__((ext_vector_type(4)));

// C = X Y^+ over 64 columns of k, for 64 x 64 complex tiles:
//   MODE 0: X = A_Ip, Y = W (L_pp^-1), C = A_Ip in place (panel solve)
//   MODE 1: X = A_Ip, Y = A_Jp, C = A_IJ - X Y^+ for the tile pair
//           (I, J), I >= J > p, numbered row by row.
// Four wavefronts each own a 32 x 32 quadrant as 2 x 2 MFMA tiles with
// separate real and imaginary accumulators.  MFMA 16x16x4 f64 operands:
// lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; element r of its
// accumulator is D[l / 16 + 4 r][l % 16].  Here
// B[k][n] = conj(Y[n][k]), so re C += Xr Yr + Xi Yi, im C += Xi Yr - Xr Yi.
template <int MODE>
__global__ __launch_bounds__(256) void k_tile_gemm(double2 *__restrict__ A, long np, int p,
                                                   const double2 *__restrict__ W)
{
    __shared__ double xr[TW][KC + 1], xi[TW][KC + 1], yr[TW][KC + 1], yi[TW][KC + 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double2 *Aq = A + (long)blockIdx.y * np * np;
    int I, J;
    if (MODE == 0) {
        I = p + 1 + blockIdx.x;
        J = p;
    } else {
        const int x = blockIdx.x;
        int ii = (int)((sqrt(8.0 * x + 1.0) - 1.0) * 0.5);
        while ((ii + 1) * (ii + 2) / 2 <= x) ++ii;
        while (ii * (ii + 1) / 2 > x) --ii;
        I = p + 1 + ii;
        J = p + 1 + (x - ii * (ii + 1) / 2);
    }
    const double2 *X = Aq + (long)TW * I * np + TW * p;
    const double2 *Y = MODE == 0 ? W + (long)blockIdx.y * TW * TW : Aq + (long)TW * J * np + TW * p;
    const long ys = MODE == 0 ? TW : np;
    const int r0 = 32 * (wv >> 1), c0 = 32 * (wv & 1), m = lane & 15, kl = lane >> 4;
    d4 cre[2][2], cim[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) cre[a][b] = cim[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    for (int kc = 0; kc < TW; kc += KC) {
        for (int i = tid; i < TW * KC; i += 256) {
            const int r = i / KC, k = i % KC;
            const double2 u = X[(long)r * np + kc + k], v = Y[(long)r * ys + kc + k];
            xr[r][k] = u.x;
            xi[r][k] = u.y;
            yr[r][k] = v.x;
            yi[r][k] = v.y;
        }
        __syncthreads();
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
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    cre[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], cre[a][b], 0, 0, 0);
                    cre[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], bi[b], cre[a][b], 0, 0, 0);
                    cim[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], br[b], cim[a][b], 0, 0, 0);
                    cim[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ar[a], bi[b], cim[a][b], 0, 0, 0);
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
                if (MODE == 0) {
                    C[idx] = make_double2(cre[a][b][r], cim[a][b][r]);
                } else {
                    const double2 o = C[idx];
                    C[idx] = make_double2(o.x - cre[a][b][r], o.y - cim[a][b][r]);
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
    for (int q0 = 0; q0 < nm; q0 += per_pass) {
        const int m = std::min(per_pass, nm - q0);
        k_normal<<<dim3(ncg, m), g.Vb, 0, s>>>(g, U0->u64, U1 ? U1->u64 : U0->u64, q0, cols, kappa, np, A);
        if (np > n) k_pad<<<dim3((unsigned)std::min<long>(64, ((np - n) * np + 255) / 256), m), 256, 0, s>>>(n, np, A);
        for (int p = 0; p < T; ++p) {
            k_potrf_tile<<<m, 256, 0, s>>>(A, np, p, q0, W, ld, bad);
            const int rest = (int)(T - 1 - p);
            if (rest > 0) {
                k_tile_gemm<0><<<dim3(rest, m), 256, 0, s>>>(A, np, p, W);
                k_tile_gemm<1><<<dim3(rest * (rest + 1) / 2, m), 256, 0, s>>>(A, np, p, W);
            }
        }
    }
    WDR_HIP(hipGetLastError());
    std::vector<double> hl(nm);
    std::vector<int32_t> hb(nm);
    WDR_HIP(hipMemcpyAsync(hl.data(), ld, sizeof(double) * nm, hipMemcpyDeviceToHost, s));
    WDR_HIP(hipMemcpyAsync(hb.data(), bad, sizeof(int32_t) * nm, hipMemcpyDeviceToHost, s));
    WDR_HIP(hipStreamSynchronize(s));
    int nbad = 0;
    for (int f = 0; f < nf; ++f)
        for (int b = 0; b < g.nblk; ++b) {
            const int q = f * g.nblk + c->slot_of_block[b];
            out[f * g.nblk + b] = hb[q] ? NAN : hl[q];
            nbad += hb[q] != 0;
        }
    if (nbad) {
        set_error(std::to_string(nbad) + " block normal matrices met a non-positive Cholesky pivot in FP64");
        return WDR_ENOCONV;
    }
    return WDR_OK;
}

}  // namespace wdr
