// Fused kernels of the solvers on 4^4 blocks, built on the block-staged
// stencil bodies (blk_stencil.h): the end of a round of the FP16 block
// solves (paper Sec. 3, the block solves inside eq. ddfactor) and the
// persistent form of the even-odd CG steps (Sec. 4, the inversions).
#include <hip/hip_cooperative_groups.h>

#include <algorithm>

#include "blk_stencil.h"

namespace wdr {
namespace {

using namespace dev;

// The end of a round of the FP16 block solves in one pass over each block
// (one workgroup per block, one lane per site): x += d (d the FP16 block-MR
// result with its block scale), r = b - D_b x in FP64 (hops inside the
// block, the new x staged in LDS), the block's |r|^2 into rn, and r in FP16
// for the next round (block scale 2^ceil(log2 max |component|), the rounding
// of k_to_h16).  The FP64 r itself is not stored.
__global__ __launch_bounds__(Cube<4>::Vb) void k_block_round16(Geo g, const int32_t *__restrict__ active,
                                                              UTab<double> Utab, const double *__restrict__ kap,
                                                              long n, const int32_t *__restrict__ sched,
                                                              const h2 *__restrict__ d16,
                                                              const float *__restrict__ dscale,
                                                              double2 *__restrict__ x, const double2 *__restrict__ b,
                                                              h2 *__restrict__ r16, float *__restrict__ rscale,
                                                              double *__restrict__ rn, double kappa)
{
    typedef Cube<4> CB;
    constexpr int Vb = CB::Vb;
    __shared__ double2 sh[12][Vb];
    __shared__ double red[Vb / 64];
    __shared__ float redm[Vb / 64];
    const int m = blockIdx.y;
    if (active && !active[m]) return;
    if (kap) kappa = kap[m];
    const int slot = sched[blockIdx.x];
    const int l = threadIdx.x;
    const auto *Ug = as_global(Utab[m]);
    const long base = m * n + (long)slot * 12 * Vb + l;
    const float ds = dscale[(long)m * g.nblk + slot];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const long i = base + (long)c * Vb;
        const h2 dv = d16[i];
        const double2 xo = x[i];
        const double2 xn = make_double2(xo.x + (double)((float)dv.x * ds), xo.y + (double)((float)dv.y * ds));
        x[i] = xn;
        sh[c][l] = xn;
    }
    int xc[4];
    CB::coords(l, xc);
    int nbr[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) nbr[k] = g.slot_nbr[slot * 8 + k];
    __syncthreads();
    spinor<double> acc;
    zero(acc);
    const auto *xg = as_global(static_cast<const double2 *>(x + m * n));  // not read: the hops stay in the block
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        int pin = 0;
        asm volatile("" : "+s"(pin));
        switch (mu) {
        case 0: hop_blk<double, 4, 0, HOPS_IN, 0, Vb>(&sh[0][0], 0, xg, Ug, slot, nbr, l, xc, pin, acc, 1.0, 1.0); break;
        case 1: hop_blk<double, 4, 1, HOPS_IN, 0, Vb>(&sh[0][0], 0, xg, Ug, slot, nbr, l, xc, pin, acc, 1.0, 1.0); break;
        case 2: hop_blk<double, 4, 2, HOPS_IN, 0, Vb>(&sh[0][0], 0, xg, Ug, slot, nbr, l, xc, pin, acc, 1.0, 1.0); break;
        default: hop_blk<double, 4, 3, HOPS_IN, 0, Vb>(&sh[0][0], 0, xg, Ug, slot, nbr, l, xc, pin, acc, 1.0, 1.0); break;
        }
    }
    cx<double> r[12];
    double nr = 0;
    float mx = 0.f;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int c = 3 * sp + a;
            const cx<double> v = ld<double>(&sh[c][0], l) - scale(kappa, acc.s[sp].c[a]);
            r[c] = ld<double>(b, base + (long)c * Vb) - v;
            nr += r[c].re * r[c].re + r[c].im * r[c].im;
            mx = fmaxf(mx, fmaxf(fabsf((float)r[c].re), fabsf((float)r[c].im)));
        }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        nr += __shfl_down(nr, off, 64);
        mx = fmaxf(mx, __shfl_down(mx, off, 64));
    }
    if ((l & 63) == 0) {
        red[l >> 6] = nr;
        redm[l >> 6] = mx;
    }
    __syncthreads();
    float bmax = redm[0];
#pragma unroll
    for (int w = 1; w < Vb / 64; ++w) bmax = fmaxf(bmax, redm[w]);
    const float rs = pow2_at_least(bmax), inv = 1.f / rs;
#pragma unroll
    for (int c = 0; c < 12; ++c) r16[base + (long)c * Vb] = to_h2(mk<float>((float)r[c].re, (float)r[c].im), inv);
    if (l == 0) {
        double tot = 0;
#pragma unroll
        for (int w = 0; w < Vb / 64; ++w) tot += red[w];
        rn[(long)m * g.nblk + slot] = tot;
        rscale[(long)m * g.nblk + slot] = rs;
    }
}

// ---------------------------------------------------------------- persistent CG steps
// The steps of the even-odd CGNE (Dhat Dhat^+ y = bh, vectors in T on the
// even sites) as one cooperative launch: each step's four stencil halves, its
// x / r update and its new search direction are phases of one grid,
// separated by grid-wide barriers instead of kernel boundaries.  A phase's
// work items are (block, system) pairs dealt round-robin to the workgroups,
// one lane per even site; the stencil halves are blk_eo_block.  Inner
// products go through one partial sum per item (|w|^2 in the second half,
// |r|^2 in the update), which every workgroup adds over the blocks of a
// system in the same order, so all workgroups hold the same scalars.  The
// control of a step (iteration count, reliable-update flag, largest residual)
// is that of k_cgm_beta, done by the workgroup holding the system's first
// block; the CG scalars are written back after the last step.

template <typename T> struct CgSteps {
    const int32_t *active, *list;
    int nsys, nslots, steps, max_iter;
    UTab<T> U;
    const double *kap;
    long n;
    const int32_t *sched;
    T kappa;
    T2<T> *p, *t, *w, *q, *r, *e;
    double2 *sc;    // 8 per system: [0] rr, [1] |w|^2, [3] new rr, [4] beta
    double *part;   // 3 x items: |w|^2, then |r|^2 of even and of odd steps
    double delta2;  // reliable-update threshold (squared)
    double *rmax;
    int32_t *upd, *its;
};

// sum over the 128 lanes of a workgroup (two wavefronts); every lane gets it
__device__ __forceinline__ double wg_sum(double v, double *sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = sh[0] + sh[1];
    __syncthreads();
    return r;
}

// the partial sums of system j's items, added in the same order everywhere
__device__ __forceinline__ double sys_sum(const double *part, int j, int nslots, double *sh)
{
    double v = 0;
    for (int i = threadIdx.x; i < nslots; i += Cube<4>::Vh) v += part[(long)j * nslots + i];
    return wg_sum(v, sh);
}

template <typename T>
__global__ __launch_bounds__(Cube<4>::Vh) void k_cg_steps(Geo g, CgSteps<T> a)
{
    constexpr int B = 4, Vb = Cube<B>::Vb, Vh = Cube<B>::Vh;
    __shared__ T2<T> sh[12][Vh];
    __shared__ double rs[2];
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    const int t = threadIdx.x, items = a.nslots * a.nsys, G = gridDim.x;
    double *pww = a.part, *prr[2] = {a.part + items, a.part + 2 * (long)items};
    // the residual the step starts from: the stored one, or the last step's
    auto rr_in = [&](int k, int j, int m) -> double {
        return k == 0 ? a.sc[8L * m].x : sys_sum(prr[(k + 1) & 1], j, a.nslots, rs);
    };
    for (int k = 0; k < a.steps; ++k) {
        // w = Dhat^+ p: odd half from p, then the even half with p as diagonal
        for (int it = blockIdx.x; it < items; it += G) {
            const int m = sys_at(a.list, it / a.nslots);
            if (a.active && !a.active[m]) continue;
            blk_eo_block<T, B, 1, CLOV_NONE, 0>(g, m, a.sched[it % a.nslots], t, a.U, a.kap, 0, nullptr, a.n, 1, a.p,
                                                nullptr, a.t, a.kappa, sh);
            __syncthreads();
        }
        grid.sync();
        for (int it = blockIdx.x; it < items; it += G) {
            const int m = sys_at(a.list, it / a.nslots);
            if (a.active && !a.active[m]) continue;
            const double v = blk_eo_block<T, B, 1, CLOV_NONE, 1>(g, m, a.sched[it % a.nslots], t, a.U, a.kap, 1,
                                                                 nullptr, a.n, 0, a.t, a.p, a.w, -a.kappa, sh);
            const double s = wg_sum(v, rs);
            if (t == 0) pww[it] = s;
        }
        grid.sync();
        // q = Dhat w
        for (int it = blockIdx.x; it < items; it += G) {
            const int m = sys_at(a.list, it / a.nslots);
            if (a.active && !a.active[m]) continue;
            blk_eo_block<T, B, 0, CLOV_NONE, 0>(g, m, a.sched[it % a.nslots], t, a.U, a.kap, 0, nullptr, a.n, 1, a.w,
                                                nullptr, a.t, a.kappa, sh);
            __syncthreads();
        }
        grid.sync();
        for (int it = blockIdx.x; it < items; it += G) {
            const int m = sys_at(a.list, it / a.nslots);
            if (a.active && !a.active[m]) continue;
            blk_eo_block<T, B, 0, CLOV_NONE, 0>(g, m, a.sched[it % a.nslots], t, a.U, a.kap, 1, nullptr, a.n, 0, a.t,
                                                a.w, a.q, -a.kappa, sh);
            __syncthreads();
        }
        grid.sync();
        // alpha = rr / |w|^2; e += alpha w, r -= alpha q on the block's even
        // sites, and the partial |r|^2
        for (int it = blockIdx.x; it < items; it += G) {
            const int j = it / a.nslots, m = sys_at(a.list, j);
            if (a.active && !a.active[m]) continue;
            const double ww = sys_sum(pww, j, a.nslots, rs), rr = rr_in(k, j, m);
            const T al = (T)(ww > 0 ? rr / ww : 0.0);
            const long base = m * a.n + (long)a.sched[it % a.nslots] * 12 * Vb + t;
            double nr = 0;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const long i = base + (long)c * Vb;
                T2<T> ei = a.e[i], ri = a.r[i];
                const T2<T> wi = a.w[i], qi = a.q[i];
                ei.x = ei.x + al * wi.x;
                ei.y = ei.y + al * wi.y;
                ri.x = ri.x - al * qi.x;
                ri.y = ri.y - al * qi.y;
                a.e[i] = ei;
                a.r[i] = ri;
                nr += (double)ri.x * (double)ri.x + (double)ri.y * (double)ri.y;
            }
            const double s = wg_sum(nr, rs);
            if (t == 0) prr[k & 1][it] = s;
        }
        grid.sync();
        // beta = rr_new / rr, p = r + beta p; the step's control
        for (int it = blockIdx.x; it < items; it += G) {
            const int j = it / a.nslots, m = sys_at(a.list, j);
            if (a.active && !a.active[m]) continue;
            const double rr0 = rr_in(k, j, m), rr = sys_sum(prr[k & 1], j, a.nslots, rs);
            const T b = (T)(rr0 > 0 ? rr / rr0 : 0.0);
            const long base = m * a.n + (long)a.sched[it % a.nslots] * 12 * Vb + t;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const long i = base + (long)c * Vb;
                const T2<T> ri = a.r[i], pi = a.p[i];
                a.p[i].x = ri.x + b * pi.x;
                a.p[i].y = ri.y + b * pi.y;
            }
            if (it % a.nslots == 0 && t == 0) {
                const int kk = ++a.its[m];
                a.rmax[m] = fmax(a.rmax[m], rr);
                if (!(rr > a.delta2 * a.rmax[m]) || kk >= a.max_iter) a.upd[m] = 1;
            }
        }
        grid.sync();
    }
    // the CG scalars of the last step, as the step-by-step form leaves them
    for (int it = blockIdx.x; it < items; it += G) {
        if (it % a.nslots) continue;
        const int j = it / a.nslots, m = sys_at(a.list, j);
        if (a.active && !a.active[m]) continue;
        const double rr0 = rr_in(a.steps - 1, j, m), rr = sys_sum(prr[(a.steps - 1) & 1], j, a.nslots, rs);
        const double ww = sys_sum(pww, j, a.nslots, rs);
        if (t == 0) {
            a.sc[8L * m + 1] = make_double2(ww, 0.0);
            a.sc[8L * m + 3] = make_double2(rr, 0.0);
            a.sc[8L * m + 4] = make_double2(rr0 > 0 ? rr / rr0 : 0.0, 0.0);
            a.sc[8L * m] = make_double2(rr, 0.0);
        }
    }
}

}  // namespace

bool launch_block_round16(const Geo &g, const Sys &sy, Links<double> U, H16c d, double2 *x, const double2 *b,
                          H16 r16, double *rn, double kappa, int slot0, int nslots, hipStream_t s)
{
    if (nslots <= 0 || sy.M <= 0) return true;
    if (g.B[0] != 4 || g.B[1] != 4 || g.B[2] != 4 || g.B[3] != 4 || !U.su3 || U.ctab || sy.list) return false;
    const int si = sched_index(g, slot0, nslots);
    if (si < 0) return false;
    k_block_round16<<<dim3(nslots, sy.M), Cube<4>::Vb, 0, s>>>(g, sy.active, U.tab, U.kap, sy.n, g.sched[si], d.v,
                                                              d.s, x, b, r16.v, r16.s, rn, kappa);
    return true;
}

bool cg_steps_fit(const Geo &g, bool su3, bool clover)
{
    return g.B[0] == 4 && g.B[1] == 4 && g.B[2] == 4 && g.B[3] == 4 && su3 && !clover &&
           sched_index(g, 0, g.nblk) >= 0;
}

template <typename T>
hipError_t launch_cg_steps(const Geo &g, const Sys &sy, Links<T> U, T kappa, int steps, T2<T> *p, T2<T> *t,
                           T2<T> *w, T2<T> *q, T2<T> *r, T2<T> *e, double2 *sc, double *part, double delta2,
                           int max_iter, double *rmax, int32_t *upd, int32_t *its, hipStream_t s)
{
    if (!cg_steps_fit(g, U.su3, U.ctab != nullptr)) return hipErrorInvalidValue;
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e0 = hipGetDevice(&dev);
    if (e0 == hipSuccess) e0 = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e0 == hipSuccess)
        e0 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(&k_cg_steps<T>),
                                                          Cube<4>::Vh, 0);
    if (e0 != hipSuccess) return e0;
    const long items = (long)g.nblk * sy.launch_m();
    // every workgroup must be resident at once (the launch is refused otherwise)
    const int G = (int)std::max<long>(1, std::min<long>(items, (long)per_cu * cus));
    Geo gc = g;
    CgSteps<T> a{sy.active, sy.list, sy.launch_m(), g.nblk, steps, max_iter, U.tab, U.kap, sy.n,
                 g.sched[sched_index(g, 0, g.nblk)], kappa, p, t, w, q, r, e, sc, part, delta2, rmax, upd, its};
    void *args[] = {&gc, &a};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_cg_steps<T>), dim3(G), dim3(Cube<4>::Vh),
                                      args, 0, s);
}

template hipError_t launch_cg_steps<double>(const Geo &, const Sys &, Links<double>, double, int, double2 *,
                                            double2 *, double2 *, double2 *, double2 *, double2 *, double2 *, double *,
                                            double, int, double *, int32_t *, int32_t *, hipStream_t);
template hipError_t launch_cg_steps<float>(const Geo &, const Sys &, Links<float>, float, int, float2 *, float2 *,
                                           float2 *, float2 *, float2 *, float2 *, double2 *, double *, double, int,
                                           double *, int32_t *, int32_t *, hipStream_t);

}  // namespace wdr
