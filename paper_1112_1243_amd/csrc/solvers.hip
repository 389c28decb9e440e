// Batched solver drivers: Schwarz preconditioner, flexible GCR, CG on the
// normal equations, Dirichlet block solves and the Schur complement
// (paper Sec. 3, eqs. domdec and ddfactor; Sec. 4, "one inversion for each
// factor").
//
// A call advances M independent systems (same geometry, own gauge field,
// own right-hand side) in lockstep: every kernel launch covers all systems
// that are still iterating, so small lattices still fill the GPU.  Outer
// iterations are FP64 with FP64 true residuals and deterministic FP64
// reductions; the Schwarz preconditioner and the inner block MR run in
// sp.inner (FP32 by default).  Krylov scalars stay in device memory; the
// host reads the M residual norms once per iteration to stop converged
// systems.
#include <memory>
#include <algorithm>
#include <cmath>
#include <vector>

#include "runtime.h"

namespace wdr {
namespace {

// ------------------------------------------------------------ small kernels

// CG scalars per system, 8 per system: [0] rr, [1] ww, [3] rr_new,
// [4] beta, [5] true residual (alpha = rr / ww is formed where it is used)
// p = r + beta p
template <typename T>
__global__ __launch_bounds__(256) void k_cg_p(const int32_t *active, const int32_t *list, long n, int hs, long total,
                                              const double2 *sc, const T2<T> *r, T2<T> *p)
{
    const long k = (long)blockIdx.x * 256 + threadIdx.x;
    if (k >= total) return;
    int m;
    const long i = batch_elem(list, n, hs, k, m);
    if (active && !active[m]) return;
    const T b = (T)sc[8L * m + 4].x;
    const T2<T> ri = r[i], pi = p[i];
    p[i].x = ri.x + b * pi.x;
    p[i].y = ri.y + b * pi.y;
}

// ---- mixed-precision CGNE control (one thread per system); sc[8 m + k]:
// 0 rr, 1 |w|^2, 2 alpha, 3 new rr, 4 beta, 5 true FP64 residual^2
__global__ void k_cgm_init(int M, const double2 *sc, double *bn2, double *rmax, int32_t *alive, int32_t *upd,
                           int32_t *its)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const double b = sc[8L * m + 5].x;
    bn2[m] = b;
    rmax[m] = b;
    alive[m] = b > 0;
    upd[m] = 0;
    its[m] = 0;
}
// after an FP32 step: beta = rr_new / rr, rr = rr_new; then ask for a
// reliable update once the iterated residual fell by RELIABLE_DELTA below its
// largest value since the last update (or at the iteration limit, where the
// true residual decides)
__global__ void k_cgm_beta(int M, double2 *sc, double delta2, int max_iter, const int32_t *alive, double *rmax,
                           int32_t *upd, int32_t *its)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M || !alive[m]) return;
    double2 *q = sc + 8L * m;
    const double rr0 = q[0].x, rr = q[3].x;
    q[4] = make_double2(rr0 > 0 ? rr / rr0 : 0.0, 0.0);
    q[0] = q[3];
    const int k = ++its[m];
    rmax[m] = fmax(rmax[m], rr);
    if (!(rr > delta2 * rmax[m]) || k >= max_iter) upd[m] = 1;
}
// after the FP64 true residual of the updated systems: retire converged ones,
// restart the reference of the others from the true residual
__global__ void k_cgm_update(int M, double2 *sc, const double *bn2, double tol2, int max_iter, const int32_t *its,
                             int32_t *alive, int32_t *upd, double *rmax, int32_t *nupd)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M || !upd[m]) return;
    ++nupd[m];
    const double r = sc[8L * m + 5].x;
    if (!isfinite(r) || r <= tol2 * bn2[m] || its[m] >= max_iter) alive[m] = 0;
    sc[8L * m] = make_double2(r, 0.0);
    rmax[m] = r;
}
// r = (FP32) r64 and e = 0 for the updated systems; clears their flag
template <typename T>
__global__ __launch_bounds__(256) void k_cgm_refresh(const int32_t *list, long n, int hs, long total, int32_t *upd,
                                                     const double2 *r64, T2<T> *r, T2<T> *e)
{
    const long k = (long)blockIdx.x * 256 + threadIdx.x;
    if (k >= total) return;
    int m;
    const long i = batch_elem(list, n, hs, k, m);
    if (!upd[m]) return;
    const double2 v = r64[i];
    r[i].x = (T)v.x;
    r[i].y = (T)v.y;
    e[i].x = e[i].y = (T)0;
}
// reference of the first reliable-update test: the initial iterated residual
__global__ void k_cgm_rmax(int M, const double2 *sc, double *rmax)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < M) rmax[m] = sc[8L * m].x;
}
__global__ void k_cgm_clear(int M, int32_t *upd)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < M) upd[m] = 0;
}

// relative residual from |r|^2 and |b|^2: 0 for b = 0 (x = 0 is exact), and
// infinite when either norm is not finite (a NaN right-hand side must not
// count as solved)
inline double rel_resid(double r2, double b2)
{
    if (!std::isfinite(b2) || !std::isfinite(r2)) return INFINITY;
    return b2 > 0 ? std::sqrt(r2 / b2) : 0.0;
}

inline unsigned nb256(long n) { return (unsigned)((n + 255) / 256); }
inline unsigned nb64(long n) { return (unsigned)((n + 63) / 64); }


// reads `count` device values (`stride` complex numbers apart, the .x part)
// to host; copies exactly the (count - 1) * stride + 1 entries spanned
void read_x(const double2 *dev, int count, int stride, std::vector<double> &out, hipStream_t s)
{
    std::vector<double2> tmp((size_t)(count - 1) * stride + 1);
    (void)hipMemcpyAsync(tmp.data(), dev, tmp.size() * sizeof(double2), hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
    out.resize(count);
    for (int m = 0; m < count; ++m) out[m] = tmp[(size_t)m * stride].x;
}

// Asynchronous read-back of per-system device flags into the context's
// pinned buffer (two slots).  A solver loop posts the flags after queueing
// iteration j and inspects those of iteration j - 1, so the GPU already has
// iteration j while the host waits.
struct FlagPoll {
    wdr_ctx *c;
    int M;
    bool ok = false;
    FlagPoll(wdr_ctx *c_, int M_) : c(c_), M(M_)
    {
        if (c->poll_cap < 2 * (size_t)M) {
            if (c->poll_host) (void)hipHostFree(c->poll_host);
            c->poll_host = nullptr;
            c->poll_cap = 0;
            if (hipHostMalloc((void **)&c->poll_host, 2 * (size_t)M * sizeof(int32_t)) != hipSuccess) return;
            c->poll_cap = 2 * (size_t)M;
        }
        for (auto &e : c->poll_ev)
            if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return;
        ok = true;
    }
    int32_t *slot(int k) const { return c->poll_host + (size_t)k * M; }
    void post(const int32_t *dev, int k, hipStream_t s) const
    {
        (void)hipMemcpyAsync(slot(k), dev, (size_t)M * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        (void)hipEventRecord(c->poll_ev[k], s);
    }
    // the same with M per-system values (.x of vals) read along with the
    // flags into vals_at(k); false if the pinned value buffer is missing
    bool want_vals()
    {
        if (c->poll_val_cap < 3 * (size_t)M) {
            if (c->poll_val) (void)hipHostFree(c->poll_val);
            c->poll_val = nullptr;
            c->poll_val_cap = 0;
            if (hipHostMalloc((void **)&c->poll_val, 3 * (size_t)M * sizeof(double2)) != hipSuccess) return false;
            c->poll_val_cap = 3 * (size_t)M;
        }
        return true;
    }
    double2 *vals_at(int k) const { return c->poll_val + (size_t)k * M; }
    void post(const int32_t *dev, const double2 *vals, int k, hipStream_t s) const
    {
        (void)hipMemcpyAsync(vals_at(k), vals, (size_t)M * sizeof(double2), hipMemcpyDeviceToHost, s);
        post(dev, k, s);
    }
    // waits for the copy posted in slot k; true if every flag there is 0
    bool none(int k) const
    {
        (void)hipEventSynchronize(c->poll_ev[k]);
        for (int m = 0; m < M; ++m)
            if (slot(k)[m]) return false;
        return true;
    }
};

// ---- FGCR control on the device (one thread per system)

__global__ void k_fgcr_init(int M, const double2 *nr, double *bn2, int32_t *alive, int32_t *act, int32_t *cnt,
                            int32_t *its)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const double b = nr[m].x;
    bn2[m] = b;
    alive[m] = act[m] = b > 0;
    cnt[m] = its[m] = 0;
}

// after Krylov step j: count it and stop the cycle of a converged system
__global__ void k_fgcr_inner(int M, int j, const double2 *nr, const double *bn2, double tol2, int max_iter,
                             int32_t *act, int32_t *cnt, int32_t *its)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M || !act[m]) return;
    cnt[m] = j + 1;
    const int k = ++its[m];
    if (!(nr[m].x > tol2 * bn2[m]) || k >= max_iter) act[m] = 0;
}

// coefficients of x += sum_l al_l phi_l from the Gram-Schmidt data:
// D phi_j = b_j chi_j + sum_{l<j} A_lj chi_l, r-component c_l along chi_l
__global__ void k_fgcr_backsub(int M, const double2 *A, const double2 *bj, const double2 *cj, const int32_t *cnt,
                               const int32_t *alive, double2 *al)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M || !alive[m]) return;
    const int k = cnt[m];
    for (int l = k - 1; l >= 0; --l) {
        double re = cj[m * 16 + l].x, im = cj[m * 16 + l].y;
        for (int jj = l + 1; jj < k; ++jj) {
            const double2 a0 = A[(size_t)m * 256 + jj * 16 + l], a1 = A[(size_t)M * 256 + (size_t)m * 256 + jj * 16 + l];
            const double ar = a0.x + a1.x, ai = a0.y + a1.y;
            const double2 aj = al[m * 16 + jj];
            re -= ar * aj.x - ai * aj.y;
            im -= ar * aj.y + ai * aj.x;
        }
        const double bb = sqrt(bj[m * 16 + l].x);
        al[m * 16 + l] = make_double2(re / bb, im / bb);
    }
}

// after the true residual of a cycle: retire converged systems, start the next cycle
__global__ void k_fgcr_outer(int M, const double2 *nr, const double *bn2, double tol2, int max_iter,
                             const int32_t *its, int32_t *alive, int32_t *act, int32_t *cnt)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    if (alive[m]) {
        const double r = nr[m].x;
        if (!isfinite(r) || r <= tol2 * bn2[m] || its[m] >= max_iter) alive[m] = 0;
    }
    act[m] = alive[m];
    cnt[m] = 0;
}

// ---- block-solve control on the device (one thread per system): the worst
// relative residual over the selected blocks decides convergence

// per-system control of a block solve, one workgroup of BC_NT threads per
// system: the largest per-block ratio |r_b|^2 / |b_b|^2 over the slots in
// range (blocks with b_b = 0 are left out); a non-finite norm makes it
// infinite (fmax alone would drop a NaN)
constexpr int BC_NT = 256;
__device__ double worst_ratio(int m, int nblk, int slot0, int ns, const double *bn, const double *rn)
{
    __shared__ double sh[BC_NT];
    double wv = 0;
    for (int i = slot0 + threadIdx.x; i < slot0 + ns; i += BC_NT) {
        const size_t k = (size_t)m * nblk + i;
        const double b = bn[k];
        if (!isfinite(b)) {
            wv = INFINITY;
        } else if (b > 0) {
            const double q = rn ? rn[k] / b : 1.0;
            wv = isfinite(q) ? fmax(wv, q) : INFINITY;
        }
    }
    sh[threadIdx.x] = wv;
    __syncthreads();
    for (int off = BC_NT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    return sh[0];
}

// alive = some block has a nonzero right-hand side; a non-finite right-hand
// side ends the system at once, unconverged
__global__ __launch_bounds__(BC_NT) void k_block_init(int nblk, int slot0, int ns, const double *bn, int32_t *alive,
                                                      int32_t *its, double *worst)
{
    const int m = blockIdx.x;
    const double any = worst_ratio(m, nblk, slot0, ns, bn, nullptr);
    if (threadIdx.x == 0) {
        alive[m] = any > 0 && isfinite(any);
        its[m] = 0;
        worst[m] = isfinite(any) ? 0 : INFINITY;
    }
}

__global__ __launch_bounds__(BC_NT) void k_block_check(int nblk, int slot0, int ns, const double *bn, const double *rn,
                                                       double tol2, int32_t *alive, int32_t *its, double *worst)
{
    const int m = blockIdx.x;
    if (!alive[m]) return;
    double wv = worst_ratio(m, nblk, slot0, ns, bn, rn);
    if (threadIdx.x == 0) {
        ++its[m];
        worst[m] = wv;
        // converged, or a residual that is no longer finite (nothing more to gain)
        if (!(wv > tol2) || !isfinite(wv)) alive[m] = 0;
    }
}

// clears the fields of the systems whose flag is 0
__global__ __launch_bounds__(256) void k_zero_dead(const int32_t *alive, long n, long total, double2 *f)
{
    const long i = blockIdx.x * 256L + threadIdx.x;
    if (i < total && !alive[i / n]) f[i] = make_double2(0.0, 0.0);
}

}  // namespace

void apply_D64(wdr_ctx *c, const Sys &sy, const GaugeTab &U, double kappa, const double2 *in, double2 *out,
               hipStream_t s)
{
    Links<double> L = U.u64;
    L.cmode = CLOV_DIAG;  // with a clover term the diagonal is A
    launch_dslash<double>(c->g, sy, L, HOPS_ALL, -1, 0, in, in, out, kappa, 0, c->g.nblk, s);
}

// ------------------------------------------------------------ SAP

// x_zero: x is already zero
template <typename T>
static void sap_run(wdr_ctx *c, const Sys &sy, Links<T> U, T kappa, int ncy, int nmr, const T2<T> *eta, T2<T> *x,
                    hipStream_t s, bool x_zero = false)
{
    if (!x_zero) launch_zero<T>(x, sy.n * sy.M, s);
    int b0, bn, w0, wn;
    colour_slots(c, 0, b0, bn);
    colour_slots(c, 1, w0, wn);
    for (int cy = 0; cy < ncy; ++cy) {
        launch_sap_colour<T>(c->g, sy, U, eta, x, kappa, nmr, b0, bn, s);
        launch_sap_colour<T>(c->g, sy, U, eta, x, kappa, nmr, w0, wn, s);
    }
}

// FP16 fields of M systems in the context's workspace pool
struct H16Work {
    Work v, sc;
    H16Work(wdr_ctx *c, int M)
        : v(c, field_bytes(c, WDR_F16) * M), sc(c, sizeof(float) * (size_t)c->g.nblk * M)
    {
    }
    bool ok() const { return v.ok() && sc.ok(); }
    H16 f() const { return {v.as<h2>(), sc.as<float>()}; }
    H16c cf() const { return {v.as<const h2>(), sc.as<const float>()}; }
};

static wdr_status need16(const GaugeTab &U)
{
    if (U.u16.tab) return WDR_OK;
    set_error("the FP16 inner solver needs SU(3) links and 4^4 blocks");
    return WDR_EINVAL;
}

wdr_status sap64(wdr_ctx *c, const Sys &sy, const GaugeTab &U, double kappa, const wdr_solver_params &sp,
                 const double2 *in, double2 *out, hipStream_t s)
{
    if (sp.inner == WDR_F64) {
        sap_run<double>(c, sy, U.u64, kappa, sp.sap_cycles, sp.mr_steps, in, out, s);
        return WDR_OK;
    }
    // the FP16 sweep kernels keep no 6 x 6 blocks of A beside their LDS
    // fields: with the clover term an FP16 inner level sweeps in FP32
    if (sp.inner == WDR_F16 && !U.u64.ctab) {
        wdr_status e = need16(U);
        if (e != WDR_OK) return e;
        H16Work eh(c, sy.M), xh(c, sy.M);
        if (!eh.ok() || !xh.ok()) return WDR_ENOMEM;
        const Geo &g = c->g;
        launch_to_h16<double>(g, sy, in, eh.f(), 0, g.nblk, s);
        launch_zero_h16(g, sy, xh.f(), s);
        int b0, bn, w0, wn;
        colour_slots(c, 0, b0, bn);
        colour_slots(c, 1, w0, wn);
        for (int cy = 0; cy < sp.sap_cycles; ++cy)
            if (!launch_mr_h16(0, g, sy, U.u16, eh.cf(), xh.f(), (float)kappa, sp.mr_steps, b0, bn, s) ||
                !launch_mr_h16(0, g, sy, U.u16, eh.cf(), xh.f(), (float)kappa, sp.mr_steps, w0, wn, s))
                return need16(GaugeTab{});
        launch_from_h16(g, sy, xh.cf(), out, 0, 0, g.nblk, s);
        return WDR_OK;
    }
    Work e(c, field_bytes(c, WDR_F32) * sy.M), x(c, field_bytes(c, WDR_F32) * sy.M);
    if (!e.ok() || !x.ok()) return WDR_ENOMEM;
    launch_convert_zero_f32(sy, in, e.as<float2>(), x.as<float2>(), s);
    sap_run<float>(c, sy, U.u32, (float)kappa, sp.sap_cycles, sp.mr_steps, e.as<float2>(), x.as<float2>(), s, true);
    launch_convert<double, float>(sy, x.as<float2>(), out, s);
    return WDR_OK;
}

// ------------------------------------------------------------ FGCR + SAP

static wdr_status fgcr(wdr_ctx *c, int M, const GaugeTab &U, double kappa, const wdr_solver_params &sp, double tol,
                       const double2 *b, double2 *x, std::vector<Stats> &st, hipStream_t s)
{
    const long n = field_n(c);
    const size_t fb = field_bytes(c, WDR_F64) * M;
    const int nkv = sp.restart;
    std::vector<Work *> bufs;
    struct Cleanup {
        std::vector<Work *> &v;
        ~Cleanup()
        {
            for (auto *w : v) delete w;
        }
    } cleanup{bufs};
    for (int j = 0; j < 2 * nkv + 2; ++j) {
        bufs.push_back(new Work(c, fb));
        if (!bufs.back()->ok()) return WDR_ENOMEM;
    }
    double2 *r = bufs[2 * nkv]->as<double2>(), *t = bufs[2 * nkv + 1]->as<double2>();
    // device tables: chi_0..chi_{nkv-1}, phi_0..phi_{nkv-1}
    Work tab(c, 2 * nkv * sizeof(void *));
    // scalars: A[2][M][16][16] (two CGS passes), bj[M][16], cj[M][16], al[M][16], nr[M]
    Work scal(c, sizeof(double2) * ((size_t)M * (2 * 256 + 16 * 3 + 1)));
    Work red(c, sizeof(double) * red_scratch(M));
    if (!tab.ok() || !scal.ok() || !red.ok()) return WDR_ENOMEM;
    std::vector<const void *> hp(2 * nkv);
    for (int j = 0; j < nkv; ++j) {
        hp[j] = bufs[j]->as<void>();
        hp[nkv + j] = bufs[nkv + j]->as<void>();
    }
    WDR_HIP(hipMemcpyAsync(tab.as<void>(), hp.data(), hp.size() * sizeof(void *), hipMemcpyHostToDevice, s));
    const double2 *const *chis = tab.as<const double2 *const>();
    const double2 *const *phis = chis + nkv;
    auto chi = [&](int j) { return bufs[j]->as<double2>(); };
    auto phi = [&](int j) { return bufs[nkv + j]->as<double2>(); };
    double2 *A = scal.as<double2>();
    double2 *bj = A + (size_t)M * 512, *cj = bj + (size_t)M * 16, *al = cj + (size_t)M * 16, *nr = al + (size_t)M * 16;

    const Sys all = all_sys(c, M);
    // per-system control state on the device: bn2 (|b|^2), act (in the current
    // cycle), alive (not converged), cnt (Krylov vectors of the cycle), its
    Work ctl(c, sizeof(double) * M + 4 * sizeof(int32_t) * M);
    FlagPoll poll(c, M);
    if (!ctl.ok() || !poll.ok) return WDR_ENOMEM;
    double *bn2 = ctl.as<double>();
    int32_t *act = reinterpret_cast<int32_t *>(bn2 + M), *alive = act + M, *cnt = alive + M, *its = cnt + M;
    const double tol2 = tol * tol;
    const unsigned nbm = (unsigned)((M + 63) / 64);
    launch_norm2<double>(all, b, red.as<double>(), nr, 1, s);
    k_fgcr_init<<<nbm, 64, 0, s>>>(M, nr, bn2, alive, act, cnt, its);
    // |b|^2 to the host with the first flags, for the convergence forecast below
    const bool fc = poll.want_vals();
    if (fc) (void)hipMemcpyAsync(poll.vals_at(2), nr, (size_t)M * sizeof(double2), hipMemcpyDeviceToHost, s);
    std::vector<double> last(M, 0.0);  // |r|^2 of each system after the previous step read
    launch_zero<double>(x, n * M, s);
    launch_convert<double, double>(all, b, r, s);
    const Sys sa{M, act, n}, sw{M, alive, n};
    for (;;) {
        for (int j = 0; j < nkv; ++j) {
            wdr_status e = sap64(c, sa, U, kappa, sp, r, phi(j), s);
            if (e != WDR_OK) return e;
            apply_D64(c, sa, U, kappa, phi(j), chi(j), s);
            // classical Gram-Schmidt, twice (CGS2), each update fused with the
            // next reduction; then bj = |chi_j|^2, cj = <chi_j, r> / |chi_j|
            if (j > 0) {
                double2 *co0 = A + j * 16, *co1 = A + (size_t)M * 256 + j * 16;
                launch_multidot<double>(sa, chis, j, chi(j), red.as<double>(), co0, 256, s);
                launch_cgs_multidot(sa, co0, 256, chis, j, chi(j), red.as<double>(), co1, 256, s);
                launch_cgs_norm_dot(sa, co1, 256, chis, j, chi(j), r, red.as<double>(), bj + j, 16, cj + j, 16, s);
            } else {
                launch_norm_dot(sa, chi(j), r, red.as<double>(), bj + j, 16, cj + j, 16, s);
            }
            // chi_j /= |chi_j|, r -= cj chi_j, nr = |r|^2
            launch_orth_norm(sa, bj + j, 16, cj + j, 16, chi(j), r, red.as<double>(), nr, 1, s);
            k_fgcr_inner<<<nbm, 64, 0, s>>>(M, j, nr, bn2, tol2, sp.max_iter, act, cnt, its);
            if (fc) poll.post(act, nr, j & 1, s);
            else poll.post(act, j & 1, s);
            // step j is queued; stop once step j - 1 left no system active
            // (step j then runs as a no-op)
            if (j > 0 && poll.none((j - 1) & 1)) break;
            // Forecast: if every system still active after step j - 1 reaches
            // the tolerance in step j at the rate of its last step, wait for
            // step j's flags now instead of queueing step j + 1, which would
            // most likely run as a no-op.  Either way the numbers are the same.
            if (fc && j > 0) {
                const int32_t *f = poll.slot((j - 1) & 1);
                const double2 *v = poll.vals_at((j - 1) & 1), *b2 = poll.vals_at(2);
                bool done = true;
                for (int m = 0; m < M && done; ++m) {
                    if (!f[m]) continue;
                    const double now = v[m].x, q = last[m] > 0 ? now / last[m] : 1.0;
                    done = now * q <= tol2 * b2[m].x;
                }
                for (int m = 0; m < M; ++m) last[m] = v[m].x;
                if (done && poll.none(j & 1)) break;
            }
        }
        k_fgcr_backsub<<<nbm, 64, 0, s>>>(M, A, bj, cj, cnt, alive, al);
        launch_multi_axpy(sw, al, 16, 1.0, phis, nkv, cnt, x, 1, s);
        // true residual
        apply_D64(c, sw, U, kappa, x, t, s);
        launch_sub_norm(sw, b, t, r, red.as<double>(), nr, 1, s);
        k_fgcr_outer<<<nbm, 64, 0, s>>>(M, nr, bn2, tol2, sp.max_iter, its, alive, act, cnt);
        poll.post(alive, 0, s);
        if (poll.none(0)) break;
    }
    std::vector<double> hbn2(M), rn2;
    std::vector<int32_t> hits(M);
    WDR_HIP(hipMemcpyAsync(hbn2.data(), bn2, sizeof(double) * M, hipMemcpyDeviceToHost, s));
    WDR_HIP(hipMemcpyAsync(hits.data(), its, sizeof(int32_t) * M, hipMemcpyDeviceToHost, s));
    read_x(nr, M, 1, rn2, s);
    const std::vector<double> &bn2h = hbn2;
    const std::vector<int32_t> &itsh = hits;
    st.assign(M, Stats());
    bool ok = true;
    for (int m = 0; m < M; ++m) {
        st[m].iters = itsh[m];
        st[m].total = itsh[m];
        st[m].rel = rel_resid(rn2[m], bn2h[m]);
        st[m].converged = st[m].rel <= tol;
        ok = ok && st[m].converged;
    }
    WDR_HIP(hipGetLastError());
    if (!ok) {
        const Stats sm = summarize(st);
        set_error("FGCR stopped at " + std::to_string(sm.iters) + " iterations, relative residual " +
                  std::to_string(sm.rel));
        return WDR_ENOCONV;
    }
    return WDR_OK;
}

// ------------------------------------------------------------ CGNE

// Even-odd reduction: with D = [[A_ee, -k H_eo], [-k H_oe, A_oo]] on (even,
// odd) sites (A = 1 without a clover term), D x = b becomes
//     Dhat x_e = bh_e,  Dhat = A_ee - k^2 H_eo A_oo^-1 H_oe,
//     bh_e = b_e + k H_eo A_oo^-1 b_o,  x_o = A_oo^-1 (b_o + k H_oe x_e),
// and then b - D x is bh_e - Dhat x_e on even sites and 0 on odd ones (up to
// the rounding of A_oo^-1), so the solver's FP64 residual is that of the
// full system.  The clover factors ride in the stencil launches (CLOV_INV
// on the odd half, CLOV_DIAG on the even half).  CG runs on
// Dhat Dhat^+ y = bh (x_e = Dhat^+ y; Dhat^+ = g5 Dhat g5) with vectors and
// stencil in T, and reliable updates in FP64 (the scheme of Sleijpen and van
// der Vorst): whenever the iterated residual has fallen by RELIABLE_DELTA
// below its largest value since the last update, the correction e = Dhat^+
// (y - y_last) is folded into the FP64 x_e and the iterated residual replaced
// by the FP64 true residual, keeping the search direction.  Vectors keep the
// full-field layout with odd sites zero.
constexpr double RELIABLE_DELTA = 0.1;

// An instantiated HIP graph of one solver period.  Capture runs on the
// context's own stream (the caller's may be the legacy default stream, which
// cannot be captured) in thread-local mode, so other host threads driving
// other contexts are unaffected; nothing executes while capturing.
// Replaced graphs may still be running on the launch stream, so they are kept
// until the destructor, which first waits for that stream.
struct PeriodGraph {
    hipStream_t s;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<std::pair<hipGraph_t, hipGraphExec_t>> done;
    explicit PeriodGraph(hipStream_t s_) : s(s_) {}
    void reset()
    {
        if (graph || exec) done.emplace_back(graph, exec);
        exec = nullptr;
        graph = nullptr;
    }
    ~PeriodGraph()
    {
        reset();
        if (done.empty()) return;
        (void)hipStreamSynchronize(s);
        for (auto &d : done) {
            if (d.second) (void)hipGraphExecDestroy(d.second);
            if (d.first) (void)hipGraphDestroy(d.first);
        }
    }
    template <typename F> wdr_status capture(wdr_ctx *c, F &&enqueue)
    {
        if (!c->cap) WDR_HIP(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
        WDR_HIP(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
        enqueue(c->cap);
        const hipError_t le = hipGetLastError();
        const hipError_t ee = hipStreamEndCapture(c->cap, &graph);
        WDR_HIP(le);
        WDR_HIP(ee);
        WDR_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        return WDR_OK;
    }
};

template <typename T> Links<T> links_of(const GaugeTab &U);
template <> Links<double> links_of<double>(const GaugeTab &U) { return U.u64; }
template <> Links<float> links_of<float>(const GaugeTab &U) { return U.u32; }

// The operator an even-odd solve works on: D (all hops, every block), or
// the Dirichlet block operator D_b (hops inside the blocks) on the blocks of
// slots [slot0, slot0 + ns), whose even-odd reduction is again block by block
// (a block of even extent holds both parities of its sites).
struct EoOp {
    int hops = HOPS_ALL;
    int slot0 = 0, ns = -1;  // ns < 0: every block
    int count(const Geo &g) const { return ns < 0 ? g.nblk : ns; }
};

// out_e = (Dhat in)_e, or (Dhat^+ in)_e with dag; tmp receives
// -k A_oo^-1 H_oe in_e on odd sites; odd sites of out are not written (nor
// blocks outside op's slots)
template <typename T>
static void apply_dhat(const Geo &g, const Sys &sy, Links<T> U, T kappa, int dag, const T2<T> *in, T2<T> *tmp,
                       T2<T> *out, hipStream_t s, const EoOp &op = EoOp())
{
    Links<T> Ui = U, Un = U;
    Ui.cmode = CLOV_INV;
    Un.kneg = 1;
    Un.cmode = CLOV_DIAG;
    launch_dslash<T>(g, sy, Ui, op.hops, 1, dag, in, nullptr, tmp, kappa, op.slot0, op.count(g), s);
    launch_dslash<T>(g, sy, Un, op.hops, 0, dag, tmp, in, out, -kappa, op.slot0, op.count(g), s);
}

// op selects D or the Dirichlet blocks of some slots (b must then vanish on
// the other blocks, and x does there)
template <typename T>
static wdr_status cgne_eo(wdr_ctx *c, int M, const GaugeTab &U, double kappa, const wdr_solver_params &sp, double tol,
                          const double2 *b, double2 *x, std::vector<Stats> &st, hipStream_t s,
                          const EoOp &op = EoOp())
{
    const long n = field_n(c), total = n * M;
    const int prec = sizeof(T) == 8 ? WDR_F64 : WDR_F32;
    const size_t fb = field_bytes(c, WDR_F64) * M, fbT = field_bytes(c, prec) * M;
    Work bhw(c, fb), r64w(c, fb), t64w(c, fb), o64w(c, fb), rw(c, fbT), pw(c, fbT), ww(c, fbT), qw(c, fbT),
        ew(c, fbT), tw(c, fbT), scal(c, sizeof(double2) * 8 * M), red(c, sizeof(double) * red_scratch(M)),
        ctl(c, 2 * sizeof(double) * M + 4 * sizeof(int32_t) * M), lw(c, sizeof(int32_t) * M);
    FlagPoll poll(c, M);
    if (!bhw.ok() || !r64w.ok() || !t64w.ok() || !o64w.ok() || !rw.ok() || !pw.ok() || !ww.ok() || !qw.ok() ||
        !ew.ok() || !tw.ok() || !scal.ok() || !red.ok() || !ctl.ok() || !lw.ok() || !poll.ok)
        return WDR_ENOMEM;
    double2 *bh = bhw.as<double2>(), *r64 = r64w.as<double2>(), *t64 = t64w.as<double2>(), *o64 = o64w.as<double2>();
    T2<T> *r = rw.as<T2<T>>(), *p = pw.as<T2<T>>(), *w = ww.as<T2<T>>(), *qv = qw.as<T2<T>>(),
          *e = ew.as<T2<T>>(), *t = tw.as<T2<T>>();
    double2 *sc = scal.as<double2>();
    double *bn2 = ctl.as<double>(), *rmax = bn2 + M;
    int32_t *alive = reinterpret_cast<int32_t *>(rmax + M), *upd = alive + M, *its = upd + M, *nupd = its + M;
    const auto &g = c->g;
    const Links<T> UT = links_of<T>(U);
    Links<double> U64n = U.u64;
    U64n.kneg = 1;
    U64n.cmode = CLOV_NONE;  // the diagonal input b_e enters as it is
    const T kT = (T)kappa;
    const Sys all = all_sys(c, M);
    const int o0 = op.slot0, on = op.count(g);
    // the iterated vectors live on even sites: their updates and norms skip
    // the odd halves (zero) where the half-block volume allows it
    Sys sa{M, alive, n}, su{M, upd, n};
    sa.hs = su.hs = even_shift(g);
    std::vector<int32_t> live;
    int launch_m = M;
    const unsigned nbm = nb64(M);
    // the persistent form of the steps (wdr_cg_form) on the whole operator
    const bool persist = g.cg_form == WDR_CG_PERSISTENT && op.hops == HOPS_ALL && op.count(g) == g.nblk &&
                         cg_steps_fit(g, UT.su3, U.u64.ctab != nullptr);
    Work partw(c, persist ? sizeof(double) * 3 * g.nblk * M : 64);
    if (!partw.ok()) return WDR_ENOMEM;
    hipError_t persist_err = hipSuccess;

    // bh = [b_e + k H_eo A_oo^-1 b_o; 0]; odd parts of every iterated field stay 0
    launch_zero<double>(x, total, s);
    launch_zero<double>(bh, total, s);
    launch_zero<double>(t64, total, s);
    const bool clov = U.u64.ctab != nullptr;
    if (clov) launch_clover_mul<double>(g, all, U.u64.ctab, 1, 1, b, o64, s);  // odd sites of o64
    launch_dslash<double>(g, all, U64n, op.hops, 0, 0, clov ? o64 : b, b, bh, -kappa, o0, on, s);
    launch_norm2<double>(all, b, red.as<double>(), sc + 5, 8, s);
    k_cgm_init<<<nbm, 64, 0, s>>>(M, sc, bn2, rmax, alive, upd, its);  // |b|^2 of the full system
    launch_convert<T, double>(all, bh, r, s);
    launch_convert<T, T>(all, r, p, s);
    launch_zero<T>(e, total, s);
    launch_zero<T>(w, total, s);
    launch_zero<T>(qv, total, s);
    launch_norm2<T>(sa, r, red.as<double>(), sc, 8, s);
    k_cgm_rmax<<<nbm, 64, 0, s>>>(M, sc, rmax);
    k_cgm_clear<<<nbm, 64, 0, s>>>(M, nupd);
    // one period: ue steps, then the reliable update of the flagged systems
    const int ue = sp.update_every;
    auto period = [&](hipStream_t q) {
        const long tl = sa.ne() * sa.launch_m();
        if (persist) {
            const hipError_t le = launch_cg_steps<T>(g, sa, UT, kT, ue, p, t, w, qv, r, e, sc, partw.as<double>(),
                                                     RELIABLE_DELTA * RELIABLE_DELTA, sp.max_iter, rmax, upd, its, q);
            if (le != hipSuccess && persist_err == hipSuccess) persist_err = le;
        }
        for (int i = 0; i < (persist ? 0 : ue); ++i) {
            // w = Dhat^+ p, q = Dhat w, e += alpha w, r -= alpha q, p = r + beta p
            apply_dhat<T>(g, sa, UT, kT, 1, p, t, w, q, op);
            apply_dhat<T>(g, sa, UT, kT, 0, w, t, qv, q, op);
            launch_norm2<T>(sa, w, red.as<double>(), sc + 1, 8, q);
            launch_cg_xr_norm<T>(sa, sc, 8, e, w, r, qv, red.as<double>(), sc + 3, 8, q);
            k_cgm_beta<<<nbm, 64, 0, q>>>(M, sc, RELIABLE_DELTA * RELIABLE_DELTA, sp.max_iter, alive, rmax, upd,
                                          its);
            k_cg_p<T><<<nb256(tl), 256, 0, q>>>(alive, sa.list, n, sa.hs, tl, sc, r, p);
        }
        // x_e += e, r = bh - Dhat x_e in FP64
        launch_add_to64<T>(su, e, x, q);
        apply_dhat<double>(g, su, U.u64, kappa, 0, x, o64, t64, q, op);
        launch_sub_norm(su, bh, t64, r64, red.as<double>(), sc + 5, 8, q);
        k_cgm_update<<<nbm, 64, 0, q>>>(M, sc, bn2, tol * tol, sp.max_iter, its, alive, upd, rmax, nupd);
        k_cgm_refresh<T><<<nb256(tl), 256, 0, q>>>(su.list, n, su.hs, tl, upd, r64, r, e);
        k_cgm_clear<<<nbm, 64, 0, q>>>(M, upd);
    };
    // With sp.graph the period's launches (kernels only) are captured once on
    // the context's capture stream and replayed on s; the capture is redone
    // whenever compaction changes the launch list.
    PeriodGraph pg(s);
    for (int pt = 0;; ++pt) {
        if (sp.graph && !persist) {
            if (!pg.exec) {
                const wdr_status cs = pg.capture(c, period);
                if (cs != WDR_OK) return cs;
            }
            WDR_HIP(hipGraphLaunch(pg.exec, s));
        } else {
            period(s);
        }
        // poll one period behind; compact the launches to the live systems
        poll.post(alive, pt & 1, s);
        if (pt > 0) {
            if (poll.none((pt - 1) & 1)) break;
            const int32_t *fl = poll.slot((pt - 1) & 1);
            int cnt = 0;
            for (int m = 0; m < M; ++m) cnt += fl[m] != 0;
            if (2 * cnt <= launch_m) {
                live.clear();
                for (int m = 0; m < M; ++m)
                    if (fl[m]) live.push_back(m);
                // ordered after every launch already queued with the old list
                WDR_HIP(hipMemcpyAsync(lw.as<void>(), live.data(), live.size() * sizeof(int32_t),
                                       hipMemcpyHostToDevice, s));
                launch_m = cnt;
                sa.list = su.list = lw.as<int32_t>();
                sa.count = su.count = cnt;
                pg.reset();
            }
        }
        if (persist_err != hipSuccess) break;
    }
    if (persist_err != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        set_error(std::string("cooperative launch of the CG steps refused: ") + hipGetErrorString(persist_err));
        return WDR_EDEVICE;
    }
    // x_o = A_oo^-1 (b_o + k H_oe x_e), written into the odd sites of x in
    // place: the launch reads only the even sites of x
    Links<double> U64i = U64n;
    U64i.cmode = CLOV_INV;
    launch_dslash<double>(g, all, U64i, op.hops, 1, 0, x, b, x, -kappa, o0, on, s);

    std::vector<double> hbn2(M), rn2;
    std::vector<int32_t> hits(M), hupd(M);
    WDR_HIP(hipMemcpyAsync(hbn2.data(), bn2, sizeof(double) * M, hipMemcpyDeviceToHost, s));
    WDR_HIP(hipMemcpyAsync(hits.data(), its, sizeof(int32_t) * M, hipMemcpyDeviceToHost, s));
    WDR_HIP(hipMemcpyAsync(hupd.data(), nupd, sizeof(int32_t) * M, hipMemcpyDeviceToHost, s));
    read_x(sc + 5, M, 8, rn2, s);
    st.assign(M, Stats());
    bool ok = true;
    // compulsory bytes per system: setup and final step, then per CG step
    // (four halves in T, |w|^2, the x / r update, the p update) and per
    // reliable update (e into x, FP64 Dhat x, r64 = bh - Dhat x, the refresh);
    // the stencil halves cover the sites of op's blocks (Vo), the vector
    // kernels whole fields
    const double V = g.V, H = V / 2, Vo = V * on / g.nblk, Ho = Vo / 2;
    const double setup = 3 * V * spin_b<double>() + half_b<double>(Vo, true) + V * spin_b<double>() +
                         V * (spin_b<double>() + spin_b<T>()) + 2 * V * spin_b<T>() + 3 * V * spin_b<T>() +
                         H * spin_b<T>() + V * spin_b<double>() + half_b<double>(Vo, true) + 3 * V * spin_b<double>();
    const double step = 2 * half_b<T>(Vo, false) + 2 * half_b<T>(Vo, true) + H * spin_b<T>() + 6 * H * spin_b<T>() +
                        3 * H * spin_b<T>();
    const double update = H * (spin_b<T>() + 2 * spin_b<double>()) + half_b<double>(Vo, false) +
                          half_b<double>(Vo, true) + 3 * H * spin_b<double>() + H * (spin_b<double>() + 2 * spin_b<T>());
    // the clover blocks of every output site of every half (and A_oo^-1 b_o)
    const double cl_setup = clov ? H * (2 * spin_b<double>() + clov_b<double>()) + Ho * clov_b<double>() : 0;
    const double cl_step = clov ? 4 * Ho * clov_b<T>() : 0, cl_update = clov ? 2 * Ho * clov_b<double>() : 0;
    double bytes = 0;
    for (int m = 0; m < M; ++m) {
        bytes += setup + cl_setup + hits[m] * (step + cl_step) + hupd[m] * (update + cl_update);
        st[m].iters = hits[m];
        st[m].total = hits[m];
        st[m].rel = rel_resid(rn2[m], hbn2[m]);
        st[m].converged = st[m].rel <= tol;
        ok = ok && st[m].converged;
    }
    add_traffic(bytes);
    WDR_HIP(hipGetLastError());
    if (!ok) {
        const Stats sm = summarize(st);
        set_error("CGNE stopped at " + std::to_string(sm.iters) + " iterations, relative residual " +
                  std::to_string(sm.rel));
        return WDR_ENOCONV;
    }
    return WDR_OK;
}

// ---- FP16 even-odd CGNE control (one thread per system); sc[8 m + k]:
// 0 iterated rr, 1 |w|^2, 3 new rr, 4 beta, 5 FP64 true residual^2,
// 6 FP32 (middle) true residual^2
// after the middle level's residual: restart the iterated residual from it;
// ask for the outer update when it fell by OUTER_DELTA below the middle
// system's right-hand side, reached the tolerance, stopped falling (less
// than 2x since the previous middle update: the FP32 level has reached what
// its arithmetic resolves), or at the iteration limit
__global__ void k_c16_mid(int M, double2 *sc, const double *bn2, const double *b32n2, double tol2, double delta2,
                          int max_iter, const int32_t *its, int32_t *upd, int32_t *upd64, double *rmax, double *rprev,
                          int32_t *nmid)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M || !upd[m]) return;
    ++nmid[m];
    const double r = sc[8L * m + 6].x;
    sc[8L * m] = make_double2(r, 0.0);
    rmax[m] = r;
    const bool stalled = !(r < 0.25 * rprev[m]);
    rprev[m] = r;
    if (!(r > delta2 * b32n2[m]) || !(r > tol2 * bn2[m]) || its[m] >= max_iter || stalled) upd64[m] = 1;
    upd[m] = 0;
}
// two levels: every reliable update goes to the FP64 level
__global__ void k_c16_promote(int M, int32_t *upd, int32_t *upd64)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M || !upd[m]) return;
    upd64[m] = 1;
    upd[m] = 0;
}
// after the FP64 true residual: retire converged systems, else restart the
// middle system (right-hand side = that residual) and the iterated residual
__global__ void k_c16_outer(int M, double2 *sc, const double *bn2, double *b32n2, double tol2, int max_iter,
                            const int32_t *its, int32_t *alive, int32_t *upd64, double *rmax, double *rprev,
                            int32_t *nout)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M || !upd64[m]) return;
    ++nout[m];
    const double r = sc[8L * m + 5].x;
    if (!isfinite(r) || r <= tol2 * bn2[m] || its[m] >= max_iter) alive[m] = 0;
    sc[8L * m] = make_double2(r, 0.0);
    rmax[m] = r;
    b32n2[m] = r;
    rprev[m] = r;
}
__global__ void k_c16_clear(int M, int32_t *upd64)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < M) upd64[m] = 0;
}

// the middle level hands a system to the FP64 level once its residual fell
// by this factor (FP32 arithmetic resolves the middle system several orders
// further, so the FP64 updates stay rare)
constexpr double OUTER_DELTA = 1e-4;
// the FP16 steps hand over to the middle (or outer) level once the iterated
// residual fell by this factor.  Each middle update costs an FP32 Dhat and a
// conversion, about half a CG step; at the 32^4 workload 0.03 keeps the CG
// iteration count of 0.1 (0.02 and 0.01 add iterations) with fewer updates:
// 931 vs 980 ms per estimate (0.05: 961 ms)
constexpr double RELIABLE_DELTA_F16 = 0.03;

// the FP16 steps' x updates wait for up to this many steps and then run as
// one pass over x (x is read and written once instead of once per step)
constexpr int XDEFER = 4;

// Even-odd CG on the normal equations with FP16 storage (4^4 blocks, SU(3)
// links), the system and FP64 residual of cgne_eo.  Inner level: CG steps
// on FP16 vectors (E16 layout, per-block scales) with the FP16 stencil and
// FP32 arithmetic; the solution increment accumulates in FP32.  Three
// levels (middle = F32): when the iterated residual has fallen by
// RELIABLE_DELTA_F16, it is replaced by the FP32 true residual of the middle
// system Dhat x32 = bh32; when that has fallen by OUTER_DELTA (or reached the
// tolerance), x32 is folded into the FP64 solution, the FP64 true residual
// becomes the middle system's new right-hand side and x32 restarts at zero.
// Two levels (middle = F64): every reliable update is the FP64 one.  The
// search direction is kept across updates (Sleijpen and van der Vorst).
static wdr_status cgne_eo16(wdr_ctx *c, int M, const GaugeTab &U, double kappa, const wdr_solver_params &sp,
                            double tol, const double2 *b, double2 *x, std::vector<Stats> &st, hipStream_t s)
{
    const auto &g = c->g;
    if (!U.e16.tab || !e16_geometry(g)) {
        set_error("the FP16 even-odd CG needs SU(3) links and 4^4 blocks in a 2-colourable checkerboard");
        return WDR_EINVAL;
    }
    const bool three = sp.middle == WDR_F32;
    const long n = field_n(c), total = n * M;
    const size_t fb = field_bytes(c, WDR_F64) * M, f32 = field_bytes(c, WDR_F32) * M, fe = e16_field_bytes(g, M);
    // the x updates of up to XDEFER steps wait for one pass over x (w of each
    // of those steps kept, in its own buffer)
    const int ue = sp.update_every, K = std::min(ue, XDEFER);
    const size_t fes = (fe + 255) & ~(size_t)255;  // buffer stride, aligned for the 16 B loads
    Work wx(c, fes * (K - 1) + 64), alw(c, sizeof(float) * XDEFER * M);
    Work bhw(c, fb), r64w(c, fb), t64w(c, fb), o64w(c, fb), x32w(c, f32), b32w(c, f32), d32w(c, f32), t32w(c, f32),
        pw(c, fe), ww(c, fe), qw(c, fe), rw(c, fe), tw(c, fe), scal(c, sizeof(double2) * 8 * M),
        red(c, sizeof(double) * std::max<long>(red_scratch(M), 2L * g.nblk * M)),
        ctl(c, 4 * sizeof(double) * M + 6 * sizeof(int32_t) * M), lw(c, sizeof(int32_t) * M);
    FlagPoll poll(c, M);
    if (!bhw.ok() || !r64w.ok() || !t64w.ok() || !o64w.ok() || !x32w.ok() || !b32w.ok() || !d32w.ok() || !t32w.ok() ||
        !pw.ok() || !ww.ok() || !qw.ok() || !rw.ok() || !tw.ok() || !scal.ok() || !red.ok() || !ctl.ok() ||
        !lw.ok() || !poll.ok || !wx.ok() || !alw.ok())
        return WDR_ENOMEM;
    double2 *bh = bhw.as<double2>(), *r64 = r64w.as<double2>(), *t64 = t64w.as<double2>(), *o64 = o64w.as<double2>();
    float2 *x32 = x32w.as<float2>(), *b32 = b32w.as<float2>(), *d32 = d32w.as<float2>(), *t32 = t32w.as<float2>();
    const E16 P = e16_field(g, M, pw.as<void>()), Q = e16_field(g, M, qw.as<void>()),
              R = e16_field(g, M, rw.as<void>()), T = e16_field(g, M, tw.as<void>());
    E16 Wk[XDEFER];
    E16c Wc[XDEFER];
    for (int j = 0; j < K; ++j) {
        Wk[j] = e16_field(g, M, j == 0 ? ww.as<void>() : static_cast<void *>(wx.as<char>() + fes * (j - 1)));
        Wc[j] = cref(Wk[j]);
    }
    float *alphas = alw.as<float>();
    double2 *sc = scal.as<double2>();
    double *part = red.as<double>();
    double *bn2 = ctl.as<double>(), *rmax = bn2 + M, *b32n2 = rmax + M, *rprev = b32n2 + M;
    int32_t *alive = reinterpret_cast<int32_t *>(rprev + M), *upd = alive + M, *upd64 = upd + M, *its = upd64 + M;
    int32_t *nmid = its + M, *nout = nmid + M;  // middle and outer updates per system
    const Links<double> U64 = U.u64;
    Links<double> U64n = U.u64;
    U64n.kneg = 1;
    U64n.cmode = CLOV_NONE;  // the diagonal input b_e enters as it is
    const Links<float> U32 = U.u32;
    const Links16 U16 = U.e16;
    // with a clover term: A_oo^-1 on the odd halves, A_ee on the diagonal (FP32 blocks)
    const bool clov = U.u64.ctab != nullptr;
    const float *const *C32 = U.u32.ctab;
    const float kf = (float)kappa;
    const Sys all = all_sys(c, M);
    Sys sa{M, alive, n}, su{M, upd, n}, s64{M, upd64, n};
    sa.hs = su.hs = s64.hs = even_shift(g);
    std::vector<int32_t> live;
    int launch_m = M;
    const unsigned nbm = nb64(M);
    const int G = g.nblk;

    // bh = [b_e + k H_eo A_oo^-1 b_o; 0]; x = 0; r64 = bh; every system starts an outer update
    launch_zero<double>(x, total, s);
    launch_zero<double>(bh, total, s);
    launch_zero<double>(t64, total, s);
    if (clov) launch_clover_mul<double>(g, all, U.u64.ctab, 1, 1, b, o64, s);  // odd sites of o64
    launch_dslash<double>(g, all, U64n, HOPS_ALL, 0, 0, clov ? o64 : b, b, bh, -kappa, 0, g.nblk, s);
    launch_norm2<double>(all, b, red.as<double>(), sc + 5, 8, s);
    k_cgm_init<<<nbm, 64, 0, s>>>(M, sc, bn2, rmax, alive, upd, its);  // |b|^2 of the full system
    launch_zero<float>(x32, total, s);
    launch_norm2<double>(sa, bh, red.as<double>(), sc, 8, s);          // |bh|^2 (even sites)
    launch_r16_from64(g, all, bh, b32, x32, R, s);
    launch_p16(g, all, sc, 1, cref(R), P, s);
    k_cgm_rmax<<<nbm, 64, 0, s>>>(M, sc, rmax);
    k_cgm_rmax<<<nbm, 64, 0, s>>>(M, sc, b32n2);
    k_cgm_rmax<<<nbm, 64, 0, s>>>(M, sc, rprev);
    k_c16_clear<<<nbm, 64, 0, s>>>(M, upd64);
    k_c16_clear<<<nbm, 64, 0, s>>>(M, nmid);
    k_c16_clear<<<nbm, 64, 0, s>>>(M, nout);
    const E16c none{nullptr, nullptr};
    auto period = [&](hipStream_t q) {
        for (int i = 0; i < ue; ++i) {
            // w = Dhat^+ p (with |w|^2), q = Dhat w, r -= alpha q, p = r + beta p;
            // x += alpha w for the last K steps at once (before the period's end)
            const int j = i % K;
            const E16 W = Wk[j];
            launch_eo16(g, sa, U16, -1.f, -kf, 1, 1, cref(P), none, T, nullptr, q, C32, CLOV_INV);
            launch_eo16(g, sa, U16, 1.f, kf, 0, 1, cref(T), cref(P), W, part, q, C32, CLOV_DIAG);
            launch_final(sa, part, G, sc + 1, 8, q);
            launch_eo16(g, sa, U16, -1.f, -kf, 1, 0, cref(W), none, T, nullptr, q, C32, CLOV_INV);
            launch_eo16(g, sa, U16, 1.f, kf, 0, 0, cref(T), cref(W), Q, nullptr, q, C32, CLOV_DIAG);
            launch_xr16(g, sa, sc, nullptr, alphas + (long)j * M, cref(W), cref(Q), R, part, q);
            launch_final(sa, part, G, sc + 3, 8, q);
            k_cgm_beta<<<nbm, 64, 0, q>>>(M, sc, RELIABLE_DELTA_F16 * RELIABLE_DELTA_F16, sp.max_iter, alive, rmax,
                                          upd, its);
            launch_p16(g, sa, sc, 0, cref(R), P, q);
            if (j == K - 1 || i == ue - 1) launch_x16_flush(g, sa, alphas, M, Wc, j + 1, x32, q);
        }
        if (three) {
            // middle: r = bh32 - Dhat x32 in FP32 for the flagged systems
            apply_dhat<float>(g, su, U32, kf, 0, x32, t32, d32, q);
            launch_r16_from32(g, su, b32, d32, R, part, q);
            launch_final(su, part, G, sc + 6, 8, q);
            k_c16_mid<<<nbm, 64, 0, q>>>(M, sc, bn2, b32n2, tol * tol, OUTER_DELTA * OUTER_DELTA, sp.max_iter, its,
                                         upd, upd64, rmax, rprev, nmid);
        } else {
            k_c16_promote<<<nbm, 64, 0, q>>>(M, upd, upd64);
        }
        // outer: x += x32, r64 = bh - Dhat x in FP64; the middle system restarts from r64
        launch_add_to64<float>(s64, x32, x, q);
        apply_dhat<double>(g, s64, U64, kappa, 0, x, o64, t64, q);
        launch_sub_norm(s64, bh, t64, r64, red.as<double>(), sc + 5, 8, q);
        k_c16_outer<<<nbm, 64, 0, q>>>(M, sc, bn2, b32n2, tol * tol, sp.max_iter, its, alive, upd64, rmax, rprev,
                                       nout);
        launch_r16_from64(g, s64, r64, b32, x32, R, q);
        k_c16_clear<<<nbm, 64, 0, q>>>(M, upd64);
    };
    PeriodGraph pg(s);
    for (int pt = 0;; ++pt) {
        if (sp.graph) {
            if (!pg.exec) {
                const wdr_status cs = pg.capture(c, period);
                if (cs != WDR_OK) return cs;
            }
            WDR_HIP(hipGraphLaunch(pg.exec, s));
        } else {
            period(s);
        }
        poll.post(alive, pt & 1, s);
        if (pt > 0) {
            if (poll.none((pt - 1) & 1)) break;
            const int32_t *fl = poll.slot((pt - 1) & 1);
            int cnt = 0;
            for (int m = 0; m < M; ++m) cnt += fl[m] != 0;
            if (2 * cnt <= launch_m) {
                live.clear();
                for (int m = 0; m < M; ++m)
                    if (fl[m]) live.push_back(m);
                WDR_HIP(hipMemcpyAsync(lw.as<void>(), live.data(), live.size() * sizeof(int32_t),
                                       hipMemcpyHostToDevice, s));
                launch_m = cnt;
                sa.list = su.list = s64.list = lw.as<int32_t>();
                sa.count = su.count = s64.count = cnt;
                pg.reset();
            }
        }
    }
    // x_o = A_oo^-1 (b_o + k H_oe x_e), written into the odd sites of x in
    // place: the launch reads only the even sites of x
    Links<double> U64i = U64n;
    U64i.cmode = CLOV_INV;
    launch_dslash<double>(g, all, U64i, HOPS_ALL, 1, 0, x, b, x, -kappa, 0, g.nblk, s);

    std::vector<double> hbn2(M), rn2;
    std::vector<int32_t> hits(M), hmid(M), hout(M);
    WDR_HIP(hipMemcpyAsync(hbn2.data(), bn2, sizeof(double) * M, hipMemcpyDeviceToHost, s));
    WDR_HIP(hipMemcpyAsync(hits.data(), its, sizeof(int32_t) * M, hipMemcpyDeviceToHost, s));
    WDR_HIP(hipMemcpyAsync(hmid.data(), nmid, sizeof(int32_t) * M, hipMemcpyDeviceToHost, s));
    WDR_HIP(hipMemcpyAsync(hout.data(), nout, sizeof(int32_t) * M, hipMemcpyDeviceToHost, s));
    read_x(sc + 5, M, 8, rn2, s);
    st.assign(M, Stats());
    bool ok = true;
    // compulsory bytes per system (V sites): setup and final step, then per
    // CG step (four FP16 halves, the x / r update, the p update), per middle
    // update (FP32 Dhat x32, the residual into FP16) and per outer update
    // (x += x32, FP64 Dhat x, r64 = bh - Dhat x, the restart)
    const double V = g.V, H = V / 2;
    const double setup = 3 * V * spin_b<double>() + half_b<double>(V, true) + V * spin_b<double>() +
                         V * spin_b<float>() + H * spin_b<double>() + H * (spin_b<double>() + 2 * spin_b<float>() + 48) +
                         H * 96 + V * spin_b<double>() + half_b<double>(V, true) + 3 * V * spin_b<double>();
    // the x / r update (q in, r in and out) and the p update, then per step
    // the share of the deferred x pass (w in, x32 in and out every K steps)
    const double half16 = H * 96 + V * 96,
                 step = 4 * half16 + 2 * H * 48 + H * 144 + H * 144 + H * (48 + 2 * spin_b<float>() / K);
    const double mid = half_b<float>(V, false) + half_b<float>(V, true) + H * (2 * spin_b<float>() + 48);
    const double outer = H * (spin_b<float>() + 2 * spin_b<double>()) + half_b<double>(V, false) +
                         half_b<double>(V, true) + 3 * H * spin_b<double>() +
                         H * (spin_b<double>() + 2 * spin_b<float>() + 48);
    // the clover blocks of every output site of the four halves, the middle
    // and the outer Dhat (FP32 in the steps and the middle, FP64 outside)
    const double cl_step = clov ? 4 * H * clov_b<float>() : 0, cl_mid = clov ? 2 * H * clov_b<float>() : 0,
                 cl_out = clov ? 2 * H * clov_b<double>() : 0;
    double bytes = 0;
    for (int m = 0; m < M; ++m) {
        bytes += setup + hits[m] * (step + cl_step) + hmid[m] * (mid + cl_mid) + hout[m] * (outer + cl_out);
        st[m].iters = hits[m];
        st[m].total = hits[m];
        st[m].rel = rel_resid(rn2[m], hbn2[m]);
        st[m].converged = st[m].rel <= tol;
        ok = ok && st[m].converged;
    }
    add_traffic(bytes);
    WDR_HIP(hipGetLastError());
    if (!ok) {
        const Stats sm = summarize(st);
        set_error("CGNE (FP16 inner) stopped at " + std::to_string(sm.iters) + " iterations, relative residual " +
                  std::to_string(sm.rel));
        return WDR_ENOCONV;
    }
    return WDR_OK;
}

wdr_status solve64(wdr_ctx *c, int M, const GaugeTab &U, double kappa, const wdr_solver_params &sp, double tol,
                   const double2 *b, double2 *x, std::vector<Stats> &st, hipStream_t s)
{
    if (sp.solver == WDR_SOLVER_CGNE) {
        if (sp.inner == WDR_F16) return cgne_eo16(c, M, U, kappa, sp, tol, b, x, st, s);
        return sp.inner == WDR_F64 ? cgne_eo<double>(c, M, U, kappa, sp, tol, b, x, st, s)
                                   : cgne_eo<float>(c, M, U, kappa, sp, tol, b, x, st, s);
    }
    return fgcr(c, M, U, kappa, sp, tol, b, x, st, s);
}

// ------------------------------------------------------------ block solves

// the relative residual each round of the clover block solves asks of its
// even-odd CG (over all blocks of the colour at once); two rounds reach the
// usual block tolerances
constexpr double BLOCK_EO_TOL = 1e-7;

// Dirichlet block solves with the clover term and an F64 / F32 inner level
// (the 6 x 6 blocks per site in those precisions do not fit beside the
// block MR's fields in LDS; the FP16 block MR keeps them as FP16): defect
// correction in FP64 around the even-odd CGNE of the block operator D_b = A -
// kappa H_in on the blocks of the colour, all of them one block-diagonal
// system.  Each round solves D_b d = r to a relative residual max(tol / 2,
// BLOCK_EO_TOL) with sp.inner iterations and FP64 reliable updates, adds d
// to x and forms the
// FP64 residual r = b - D_b x block by block; as in the MR rounds, the worst
// block ratio |r_b| / |b_b| decides.  Systems that have converged get r = 0,
// which their next CG ends at once.
static wdr_status block_solve_clover(wdr_ctx *c, int M, const GaugeTab &U, double kappa, int colour,
                                     const wdr_solver_params &sp, double tol, const double2 *b, double2 *x,
                                     std::vector<Stats> &st, hipStream_t s)
{
    const auto &g = c->g;
    int slot0, ns;
    colour_slots(c, colour, slot0, ns);
    const long n = field_n(c), total = n * M;
    const size_t fb = field_bytes(c, WDR_F64) * M;
    Work rw(c, fb), tw(c, fb), dw(c, fb), nrm(c, 2 * sizeof(double) * g.nblk * M);
    Work ctl(c, sizeof(double) * M + 2 * sizeof(int32_t) * M);
    if (!rw.ok() || !tw.ok() || !dw.ok() || !nrm.ok() || !ctl.ok()) return WDR_ENOMEM;
    double2 *r = rw.as<double2>(), *t = tw.as<double2>(), *d = dw.as<double2>();
    double *worst = ctl.as<double>();
    int32_t *alive = reinterpret_cast<int32_t *>(worst + M), *its = alive + M;
    const Sys all = all_sys(c, M), sa{M, alive, n};
    launch_zero<double>(x, total, s);
    launch_convert<double, double>(all, b, r, s);
    launch_keep_slots(g, all, r, slot0, ns, s);
    double *bn = nrm.as<double>(), *rn = bn + (size_t)g.nblk * M;
    launch_slot_norm2(g, all, r, bn, slot0, ns, s);
    k_block_init<<<M, BC_NT, 0, s>>>(g.nblk, slot0, ns, bn, alive, its, worst);
    Links<double> Ud = U.u64;
    Ud.cmode = CLOV_DIAG;
    EoOp op;
    op.hops = HOPS_IN;
    op.slot0 = slot0;
    op.ns = ns;
    const double tin = std::max(0.5 * tol, BLOCK_EO_TOL);
    std::vector<int32_t> halive(M);
    std::vector<long> inner(M, 0);
    int rounds = 0;
    for (int round = 0; round < 40; ++round) {
        k_zero_dead<<<nb256(total), 256, 0, s>>>(alive, n, total, r);
        std::vector<Stats> si;
        const wdr_status e = sp.inner == WDR_F64 ? cgne_eo<double>(c, M, U, kappa, sp, tin, r, d, si, s, op)
                                                 : cgne_eo<float>(c, M, U, kappa, sp, tin, r, d, si, s, op);
        if (e != WDR_OK && e != WDR_ENOCONV) return e;
        for (int m = 0; m < M; ++m) inner[m] += si[m].total;
        // x += d, r = b - D_b x and its norm per block on the selected blocks
        launch_add_to64<double>(sa, d, x, s);
        launch_dslash<double>(g, sa, Ud, HOPS_IN, -1, 0, x, x, t, kappa, slot0, ns, s);
        launch_block_resid_norm(g, sa, b, t, r, rn, slot0, ns, s);
        k_block_check<<<M, BC_NT, 0, s>>>(g.nblk, slot0, ns, bn, rn, tol * tol, alive, its, worst);
        WDR_HIP(hipMemcpyAsync(halive.data(), alive, sizeof(int32_t) * M, hipMemcpyDeviceToHost, s));
        WDR_HIP(hipStreamSynchronize(s));
        ++rounds;
        bool any = false;
        for (int m = 0; m < M; ++m) any = any || halive[m];
        if (!any) break;
    }
    std::vector<double> hworst(M);
    std::vector<int32_t> hits(M);
    WDR_HIP(hipMemcpyAsync(hworst.data(), worst, sizeof(double) * M, hipMemcpyDeviceToHost, s));
    WDR_HIP(hipMemcpyAsync(hits.data(), its, sizeof(int32_t) * M, hipMemcpyDeviceToHost, s));
    WDR_HIP(hipStreamSynchronize(s));
    // compulsory bytes outside the CG (which counts its own): setup, then
    // per round the clear, x += d, D_b x on the selected blocks (with their
    // clover blocks) and r = b - D_b x with its norms
    const double V = g.V, Vs = (double)ns * g.Vb, sb = spin_b<double>();
    double lin = 0;
    for (int mu = 0; mu < 4; ++mu) lin += (double)(g.B[mu] - 1) / g.B[mu];
    const double setup = V * 4 * sb + Vs * sb;
    const double round_b = V * sb + V * 3 * sb + Vs * (2 * sb + lin * 96.0 + clov_b<double>()) + Vs * 3 * sb;
    bool ok = true;
    st.assign(M, Stats());
    double bytes = 0;
    for (int m = 0; m < M; ++m) {
        bytes += setup + rounds * round_b;
        st[m].iters = hits[m];
        st[m].total = inner[m];
        st[m].rel = std::sqrt(hworst[m]);
        st[m].converged = st[m].rel <= tol;
        ok = ok && st[m].converged;
    }
    add_traffic(bytes);
    WDR_HIP(hipGetLastError());
    if (!ok) {
        set_error("block solve stopped at relative residual " + std::to_string(summarize(st).rel));
        return WDR_ENOCONV;
    }
    return WDR_OK;
}

wdr_status block_solve64(wdr_ctx *c, int M, const GaugeTab &U, double kappa, int colour, const wdr_solver_params &sp,
                         double tol, const double2 *b, double2 *x, std::vector<Stats> &st, hipStream_t s)
{
    // the clover term: CG rounds for F64 / F32 inner levels, the FP16 block
    // MR (with the blocks of A in LDS) for F16
    if (U.u64.ctab && sp.inner != WDR_F16) return block_solve_clover(c, M, U, kappa, colour, sp, tol, b, x, st, s);
    const bool clov = U.u64.ctab != nullptr;
    Links<double> Ud = U.u64;  // D_b with its diagonal A where the term is present
    if (clov) Ud.cmode = CLOV_DIAG;
    const auto &g = c->g;
    int slot0, ns;
    colour_slots(c, colour, slot0, ns);
    const long n = field_n(c);
    const size_t fb = field_bytes(c, WDR_F64) * M, fb32 = field_bytes(c, WDR_F32) * M;
    Work rw(c, fb), tw(c, fb), d32(c, fb32), r32(c, fb32), d64(c, fb), nrm(c, 2 * sizeof(double) * g.nblk * M);
    Work ctl(c, sizeof(double) * M + 2 * sizeof(int32_t) * M);
    FlagPoll poll(c, M);
    if (!rw.ok() || !tw.ok() || !d32.ok() || !r32.ok() || !d64.ok() || !nrm.ok() || !ctl.ok() || !poll.ok)
        return WDR_ENOMEM;
    double2 *r = rw.as<double2>(), *t = tw.as<double2>();
    double *worst = ctl.as<double>();
    int32_t *alive = reinterpret_cast<int32_t *>(worst + M), *its = alive + M;
    const Sys all = all_sys(c, M);
    launch_zero<double>(x, n * M, s);
    launch_convert<double, double>(all, b, r, s);
    launch_keep_slots(g, all, r, slot0, ns, s);
    // the MR kernels write only the selected slots: the rest of d stays zero
    if (sp.inner == WDR_F32) launch_zero<float>(d32.as<float2>(), n * M, s);
    if (sp.inner == WDR_F64) launch_zero<double>(d64.as<double2>(), n * M, s);
    double *bn = nrm.as<double>(), *rn = bn + (size_t)g.nblk * M;
    launch_slot_norm2(g, all, r, bn, slot0, ns, s);
    k_block_init<<<M, BC_NT, 0, s>>>(g.nblk, slot0, ns, bn, alive, its, worst);
    const int nmr = sp.block_mr_steps;
    const Sys sa{M, alive, n};
    std::unique_ptr<H16Work> r16, d16;
    if (sp.inner == WDR_F16) {
        wdr_status e = need16(U);
        if (e != WDR_OK) return e;
        r16.reset(new H16Work(c, M));
        d16.reset(new H16Work(c, M));
        if (!r16->ok() || !d16->ok()) return WDR_ENOMEM;
        launch_zero_h16(g, all, d16->f(), s);
    }
    bool fused = true;
    // FP16 rounds after the first: the previous round's fused end already
    // left r in FP16 (round16), and the FP64 r is not kept
    bool round16 = false;
    for (int round = 0; round < 40; ++round) {
        bool have_norms = false;
        if (sp.inner == WDR_F64) {
            launch_block_mr<double>(g, sa, U.u64, r, d64.as<double2>(), kappa, nmr, slot0, ns, s);
            launch_add_to64<double>(sa, d64.as<double2>(), x, s);
        } else if (sp.inner == WDR_F16) {
            if (!round16) launch_to_h16<double>(g, sa, r, r16->f(), slot0, ns, s);
            if (!launch_mr_h16(1, g, sa, U.u16, r16->cf(), d16->f(), (float)kappa, nmr, slot0, ns, s, U.u32.ctab))
                return need16(GaugeTab{});
            // x += d, r = b - D_b x with its block norms and its FP16 form
            // (the fused end has no clover form)
            round16 = launch_block_round16(g, sa, Ud, d16->cf(), x, b, r16->f(), rn, kappa, slot0, ns, s);
            have_norms = round16;
            if (!round16) launch_from_h16(g, sa, d16->cf(), x, 1, slot0, ns, s);
        } else {
            launch_convert<float, double>(sa, r, r32.as<float2>(), s);
            launch_block_mr<float>(g, sa, U.u32, r32.as<float2>(), d32.as<float2>(), (float)kappa, nmr, slot0, ns, s);
            launch_add_to64<float>(sa, d32.as<float2>(), x, s);
        }
        // r = b - D_b x and its norm per block on the selected blocks (r stays
        // zero elsewhere: nothing below writes other blocks of r)
        if (!have_norms) {
            fused = launch_block_residual(g, sa, Ud, x, b, r, kappa, slot0, ns, s);
            if (!fused) launch_dslash<double>(g, sa, Ud, HOPS_IN, -1, 0, x, x, t, kappa, slot0, ns, s);
            launch_block_resid_norm(g, sa, b, fused ? nullptr : t, r, rn, slot0, ns, s);
        }
        k_block_check<<<M, BC_NT, 0, s>>>(g.nblk, slot0, ns, bn, rn, tol * tol, alive, its, worst);
        poll.post(alive, round & 1, s);
        // round is queued; stop once round - 1 left no system alive
        if (round > 0 && poll.none((round - 1) & 1)) break;
    }
    std::vector<double> hworst(M);
    std::vector<int32_t> hits(M);
    WDR_HIP(hipMemcpyAsync(hworst.data(), worst, sizeof(double) * M, hipMemcpyDeviceToHost, s));
    WDR_HIP(hipMemcpyAsync(hits.data(), its, sizeof(int32_t) * M, hipMemcpyDeviceToHost, s));
    WDR_HIP(hipStreamSynchronize(s));
    bool ok = true;
    st.assign(M, Stats());
    // compulsory bytes per system: setup, then per round the block MR (its
    // right-hand side, result and in-block links) with its conversions, the
    // FP64 residual b - D_b x on the selected blocks and its norm
    const double V = g.V, Vs = (double)ns * g.Vb;
    double lin = 0;  // in-block links per site
    for (int mu = 0; mu < 4; ++mu) lin += (double)(g.B[mu] - 1) / g.B[mu];
    const double ps = sp.inner == WDR_F64 ? spin_b<double>() : sp.inner == WDR_F32 ? spin_b<float>() : 48.0;
    const double pl = sp.inner == WDR_F64 ? 96.0 : sp.inner == WDR_F32 ? 48.0 : 24.0;  // one two-row link
    double setup = V * (4 * spin_b<double>()) + Vs * spin_b<double>();
    setup += sp.inner == WDR_F16 ? V * 48 : V * ps;
    double round_b = Vs * (2 * ps + lin * pl + (clov ? clov_b<float>() : 0.0));
    if (sp.inner == WDR_F16 && round16)  // the fused end: d, x, b, links in; x, r16 out
        round_b += Vs * (48 + 3 * spin_b<double>() + lin * 96.0 + 48);
    else if (sp.inner == WDR_F16)
        round_b += Vs * (spin_b<double>() + 48) + Vs * (48 + 2 * spin_b<double>());
    else
        round_b += V * (ps + spin_b<double>()) * (sp.inner == WDR_F32 ? 1 : 0) + V * (ps + 2 * spin_b<double>());
    if (!(sp.inner == WDR_F16 && round16))
        round_b += fused ? Vs * (4 * spin_b<double>() + lin * 96.0)
                         : Vs * (2 * spin_b<double>() + lin * 96.0 + (clov ? clov_b<double>() : 0.0)) +
                               Vs * 3 * spin_b<double>();
    double bytes = 0;
    for (int m = 0; m < M; ++m) {
        bytes += setup + hits[m] * round_b;
        st[m].iters = hits[m];
        st[m].total = hits[m];
        st[m].rel = std::sqrt(hworst[m]);
        st[m].converged = st[m].rel <= tol;
        ok = ok && st[m].converged;
    }
    add_traffic(bytes);
    WDR_HIP(hipGetLastError());
    if (!ok) {
        set_error("block solve stopped at relative residual " + std::to_string(summarize(st).rel));
        return WDR_ENOCONV;
    }
    return WDR_OK;
}

// ------------------------------------------------------------ Schur complement

wdr_status schur64(wdr_ctx *c, int M, const GaugeTab &U, double kappa, const wdr_solver_params &sp,
                   const double2 *in, double2 *out, std::vector<Stats> &st, hipStream_t s)
{
    const auto &g = c->g;
    const long n = field_n(c);
    const size_t fb = field_bytes(c, WDR_F64) * M;
    Work t1(c, fb), t2(c, fb);
    if (!t1.ok() || !t2.ok()) return WDR_ENOMEM;
    int b0, bn, w0, wn;
    colour_slots(c, 0, b0, bn);
    colour_slots(c, 1, w0, wn);
    const Sys all = all_sys(c, M);
    std::vector<Stats> s1, s2;
    // D_wb in (white sites; cross hops from black)
    launch_zero<double>(t1.as<double2>(), n * M, s);
    launch_dslash<double>(g, all, U.u64, HOPS_CROSS, -1, 0, in, nullptr, t1.as<double2>(), kappa, w0, wn, s);
    wdr_status e = block_solve64(c, M, U, kappa, 1, sp, sp.block_tol, t1.as<double2>(), t2.as<double2>(), s1, s);
    if (e != WDR_OK && e != WDR_ENOCONV) return e;
    const wdr_status first = e;
    // D_bw (...) on black sites
    launch_zero<double>(t1.as<double2>(), n * M, s);
    launch_dslash<double>(g, all, U.u64, HOPS_CROSS, -1, 0, t2.as<double2>(), nullptr, t1.as<double2>(), kappa, b0, bn,
                          s);
    e = block_solve64(c, M, U, kappa, 0, sp, sp.block_tol, t1.as<double2>(), t2.as<double2>(), s2, s);
    if (e != WDR_OK && e != WDR_ENOCONV) return e;
    if (e == WDR_OK) e = first;
    st.assign(M, Stats());
    for (int m = 0; m < M; ++m) {
        st[m].iters = s2[m].iters;
        st[m].total = s1[m].total + s2[m].total;
        st[m].rel = std::max(s1[m].rel, s2[m].rel);
        st[m].converged = s1[m].converged && s2[m].converged;
    }
    // out = in - t2 on black, zero on white
    launch_sub(all, in, t2.as<double2>(), out, s);
    launch_keep_slots(g, all, out, b0, bn, s);
    // compulsory bytes of the kernels above (the block solves count their own):
    // two clears, two cross-block hops onto one colour (its sites, the
    // neighbours across the faces, the crossing links), the difference, the clear
    double face = 1, cross = 0;
    for (int mu = 0; mu < 4; ++mu) {
        face *= g.B[mu] > 2 ? (double)(g.B[mu] - 2) / g.B[mu] : 0.0;
        cross += 2.0 / g.B[mu];
    }
    const double V = g.V, sb = spin_b<double>();
    add_traffic(M * (2 * V * sb + 2 * (V / 2) * (sb + (1 - face) * sb + cross * 96.0) + V * 3 * sb + V * sb));
    return e;
}

}  // namespace wdr
