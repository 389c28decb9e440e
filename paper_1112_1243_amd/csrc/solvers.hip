// Solver drivers: Schwarz preconditioner, flexible GCR, CG on the normal
// equations, Dirichlet block solves and the Schur complement (paper Sec. 3,
// eqs. domdec and ddfactor; Sec. 4, "one inversion for each factor").
//
// Outer iterations are FP64 with FP64 true residuals and deterministic FP64
// reductions; the Schwarz preconditioner and the inner block MR run in
// sp.inner (FP32 by default).  Scalars of the Krylov recursions live in
// device memory; the host reads one residual norm per iteration to decide
// convergence.
#include <chrono>
#include <cmath>
#include <vector>

#include "runtime.h"

namespace wdr {
namespace {

// ------------------------------------------------------------ small kernels

// CG scalars in c->scal:  [0] rr, [1] ww, [2] alpha, [3] rr_new, [4] beta
__global__ void k_cg_alpha(double2 *sc)
{
    const double ww = sc[1].x;
    sc[2] = make_double2(ww > 0 ? sc[0].x / ww : 0.0, 0.0);
}
__global__ void k_cg_beta(double2 *sc)
{
    const double rr = sc[0].x;
    sc[4] = make_double2(rr > 0 ? sc[3].x / rr : 0.0, 0.0);
    sc[0] = sc[3];
}
// x += alpha w, r -= alpha q, y += alpha p (y optional)
__global__ __launch_bounds__(256) void k_cg_update(const double2 *sc, double2 *x, const double2 *w, double2 *r,
                                                   const double2 *q, double2 *y, const double2 *p, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double a = sc[2].x;
    double2 xi = x[i], wi = w[i], ri = r[i], qi = q[i];
    x[i] = make_double2(xi.x + a * wi.x, xi.y + a * wi.y);
    r[i] = make_double2(ri.x - a * qi.x, ri.y - a * qi.y);
    if (y) {
        double2 yi = y[i], pi = p[i];
        y[i] = make_double2(yi.x + a * pi.x, yi.y + a * pi.y);
    }
}
// p = r + beta p
__global__ __launch_bounds__(256) void k_cg_p(const double2 *sc, const double2 *r, double2 *p, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double b = sc[4].x;
    double2 ri = r[i], pi = p[i];
    p[i] = make_double2(ri.x + b * pi.x, ri.y + b * pi.y);
}

// zero the slots outside [slot0, slot0 + n) of a FP64 field
void zero_outside(wdr_ctx *c, double2 *f, int slot0, int n, hipStream_t s)
{
    const long per = 12L * c->g.Vb;
    if (slot0 > 0) launch_zero<double>(f, per * slot0, s);
    const int end = slot0 + n;
    if (end < c->g.nblk) launch_zero<double>(f + per * end, per * (c->g.nblk - end), s);
}

double read_scalar(wdr_ctx *c, int idx, hipStream_t s)
{
    double2 v;
    hipMemcpyAsync(&v, c->scal + idx, sizeof(double2), hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
    return v.x;
}

inline unsigned nb256(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void apply_D64(wdr_ctx *c, GaugeView U, double kappa, const double2 *in, double2 *out, hipStream_t s)
{
    launch_dslash<double>(c->g, HOPS_ALL, -1, 0, U.u64, in, in, out, kappa, 0, c->g.nblk, s);
}

// ------------------------------------------------------------ SAP

template <typename T>
static void sap_run(wdr_ctx *c, const typename C2<T>::type *U, T kappa, int ncy, int nmr,
                    const typename C2<T>::type *eta, typename C2<T>::type *x, hipStream_t s)
{
    launch_zero<T>(x, field_n(c), s);
    int b0, bn, w0, wn;
    colour_slots(c, 0, b0, bn);
    colour_slots(c, 1, w0, wn);
    for (int cy = 0; cy < ncy; ++cy) {
        launch_sap_colour<T>(c->g, U, eta, x, kappa, nmr, b0, bn, s);
        launch_sap_colour<T>(c->g, U, eta, x, kappa, nmr, w0, wn, s);
    }
}

wdr_status sap64(wdr_ctx *c, GaugeView U, double kappa, const wdr_solver_params &sp, const double2 *in,
                 double2 *out, hipStream_t s)
{
    if (sp.inner == WDR_F64) {
        sap_run<double>(c, U.u64, kappa, sp.sap_cycles, sp.mr_steps, in, out, s);
        return WDR_OK;
    }
    Work e(c, field_bytes(c, WDR_F32)), x(c, field_bytes(c, WDR_F32));
    if (!e.ok() || !x.ok()) return WDR_ENOMEM;
    launch_convert<float, double>(in, e.as<float2>(), field_n(c), s);
    sap_run<float>(c, U.u32, (float)kappa, sp.sap_cycles, sp.mr_steps, e.as<float2>(), x.as<float2>(), s);
    launch_convert<double, float>(x.as<float2>(), out, field_n(c), s);
    return WDR_OK;
}

// ------------------------------------------------------------ FGCR + SAP

static wdr_status fgcr(wdr_ctx *c, GaugeView U, double kappa, const wdr_solver_params &sp, double tol,
                       const double2 *b, double2 *x, Stats &st, hipStream_t s)
{
    const long n = field_n(c);
    const size_t fb = field_bytes(c, WDR_F64);
    const int nkv = sp.restart;
    std::vector<Work *> phi, chi;
    for (int j = 0; j < nkv; ++j) {
        phi.push_back(new Work(c, fb));
        chi.push_back(new Work(c, fb));
    }
    Work r(c, fb);
    struct Cleanup {
        std::vector<Work *> &a, &b;
        ~Cleanup()
        {
            for (auto *w : a) delete w;
            for (auto *w : b) delete w;
        }
    } cleanup{phi, chi};
    for (int j = 0; j < nkv; ++j)
        if (!phi[j]->ok() || !chi[j]->ok()) return WDR_ENOMEM;
    if (!r.ok()) return WDR_ENOMEM;

    // device pointer table: chi_0..chi_{nkv-1}, phi_0..phi_{nkv-1}
    std::vector<const void *> hp(2 * nkv);
    for (int j = 0; j < nkv; ++j) {
        hp[j] = chi[j]->as<void>();
        hp[nkv + j] = phi[j]->as<void>();
    }
    WDR_HIP(hipMemcpyAsync(c->ptrs, hp.data(), hp.size() * sizeof(void *), hipMemcpyHostToDevice, s));
    const double2 *const *chis = reinterpret_cast<const double2 *const *>(c->ptrs);
    const double2 *const *phis = chis + nkv;

    // scalars: A[l][j] at scal[l*16 + j] (two CGS passes summed), b_j at
    // scal[256 + j], c_j at scal[272 + j], alpha at scal[288 + j], norms at 320+
    double2 *A = c->scal, *bj = c->scal + 256, *cj = c->scal + 272, *al = c->scal + 288, *nr = c->scal + 320;

    launch_norm2<double>(b, n, c->red, nr, s);
    const double bn2 = read_scalar(c, 320, s);
    launch_zero<double>(x, n, s);
    st = Stats();
    if (bn2 == 0.0) return WDR_OK;
    launch_convert<double, double>(b, r.as<double2>(), n, s);
    const double tol2 = tol * tol * bn2;
    double rn2 = bn2;
    int it = 0;
    while (it < sp.max_iter) {
        int m = 0;
        std::vector<double2> hA(16 * 16), hb(16), hc(16);
        for (int j = 0; j < nkv && it < sp.max_iter; ++j) {
            wdr_status e = sap64(c, U, kappa, sp, r.as<double2>(), phi[j]->as<double2>(), s);
            if (e != WDR_OK) return e;
            apply_D64(c, U, kappa, phi[j]->as<double2>(), chi[j]->as<double2>(), s);
            if (j > 0) {
                // classical Gram-Schmidt, twice (CGS2); coefficients summed
                for (int pass = 0; pass < 2; ++pass) {
                    double2 *coef = c->scal + 352 + pass * 16;
                    launch_multidot<double>(chis, j, chi[j]->as<double2>(), n, c->red, coef, s);
                    launch_multi_axpy(coef, -1.0, chis, j, chi[j]->as<double2>(), n, 1, s);
                }
                // A[l][j] = coef pass0 + pass1 (host side below)
            }
            launch_norm2<double>(chi[j]->as<double2>(), n, c->red, bj + j, s);
            launch_scale_invsqrt(bj + j, chi[j]->as<double2>(), n, s);
            launch_dot<double>(chi[j]->as<double2>(), r.as<double2>(), n, c->red, cj + j, s);
            launch_axpy_dev(cj + j, -1.0, chi[j]->as<double2>(), r.as<double2>(), n, s);
            if (j > 0) {
                double2 co[32];
                WDR_HIP(hipMemcpyAsync(co, c->scal + 352, 32 * sizeof(double2), hipMemcpyDeviceToHost, s));
                WDR_HIP(hipStreamSynchronize(s));
                for (int l = 0; l < j; ++l)
                    hA[l * 16 + j] = make_double2(co[l].x + co[16 + l].x, co[l].y + co[16 + l].y);
            }
            launch_norm2<double>(r.as<double2>(), n, c->red, nr, s);
            rn2 = read_scalar(c, 320, s);
            ++it;
            ++m;
            if (!(rn2 > tol2)) break;
        }
        // x += sum_j alpha_j phi_j with back-substitution
        WDR_HIP(hipMemcpyAsync(hb.data(), bj, 16 * sizeof(double2), hipMemcpyDeviceToHost, s));
        WDR_HIP(hipMemcpyAsync(hc.data(), cj, 16 * sizeof(double2), hipMemcpyDeviceToHost, s));
        WDR_HIP(hipStreamSynchronize(s));
        std::vector<double2> ha(16);
        for (int l = m - 1; l >= 0; --l) {
            double re = hc[l].x, im = hc[l].y;
            for (int j = l + 1; j < m; ++j) {
                const double2 a = hA[l * 16 + j], aj = ha[j];
                re -= a.x * aj.x - a.y * aj.y;
                im -= a.x * aj.y + a.y * aj.x;
            }
            const double bb = std::sqrt(hb[l].x);
            ha[l] = make_double2(re / bb, im / bb);
        }
        WDR_HIP(hipMemcpyAsync(al, ha.data(), m * sizeof(double2), hipMemcpyHostToDevice, s));
        launch_multi_axpy(al, 1.0, phis, m, x, n, 1, s);
        // true residual
        apply_D64(c, U, kappa, x, chi[0]->as<double2>(), s);
        launch_sub(b, chi[0]->as<double2>(), r.as<double2>(), n, s);
        launch_norm2<double>(r.as<double2>(), n, c->red, nr, s);
        rn2 = read_scalar(c, 320, s);
        if (!std::isfinite(rn2)) break;
        if (rn2 <= tol2) break;
    }
    st.iters = it;
    st.total = it;
    st.rel = std::sqrt(rn2 / bn2);
    st.converged = st.rel <= tol;
    WDR_HIP(hipGetLastError());
    if (!st.converged) {
        set_error("FGCR stopped at " + std::to_string(it) + " iterations, relative residual " +
                  std::to_string(st.rel));
        return WDR_ENOCONV;
    }
    return WDR_OK;
}

// ------------------------------------------------------------ CGNE

static wdr_status cgne(wdr_ctx *c, GaugeView U, double kappa, const wdr_solver_params &sp, double tol,
                       const double2 *b, double2 *x, Stats &st, hipStream_t s)
{
    const long n = field_n(c);
    const size_t fb = field_bytes(c, WDR_F64);
    Work r(c, fb), p(c, fb), w(c, fb), q(c, fb);
    if (!r.ok() || !p.ok() || !w.ok() || !q.ok()) return WDR_ENOMEM;
    double2 *sc = c->scal;
    const auto &g = c->g;
    launch_zero<double>(x, n, s);
    launch_convert<double, double>(b, r.as<double2>(), n, s);
    launch_convert<double, double>(b, p.as<double2>(), n, s);
    launch_norm2<double>(b, n, c->red, sc + 0, s);
    const double bn2 = read_scalar(c, 0, s);
    st = Stats();
    if (bn2 == 0.0) return WDR_OK;
    const double tol2 = tol * tol * bn2;
    double rn2 = bn2;
    int it = 0;
    while (it < sp.max_iter) {
        // w = D^+ p, q = D w
        launch_dslash<double>(g, HOPS_ALL, -1, 1, U.u64, p.as<double2>(), p.as<double2>(), w.as<double2>(), kappa,
                              0, g.nblk, s);
        apply_D64(c, U, kappa, w.as<double2>(), q.as<double2>(), s);
        launch_norm2<double>(w.as<double2>(), n, c->red, sc + 1, s);
        k_cg_alpha<<<1, 1, 0, s>>>(sc);
        k_cg_update<<<nb256(n), 256, 0, s>>>(sc, x, w.as<double2>(), r.as<double2>(), q.as<double2>(), nullptr,
                                             nullptr, n);
        launch_norm2<double>(r.as<double2>(), n, c->red, sc + 3, s);
        k_cg_beta<<<1, 1, 0, s>>>(sc);
        k_cg_p<<<nb256(n), 256, 0, s>>>(sc, r.as<double2>(), p.as<double2>(), n);
        ++it;
        if (it % 4 == 0 || it >= sp.max_iter) {
            rn2 = read_scalar(c, 0, s);
            if (!std::isfinite(rn2)) break;
            if (rn2 <= tol2) {
                // confirm with the true residual; restart the directions from it
                apply_D64(c, U, kappa, x, q.as<double2>(), s);
                launch_sub(b, q.as<double2>(), r.as<double2>(), n, s);
                launch_norm2<double>(r.as<double2>(), n, c->red, sc + 0, s);
                rn2 = read_scalar(c, 0, s);
                if (rn2 <= tol2) break;
                launch_convert<double, double>(r.as<double2>(), p.as<double2>(), n, s);
            }
        }
    }
    apply_D64(c, U, kappa, x, q.as<double2>(), s);
    launch_sub(b, q.as<double2>(), r.as<double2>(), n, s);
    launch_norm2<double>(r.as<double2>(), n, c->red, sc + 5, s);
    rn2 = read_scalar(c, 5, s);
    st.iters = it;
    st.total = it;
    st.rel = std::sqrt(rn2 / bn2);
    st.converged = st.rel <= tol;
    WDR_HIP(hipGetLastError());
    if (!st.converged) {
        set_error("CGNE stopped at " + std::to_string(it) + " iterations, relative residual " +
                  std::to_string(st.rel));
        return WDR_ENOCONV;
    }
    return WDR_OK;
}

wdr_status solve64(wdr_ctx *c, GaugeView U, double kappa, const wdr_solver_params &sp, double tol,
                   const double2 *b, double2 *x, Stats &st, hipStream_t s)
{
    if (sp.solver == WDR_SOLVER_CGNE) return cgne(c, U, kappa, sp, tol, b, x, st, s);
    return fgcr(c, U, kappa, sp, tol, b, x, st, s);
}

// ------------------------------------------------------------ block solves

wdr_status block_solve64(wdr_ctx *c, GaugeView U, double kappa, int colour, const wdr_solver_params &sp,
                         double tol, const double2 *b, double2 *x, Stats &st, hipStream_t s)
{
    const auto &g = c->g;
    int slot0, ns;
    colour_slots(c, colour, slot0, ns);
    const long n = field_n(c);
    const size_t fb = field_bytes(c, WDR_F64);
    Work r(c, fb), t(c, fb), d32(c, field_bytes(c, WDR_F32)), r32(c, field_bytes(c, WDR_F32)), d64(c, fb);
    Work nrm(c, 2 * sizeof(double) * g.nblk);
    if (!r.ok() || !t.ok() || !d32.ok() || !r32.ok() || !d64.ok() || !nrm.ok()) return WDR_ENOMEM;
    launch_zero<double>(x, n, s);
    launch_convert<double, double>(b, r.as<double2>(), n, s);
    zero_outside(c, r.as<double2>(), slot0, ns, s);
    double *bn = nrm.as<double>(), *rn = bn + g.nblk;
    launch_slot_norm2(g, r.as<double2>(), bn, slot0, ns, s);
    std::vector<double> hb(ns), hr(ns);
    WDR_HIP(hipMemcpyAsync(hb.data(), bn, ns * sizeof(double), hipMemcpyDeviceToHost, s));
    WDR_HIP(hipStreamSynchronize(s));
    const int nmr = 16;
    st = Stats();
    double worst = 0;
    int it = 0;
    for (; it < 40; ++it) {
        if (sp.inner == WDR_F64) {
            launch_block_mr<double>(g, U.u64, r.as<double2>(), d64.as<double2>(), kappa, nmr, slot0, ns, s);
            launch_add_to64<double>(d64.as<double2>() + 12L * g.Vb * slot0, x + 12L * g.Vb * slot0,
                                    12L * g.Vb * ns, s);
        } else {
            launch_convert<float, double>(r.as<double2>(), r32.as<float2>(), n, s);
            launch_block_mr<float>(g, U.u32, r32.as<float2>(), d32.as<float2>(), (float)kappa, nmr, slot0, ns, s);
            launch_add_to64<float>(d32.as<float2>() + 12L * g.Vb * slot0, x + 12L * g.Vb * slot0, 12L * g.Vb * ns,
                                   s);
        }
        // r = b - D_b x on the selected blocks
        launch_dslash<double>(g, HOPS_IN, -1, 0, U.u64, x, x, t.as<double2>(), kappa, slot0, ns, s);
        launch_sub(b + 12L * g.Vb * slot0, t.as<double2>() + 12L * g.Vb * slot0, r.as<double2>() + 12L * g.Vb * slot0,
                   12L * g.Vb * ns, s);
        launch_slot_norm2(g, r.as<double2>(), rn, slot0, ns, s);
        WDR_HIP(hipMemcpyAsync(hr.data(), rn, ns * sizeof(double), hipMemcpyDeviceToHost, s));
        WDR_HIP(hipStreamSynchronize(s));
        worst = 0;
        for (int i = 0; i < ns; ++i)
            if (hb[i] > 0) worst = std::max(worst, hr[i] / hb[i]);
        if (!std::isfinite(worst)) break;
        if (worst <= tol * tol) {
            ++it;
            break;
        }
    }
    zero_outside(c, x, slot0, ns, s);
    st.iters = it;
    st.total = it;
    st.rel = std::sqrt(worst);
    st.converged = st.rel <= tol;
    WDR_HIP(hipGetLastError());
    if (!st.converged) {
        set_error("block solve stopped at relative residual " + std::to_string(st.rel));
        return WDR_ENOCONV;
    }
    return WDR_OK;
}

// ------------------------------------------------------------ Schur complement

wdr_status schur64(wdr_ctx *c, GaugeView U, double kappa, const wdr_solver_params &sp, const double2 *in,
                   double2 *out, Stats &st, hipStream_t s)
{
    const auto &g = c->g;
    const long n = field_n(c);
    const size_t fb = field_bytes(c, WDR_F64);
    Work t1(c, fb), t2(c, fb);
    if (!t1.ok() || !t2.ok()) return WDR_ENOMEM;
    int b0, bn, w0, wn;
    colour_slots(c, 0, b0, bn);
    colour_slots(c, 1, w0, wn);
    Stats s1;
    // D_wb in (white sites; cross hops from black)
    launch_zero<double>(t1.as<double2>(), n, s);
    launch_dslash<double>(g, HOPS_CROSS, -1, 0, U.u64, in, nullptr, t1.as<double2>(), kappa, w0, wn, s);
    wdr_status e = block_solve64(c, U, kappa, 1, sp, sp.block_tol, t1.as<double2>(), t2.as<double2>(), s1, s);
    st.merge(s1);
    if (e != WDR_OK) return e;
    // D_bw (...) on black sites
    launch_zero<double>(t1.as<double2>(), n, s);
    launch_dslash<double>(g, HOPS_CROSS, -1, 0, U.u64, t2.as<double2>(), nullptr, t1.as<double2>(), kappa, b0, bn, s);
    e = block_solve64(c, U, kappa, 0, sp, sp.block_tol, t1.as<double2>(), t2.as<double2>(), s1, s);
    st.merge(s1);
    if (e != WDR_OK) return e;
    // out = in - t2 on black, zero on white
    launch_sub(in, t2.as<double2>(), out, n, s);
    zero_outside(c, out, b0, bn, s);
    return WDR_OK;
}

}  // namespace wdr
