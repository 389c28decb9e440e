// Stochastic estimate of the log determinant ratio (paper Sec. 4).
//
// For every factor i of eq. param (U_i -> U_{i+1} on the geodesic path) and
// noise sample k, with X the operator of the chosen ratio (D, the Dirichlet
// blocks, or the Schur complement Dhat) built on U_i and X' on U_{i+1}:
//     s = -eta^+ (M^+ M - 1) eta,   M = X'^-1 X,
// so that E[exp(s)] = det(X'^+ X') / det(X^+ X) for complex Gaussian eta.
// ||M eta||^2 = ||P z||^2 with z = A'^-1 y (A' = D' or the blocks, y = X eta
// or A' Dhat eta, P the black-site projector for the Schur complement,
// because Dhat'^-1 = (D'^-1)_bb A'_bb).  It is evaluated to second order in
// the solver residual r = y - A' z:
//     ||P z||^2 = ||P z~||^2 + 2 Re w^+ r + O(|r|^2),   A'^+ w = P z~,
// with the adjoint solve done as A' (g5 w) = g5 P z~ (gamma5-hermiticity).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "runtime.h"

namespace wdr {
namespace {

struct TmpGauge {
    Work u64, u32;
    TmpGauge(wdr_ctx *c) : u64(c, (size_t)c->g.V * 36 * sizeof(double2)), u32(c, (size_t)c->g.V * 36 * sizeof(float2)) {}
    bool ok() const { return u64.ok() && u32.ok(); }
    GaugeView view() const { return {u64.as<double2>(), u32.as<float2>()}; }
};

// builds U_i of the path into dst
void make_path_gauge(wdr_ctx *c, const wdr_gauge *U, const wdr_gauge *Up, int i, int N, TmpGauge &dst, hipStream_t s)
{
    const size_t n = (size_t)c->g.V * 36;
    if (i == 0) {
        hipMemcpyAsync(dst.u64.as<double2>(), U->u64, n * sizeof(double2), hipMemcpyDeviceToDevice, s);
    } else if (i == N) {
        hipMemcpyAsync(dst.u64.as<double2>(), Up->u64, n * sizeof(double2), hipMemcpyDeviceToDevice, s);
    } else {
        launch_interpolate(c->g, U->u64, Up->u64, (double)i / N, dst.u64.as<double2>(), s);
    }
    launch_convert_gauge_f32(c->g, dst.u64.as<double2>(), dst.u32.as<float2>(), s);
}

}  // namespace

wdr_status logdet_ratio(wdr_ctx *c, const wdr_gauge *U, const wdr_gauge *Up, double kappa, const wdr_est_params &p,
                        double *host_samples, double *host_log_ratio, Stats &st, hipStream_t s)
{
    const auto &g = c->g;
    const long n = field_n(c);
    const size_t fb = field_bytes(c, WDR_F64);
    const wdr_solver_params &sp = p.sp;
    TmpGauge ga(c), gb(c);
    Work eta(c, fb), y(c, fb), z(c, fb), w(c, fb), r(c, fb), t(c, fb), per(c, sizeof(double) * g.nblk);
    if (!ga.ok() || !gb.ok() || !eta.ok() || !y.ok() || !z.ok() || !w.ok() || !r.ok() || !t.ok() || !per.ok())
        return WDR_ENOMEM;
    const int nout = p.op == WDR_OP_BLOCKS ? g.nblk : 1;
    std::vector<double> samples((size_t)p.n_steps * p.n_noise * nout, 0.0);
    std::vector<double> slot_vals(g.nblk);
    int b0, bn;
    colour_slots(c, 0, b0, bn);
    st = Stats();
    wdr_status status = WDR_OK;

    TmpGauge *cur = &ga, *nxt = &gb;
    make_path_gauge(c, U, Up, 0, p.n_steps, *cur, s);
    for (int i = 0; i < p.n_steps; ++i) {
        make_path_gauge(c, U, Up, i + 1, p.n_steps, *nxt, s);
        const GaugeView X = cur->view(), Xp = nxt->view();
        for (int k = 0; k < p.n_noise; ++k) {
            Stats s1;
            wdr_status e = WDR_OK;
            double2 *E = eta.as<double2>(), *Y = y.as<double2>(), *Z = z.as<double2>(), *W = w.as<double2>(),
                    *R = r.as<double2>(), *Tm = t.as<double2>();
            launch_noise(g, p.noise, p.seed, i, k, p.op == WDR_OP_SCHUR, E, s);
            if (p.op == WDR_OP_FULL) {
                apply_D64(c, X, kappa, E, Y, s);                                  // y = D eta
                e = solve64(c, Xp, kappa, sp, sp.tol, Y, Z, s1, s);               // D' z = y
                st.merge(s1);
                if (e != WDR_OK && e != WDR_ENOCONV) return e;
                if (e == WDR_ENOCONV) status = e;
                launch_g5<double>(g, Z, Tm, 0, g.nblk, s);                         // D' v = g5 z
                e = solve64(c, Xp, kappa, sp, sp.adj_tol, Tm, W, s1, s);
                st.total += s1.total;
                if (e != WDR_OK && e != WDR_ENOCONV) return e;
                if (e == WDR_ENOCONV) status = e;
                launch_g5<double>(g, W, W, 0, g.nblk, s);                          // w = g5 v
                apply_D64(c, Xp, kappa, Z, Tm, s);
                launch_sub(Y, Tm, R, n, s);                                        // r = y - D' z
            } else if (p.op == WDR_OP_BLOCKS) {
                launch_dslash<double>(g, HOPS_IN, -1, 0, X.u64, E, E, Y, kappa, 0, g.nblk, s);  // y = D_blk eta
                e = block_solve64(c, Xp, kappa, 2, sp, sp.block_tol, Y, Z, s1, s);
                st.merge(s1);
                if (e != WDR_OK && e != WDR_ENOCONV) return e;
                if (e == WDR_ENOCONV) status = e;
                launch_g5<double>(g, Z, Tm, 0, g.nblk, s);
                e = block_solve64(c, Xp, kappa, 2, sp, sp.block_tol, Tm, W, s1, s);
                st.total += s1.total;
                if (e != WDR_OK && e != WDR_ENOCONV) return e;
                if (e == WDR_ENOCONV) status = e;
                launch_g5<double>(g, W, W, 0, g.nblk, s);
                launch_dslash<double>(g, HOPS_IN, -1, 0, Xp.u64, Z, Z, Tm, kappa, 0, g.nblk, s);
                launch_sub(Y, Tm, R, n, s);
            } else {  // SCHUR
                e = schur64(c, X, kappa, sp, E, Tm, s1, s);                       // Dhat eta (black)
                st.total += s1.total;
                if (e != WDR_OK) return e;
                launch_zero<double>(Y, n, s);                                      // y = A' Dhat eta
                launch_dslash<double>(g, HOPS_IN, -1, 0, Xp.u64, Tm, Tm, Y, kappa, b0, bn, s);
                e = solve64(c, Xp, kappa, sp, sp.tol, Y, Z, s1, s);               // D' z = [y; 0]
                st.merge(s1);
                if (e != WDR_OK && e != WDR_ENOCONV) return e;
                if (e == WDR_ENOCONV) status = e;
                apply_D64(c, Xp, kappa, Z, Tm, s);
                launch_sub(Y, Tm, R, n, s);                                        // r = y - D' z
                launch_zero<double>(Z + 12L * g.Vb * bn, 12L * g.Vb * (g.nblk - bn), s);  // z <- P z
                launch_g5<double>(g, Z, Tm, 0, g.nblk, s);                         // D' v = g5 P z
                e = solve64(c, Xp, kappa, sp, sp.adj_tol, Tm, W, s1, s);
                st.total += s1.total;
                if (e != WDR_OK && e != WDR_ENOCONV) return e;
                if (e == WDR_ENOCONV) status = e;
                launch_g5<double>(g, W, W, 0, g.nblk, s);
            }
            launch_sample_terms(g, E, Z, W, R, per.as<double>(), 0, g.nblk, s);
            WDR_HIP(hipMemcpyAsync(slot_vals.data(), per.as<double>(), g.nblk * sizeof(double), hipMemcpyDeviceToHost, s));
            WDR_HIP(hipStreamSynchronize(s));
            double *dst = samples.data() + ((size_t)i * p.n_noise + k) * nout;
            if (p.op == WDR_OP_BLOCKS) {
                for (int b = 0; b < g.nblk; ++b) dst[b] = slot_vals[c->slot_of_block[b]];
            } else {
                double sum = 0;  // fixed order over slots
                for (int sl = 0; sl < g.nblk; ++sl) sum += slot_vals[sl];
                dst[0] = sum;
            }
        }
        std::swap(cur, nxt);
    }
    if (host_samples) std::copy(samples.begin(), samples.end(), host_samples);
    if (host_log_ratio) {
        // sum_i log( (1/K) sum_k exp(s_ik) ), summed over blocks for BLOCKS
        double total = 0;
        for (int b = 0; b < nout; ++b)
            for (int i = 0; i < p.n_steps; ++i) {
                double m = -INFINITY;
                for (int k = 0; k < p.n_noise; ++k) m = std::max(m, samples[((size_t)i * p.n_noise + k) * nout + b]);
                double acc = 0;
                for (int k = 0; k < p.n_noise; ++k) acc += std::exp(samples[((size_t)i * p.n_noise + k) * nout + b] - m);
                total += m + std::log(acc / p.n_noise);
            }
        *host_log_ratio = total;
    }
    return status;
}

}  // namespace wdr
