// Schedule autotuner: the depth of the Schwarz preconditioner (cycles x MR
// steps per block) and of the block-solve rounds decide how the work of a
// solve is cut into block launches, and the launch forms (stencil kernel of
// D and D_b, block-MR form) how blocks map onto the CUs; every choice solves
// to the same tolerances, so the fastest one is picked by timing a short
// estimate on the caller's data and cached in the context.
#include <chrono>
#include <cmath>
#include <algorithm>
#include <cstdio>

#include "runtime.h"

namespace wdr {
namespace {

double wall()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// seconds of a short estimate with parameters q, the faster of two runs
// after one untimed run, or infinity if it fails or does not converge
double trial(wdr_ctx *c, const wdr_gauge *U, const wdr_gauge *Up, double kappa, const wdr_est_params &q,
             hipStream_t s)
{
    const std::vector<Proposal> props{Proposal{U, Up, kappa, q.seed}};
    Stats st;
    if (logdet_ratio(c, props, q, nullptr, nullptr, st, s) != WDR_OK) return INFINITY;
    if (hipStreamSynchronize(s) != hipSuccess) return INFINITY;
    double best = INFINITY;
    for (int k = 0; k < 2; ++k) {
        const double t0 = wall();
        if (logdet_ratio(c, props, q, nullptr, nullptr, st, s) != WDR_OK) return INFINITY;
        if (hipStreamSynchronize(s) != hipSuccess) return INFINITY;
        best = std::min(best, wall() - t0);
    }
    return best;
}

}  // namespace
}  // namespace wdr

using namespace wdr;

extern "C" {

wdr_status wdr_autotune(wdr_ctx *c, const wdr_gauge *U, const wdr_gauge *Up, double kappa, wdr_est_params *p,
                        double *host_seconds, void *stream)
{
    if (check_ctx(c) != WDR_OK) return WDR_EINVAL;
    if (!U || !Up || U->ctx != c || Up->ctx != c) {
        set_error("gauge handles of another context (or NULL)");
        return WDR_ESTATE;
    }
    if (U->c64 || Up->c64) {
        set_error("the autotuner does not support gauge fields with a clover term");
        return WDR_EINVAL;
    }
    if (!(kappa > 0) || !p || p->n_steps < 1 || p->n_noise < 1) {
        set_error("invalid kappa or estimator parameters");
        return WDR_EINVAL;
    }
    if (p->op != WDR_OP_FULL && p->op != WDR_OP_SCHUR && p->op != WDR_OP_BLOCKS && p->op != WDR_OP_DD) {
        set_error("invalid estimator parameters");
        return WDR_EINVAL;
    }
    wdr_status e = check_params(c, p->sp, p->op != WDR_OP_FULL);
    if (e != WDR_OK) return e;
    WDR_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    char key[112];
    std::snprintf(key, sizeof(key), "op%d solver%d inner%d middle%d kappa%.9g", (int)p->op, (int)p->sp.solver,
                  (int)p->sp.inner, (int)p->sp.middle, kappa);
    double best_t = INFINITY;
    auto set_forms = [&](int stencil, int mr) {
        c->g.stencil = stencil;
        c->g.mr_form = mr;
        if (c->twin) {
            c->twin->g.stencil = stencil;
            c->twin->g.mr_form = mr;
        }
    };
    auto hit = c->tuned.find(key);
    if (hit != c->tuned.end()) {
        p->sp.sap_cycles = hit->second.sap_cycles;
        p->sp.mr_steps = hit->second.mr_steps;
        p->sp.block_mr_steps = hit->second.block_mr_steps;
        const auto &f = c->tuned_forms[key];
        set_forms(f.first, f.second);
    } else {
        wdr_est_params q = *p;
        // up to 8 path factors: the systems per launch set the balance
        // between block launches and the rest of a solve
        q.n_steps = std::min(p->n_steps, 8);
        q.seed = p->seed + 1;
        wdr_solver_params best = p->sp;
        if (p->sp.solver == WDR_SOLVER_FGCR_SAP) {
            static const int sap[][2] = {{2, 3}, {2, 4}, {3, 3}, {3, 4}, {4, 3}, {4, 4}, {4, 5}, {5, 4},
                                         {6, 3}, {6, 4}, {6, 5}, {8, 3}, {8, 4}};
            for (const auto &cand : sap) {
                q.sp = best;
                q.sp.sap_cycles = cand[0];
                q.sp.mr_steps = cand[1];
                const double t = trial(c, U, Up, kappa, q, s);
                if (t < best_t) {
                    best_t = t;
                    best.sap_cycles = cand[0];
                    best.mr_steps = cand[1];
                }
            }
        }
        if (p->op != WDR_OP_FULL) {
            static const int bmr[] = {6, 8, 12, 16, 24, 32, 48, 64};
            const wdr_solver_params base = best;
            for (int b : bmr) {
                q.sp = base;
                q.sp.block_mr_steps = b;
                const double t = trial(c, U, Up, kappa, q, s);
                if (t < best_t) {
                    best_t = t;
                    best = q.sp;
                }
            }
        }
        // launch forms, one at a time from the context's current choice
        int st0 = c->g.stencil, mr0 = c->g.mr_form;
        q.sp = best;
        if (!std::isfinite(best_t)) best_t = trial(c, U, Up, kappa, q, s);
        if (p->op != WDR_OP_FULL)
            for (int mr : {WDR_MR_AUTO, WDR_MR_ONE_PER_CU, WDR_MR_TWO_PER_CU}) {
                if (mr == mr0) continue;
                set_forms(st0, mr);
                const double t = trial(c, U, Up, kappa, q, s);
                if (t < best_t) {
                    best_t = t;
                    mr0 = mr;
                }
            }
        for (int sc : {WDR_STENCIL_AUTO, WDR_STENCIL_DIR, WDR_STENCIL_BLK}) {
            if (sc == st0) continue;
            set_forms(sc, mr0);
            const double t = trial(c, U, Up, kappa, q, s);
            if (t < best_t) {
                best_t = t;
                st0 = sc;
            }
        }
        set_forms(st0, mr0);
        if (!std::isfinite(best_t)) {
            set_error("no candidate schedule converged");
            return WDR_ENOCONV;
        }
        p->sp.sap_cycles = best.sap_cycles;
        p->sp.mr_steps = best.mr_steps;
        p->sp.block_mr_steps = best.block_mr_steps;
        c->tuned[key] = p->sp;
        c->tuned_forms[key] = {st0, mr0};
    }
    if (host_seconds) *host_seconds = best_t;
    WDR_HIP(hipGetLastError());
    return WDR_OK;
}

}  // extern "C"
