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
//
// All (i, k) samples are independent given the path, so they are solved
// together as one batch of systems (in chunks that fit a memory budget):
// every kernel launch covers every sample of the chunk.
#include <algorithm>
#include <cmath>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "runtime.h"

namespace wdr {
namespace {

struct TmpGauge {
    Work u64, u32, u16, e16, c64, c32;
    // su3: FP16 links for the block MR / Schwarz kernels; cg16: E16 links
    // for the FP16 even-odd CG as well; clov: the clover term (A, A^-1) in
    // FP64 and FP32
    TmpGauge(wdr_ctx *c, bool su3, bool cg16, bool clov)
        : u64(c, (size_t)c->g.V * 36 * sizeof(double2)), u32(c, (size_t)c->g.V * 36 * sizeof(float2)),
          u16(c, su3 ? (size_t)c->g.V * 24 * sizeof(h2) : 256),
          e16(c, su3 && cg16 ? (size_t)c->g.V * 24 * sizeof(h2) : 256),
          c64(c, clov ? (size_t)c->g.V * 144 * sizeof(double) : 256),
          c32(c, clov ? (size_t)c->g.V * 144 * sizeof(float) : 256), has16(su3), hase16(su3 && cg16), clov(clov)
    {
    }
    bool ok() const { return u64.ok() && u32.ok() && u16.ok() && e16.ok() && c64.ok() && c32.ok(); }
    bool has16, hase16, clov;
};

// U_0 .. U_N of one proposal into pts[0 .. N]: the end points are copies, the
// interior points come from one interpolation launch; then the FP32 and FP16
// copies of every point, and its clover term (coefficient csw, hopping
// parameter kappa; worst[i] receives the worst pivot measure of point i)
void make_path_gauges(wdr_ctx *c, const wdr_gauge *U, const wdr_gauge *Up, int N, TmpGauge *const *pts, double csw,
                      double kappa, void *cwork, double *worst, hipStream_t s)
{
    const size_t n = (size_t)c->g.V * 36;
    // compulsory bytes: both fields read and every interior point written,
    // the two end points copied, and the FP32 / FP16 copies of every point
    const double lb = 36.0 * sizeof(double2), V = c->g.V;
    add_traffic(V * ((2 + (N - 1)) * lb + 4 * lb +
                     (N + 1) * (lb + lb / 2 + (pts[0]->has16 ? lb + 96 : 0) + (pts[0]->hase16 ? lb + 96 : 0))));
    (void)hipMemcpyAsync(pts[0]->u64.as<double2>(), U->u64, n * sizeof(double2), hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(pts[N]->u64.as<double2>(), Up->u64, n * sizeof(double2), hipMemcpyDeviceToDevice, s);
    std::vector<double> t;
    std::vector<double2 *> out;
    for (int i = 1; i < N; ++i) {
        t.push_back((double)i / N);
        out.push_back(pts[i]->u64.as<double2>());
    }
    if (!t.empty()) launch_interpolate_many(c->g, U->u64, Up->u64, t.data(), out.data(), (int)t.size(), s);
    for (int i = 0; i <= N; ++i) {
        TmpGauge &dst = *pts[i];
        launch_convert_gauge_f32(c->g, dst.u64.as<double2>(), dst.u32.as<float2>(), s);
        if (dst.has16) launch_pack_links_h16(c->g, dst.u64.as<double2>(), dst.u16.as<h2>(), s);
        if (dst.hase16) launch_pack_links_e16(c->g, dst.u64.as<double2>(), dst.e16.as<h2>(), s);
        if (dst.clov)
            launch_clover_build(c->g, dst.u64.as<double2>(), csw, kappa, cwork, dst.c64.as<double>(),
                                dst.c32.as<float>(), worst + i, s);
    }
    // clover build per point: the links, the field strengths written and read
    // back, A and A^-1 in FP64, their FP32 copy
    if (pts[0]->clov) add_traffic(V * (N + 1) * (lb + 2 * 54 * 16.0 + 2 * 144 * 8.0 + 144 * 4.0));
}

// device memory budget for the fields of one chunk of samples (the 32
// factors of a 32^4 estimate fit in one chunk)
constexpr double CHUNK_BYTES = 96e9;

}  // namespace

// the path U_0 .. U_N of every proposal (workspace of c)
struct Path {
    std::vector<std::unique_ptr<TmpGauge>> pts;
    int N = 0, su3 = 1;
    bool has16 = false, hase16 = false, clov = false;
    TmpGauge &at(int prop, int i) const { return *pts[(size_t)prop * (N + 1) + i]; }
};

static wdr_status build_path(wdr_ctx *c, const std::vector<Proposal> &props, const wdr_est_params &p, Path &path,
                             hipStream_t s)
{
    path.N = p.n_steps;
    path.su3 = 1;
    for (const Proposal &q : props) path.su3 = path.su3 && q.U->su3 && q.Up->su3;  // the geodesic stays in SU(3)
    path.has16 = path.su3 && p.sp.inner == WDR_F16;
    path.hase16 = path.has16 && p.sp.solver == WDR_SOLVER_CGNE && e16_geometry(c->g);
    path.clov = props[0].U->c64 != nullptr;
    std::unique_ptr<Work> cwork, worst;
    if (path.clov) {
        cwork.reset(new Work(c, clover_work_bytes(c->g)));
        worst.reset(new Work(c, sizeof(double) * props.size() * (path.N + 1)));
        if (!cwork->ok() || !worst->ok()) return WDR_ENOMEM;
    }
    for (size_t k = 0; k < props.size(); ++k) {
        const Proposal &q = props[k];
        std::vector<TmpGauge *> pts;
        for (int i = 0; i <= path.N; ++i) {
            path.pts.emplace_back(new TmpGauge(c, path.has16, path.hase16, path.clov));
            if (!path.pts.back()->ok()) return WDR_ENOMEM;
            pts.push_back(path.pts.back().get());
        }
        make_path_gauges(c, q.U, q.Up, path.N, pts.data(), q.U->csw, q.kappa, path.clov ? cwork->as<void>() : nullptr,
                         path.clov ? worst->as<double>() + k * (path.N + 1) : nullptr, s);
    }
    if (path.clov) {
        std::vector<double> h(props.size() * (path.N + 1));
        WDR_HIP(hipMemcpyAsync(h.data(), worst->as<double>(), sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
        WDR_HIP(hipStreamSynchronize(s));
        for (double v : h)
            if (!(v < 1e8)) {
                set_error("the clover term of a point on the path has a (nearly) singular block");
                return WDR_EINVAL;
            }
    }
    return WDR_OK;
}

// the samples of one ratio (op FULL, SCHUR or BLOCKS) for every (proposal,
// step, noise), in batched chunks; samples[m * nout + b], nout = nblk for
// BLOCKS, else 1.  Work space comes from c; the path may belong to another
// context of the same geometry.
static wdr_status run_op(wdr_ctx *c, const Path &path, const std::vector<Proposal> &props, int op,
                         const wdr_est_params &p, std::vector<double> &samples, Stats &st, hipStream_t s)
{
    const auto &g = c->g;
    const long n = field_n(c);
    const wdr_solver_params &sp = p.sp;
    const int P = (int)props.size(), N = p.n_steps, K = p.n_noise, per_prop = N * K, total = P * per_prop;
    const int nout = op == WDR_OP_BLOCKS ? g.nblk : 1;
    const int su3 = path.su3;
    const bool want16 = path.has16;
    const bool wante16 = path.hase16;
    auto point = [&](int prop, int i) -> TmpGauge & { return path.at(prop, i); };

    // chunk size: sample fields plus solver work space per system
    const size_t fb = field_bytes(c, WDR_F64);
    const int per_system = 8 + (sp.solver == WDR_SOLVER_FGCR_SAP ? 2 * sp.restart + 4 : 6);
    int Mmax = std::max(1, std::min(total, (int)(CHUNK_BYTES / ((double)per_system * fb))));
    if (p.max_batch > 0) Mmax = std::min(Mmax, p.max_batch);

    samples.assign((size_t)total * nout, 0.0);
    std::vector<double> per((size_t)g.nblk * Mmax);
    int b0, bn;
    colour_slots(c, 0, b0, bn);
    std::vector<Stats> all_stats;
    wdr_status status = WDR_OK;
    const double kappa0 = props[0].kappa;  // used only where a launch has no kappa table

    for (int m0 = 0; m0 < total; m0 += Mmax) {
        const int M = std::min(Mmax, total - m0);
        const size_t fbm = fb * M;
        Work eta(c, fbm), y(c, fbm), z(c, fbm), w(c, fbm), r(c, fbm), t(c, fbm), pr(c, sizeof(double) * g.nblk * M);
        Work tabs(c, 12 * M * sizeof(void *)), idx(c, 2 * M * sizeof(int32_t)), kw(c, M * sizeof(double)),
            sw(c, M * sizeof(uint64_t));
        if (!eta.ok() || !y.ok() || !z.ok() || !w.ok() || !r.ok() || !t.ok() || !pr.ok() || !tabs.ok() || !idx.ok() ||
            !kw.ok() || !sw.ok())
            return WDR_ENOMEM;
        // per-system tables: X on U_i, X' on U_{i+1}; noise (step, sample, key); kappa
        std::vector<const void *> ht(12 * M, nullptr);
        std::vector<int32_t> hi(2 * M);
        std::vector<double> hk(M);
        std::vector<uint64_t> hs(M);
        for (int j = 0; j < M; ++j) {
            const int m = m0 + j, q = m / per_prop, i = (m % per_prop) / K, k = m % K;
            ht[j] = point(q, i).u64.as<void>();
            ht[M + j] = point(q, i).u32.as<void>();
            ht[2 * M + j] = point(q, i + 1).u64.as<void>();
            ht[3 * M + j] = point(q, i + 1).u32.as<void>();
            if (want16) {
                ht[4 * M + j] = point(q, i).u16.as<void>();
                ht[5 * M + j] = point(q, i + 1).u16.as<void>();
            }
            if (wante16) {
                ht[6 * M + j] = point(q, i).e16.as<void>();
                ht[7 * M + j] = point(q, i + 1).e16.as<void>();
            }
            if (path.clov) {
                ht[8 * M + j] = point(q, i).c64.as<void>();
                ht[9 * M + j] = point(q, i).c32.as<void>();
                ht[10 * M + j] = point(q, i + 1).c64.as<void>();
                ht[11 * M + j] = point(q, i + 1).c32.as<void>();
            }
            hi[j] = i;
            hi[M + j] = k;
            hk[j] = props[q].kappa;
            hs[j] = props[q].seed;
        }
        WDR_HIP(hipMemcpyAsync(tabs.as<void>(), ht.data(), ht.size() * sizeof(void *), hipMemcpyHostToDevice, s));
        WDR_HIP(hipMemcpyAsync(idx.as<void>(), hi.data(), hi.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        WDR_HIP(hipMemcpyAsync(kw.as<void>(), hk.data(), hk.size() * sizeof(double), hipMemcpyHostToDevice, s));
        WDR_HIP(hipMemcpyAsync(sw.as<void>(), hs.data(), hs.size() * sizeof(uint64_t), hipMemcpyHostToDevice, s));
        const void *const *tb = tabs.as<const void *const>();
        const double *kap = kw.as<const double>();
        GaugeTab X{{reinterpret_cast<UTab<double>>(tb), su3, kap},
                   {reinterpret_cast<UTab<float>>(tb + M), su3, kap},
                   {want16 ? reinterpret_cast<const h2 *const *>(tb + 4 * M) : nullptr, kap},
                   {wante16 ? reinterpret_cast<const h2 *const *>(tb + 6 * M) : nullptr, kap}};
        GaugeTab Xp{{reinterpret_cast<UTab<double>>(tb + 2 * M), su3, kap},
                    {reinterpret_cast<UTab<float>>(tb + 3 * M), su3, kap},
                    {want16 ? reinterpret_cast<const h2 *const *>(tb + 5 * M) : nullptr, kap},
                    {wante16 ? reinterpret_cast<const h2 *const *>(tb + 7 * M) : nullptr, kap}};
        if (path.clov) {
            X.u64.ctab = reinterpret_cast<const double *const *>(tb + 8 * M);
            X.u32.ctab = reinterpret_cast<const float *const *>(tb + 9 * M);
            Xp.u64.ctab = reinterpret_cast<const double *const *>(tb + 10 * M);
            Xp.u32.ctab = reinterpret_cast<const float *const *>(tb + 11 * M);
        }
        // the block operators D_b: with a clover term their diagonal is A
        Links<double> Xb = X.u64, Xpb = Xp.u64;
        Xb.cmode = Xpb.cmode = CLOV_DIAG;
        const Sys all = all_sys(c, M);
        double2 *E = eta.as<double2>(), *Y = y.as<double2>(), *Z = z.as<double2>(), *W = w.as<double2>(),
                *R = r.as<double2>(), *Tm = t.as<double2>();
        std::vector<Stats> s1;
        // records the solve statistics (main solves only) and a non-convergence;
        // returns false on a hard error, left in `hard`
        wdr_status hard = WDR_OK;
        auto take = [&](wdr_status e, bool main) -> bool {
            if (main) all_stats.insert(all_stats.end(), s1.begin(), s1.end());
            if (e == WDR_ENOCONV) status = e;
            if (e != WDR_OK && e != WDR_ENOCONV) hard = e;
            return e == WDR_OK || e == WDR_ENOCONV;
        };
        const double kappa = kappa0;

        launch_noise(g, all, p.noise, p.seed, sw.as<uint64_t>(), idx.as<int32_t>(), idx.as<int32_t>() + M,
                     op == WDR_OP_SCHUR, E, s);
        if (op == WDR_OP_FULL) {
            apply_D64(c, all, X, kappa, E, Y, s);                                          // y = D eta
            if (!take(solve64(c, M, Xp, kappa, sp, sp.tol, Y, Z, s1, s), true)) return hard;   // D' z = y
            launch_g5<double>(g, all, Z, Tm, s);                                           // D' v = g5 z
            if (!take(solve64(c, M, Xp, kappa, sp, sp.adj_tol, Tm, W, s1, s), false)) return hard;
            launch_g5<double>(g, all, W, W, s);                                            // w = g5 v
            apply_D64(c, all, Xp, kappa, Z, Tm, s);
            launch_sub(all, Y, Tm, R, s);                                                  // r = y - D' z
        } else if (op == WDR_OP_BLOCKS) {
            launch_dslash<double>(g, all, Xb, HOPS_IN, -1, 0, E, E, Y, kappa, 0, g.nblk, s);  // y = D_blk eta
            if (!take(block_solve64(c, M, Xp, kappa, 2, sp, sp.block_tol, Y, Z, s1, s), true)) return hard;
            launch_g5<double>(g, all, Z, Tm, s);
            if (!take(block_solve64(c, M, Xp, kappa, 2, sp, sp.block_tol, Tm, W, s1, s), false)) return hard;
            launch_g5<double>(g, all, W, W, s);
            launch_dslash<double>(g, all, Xpb, HOPS_IN, -1, 0, Z, Z, Tm, kappa, 0, g.nblk, s);
            launch_sub(all, Y, Tm, R, s);
        } else {  // SCHUR
            wdr_status e = schur64(c, M, X, kappa, sp, E, Tm, s1, s);                     // Dhat eta (black)
            if (e != WDR_OK) {
                if (e == WDR_ENOCONV) status = e;
                else return e;
            }
            launch_zero<double>(Y, n * M, s);                                              // y = A' Dhat eta
            launch_dslash<double>(g, all, Xpb, HOPS_IN, -1, 0, Tm, Tm, Y, kappa, b0, bn, s);
            if (!take(solve64(c, M, Xp, kappa, sp, sp.tol, Y, Z, s1, s), true)) return hard;  // D' z = [y; 0]
            apply_D64(c, all, Xp, kappa, Z, Tm, s);
            launch_sub(all, Y, Tm, R, s);                                                  // r = y - D' z
            launch_keep_slots(g, all, Z, b0, bn, s);                                       // z <- P z
            launch_g5<double>(g, all, Z, Tm, s);                                           // D' v = g5 P z
            if (!take(solve64(c, M, Xp, kappa, sp, sp.adj_tol, Tm, W, s1, s), false)) return hard;
            launch_g5<double>(g, all, W, W, s);
        }
        launch_sample_terms(g, all, E, Z, W, R, pr.as<double>(), s);
        {
            // compulsory bytes of this chunk's kernels outside the solvers
            // (which count their own): the noise, the operator applications,
            // differences, gamma_5 and clears, the sample sums
            double lin = 0;
            for (int mu = 0; mu < 4; ++mu) lin += (double)(g.B[mu] - 1) / g.B[mu];
            const double V = g.V, sb = spin_b<double>(), lk = su3 ? 384.0 : 576.0;
            const double D = V * (2 * sb + lk + (path.clov ? clov_b<double>() : 0.0)),
                         Din = V * (2 * sb + lin * (su3 ? 96.0 : 144.0) + (path.clov ? clov_b<double>() : 0.0));
            double b = V * sb + V * 3 * sb + V * 4 * sb;  // noise, r = y - X' z, sample sums
            if (op == WDR_OP_FULL) b += 2 * D + 2 * V * 2 * sb;
            else if (op == WDR_OP_BLOCKS) b += 2 * Din + 2 * V * 2 * sb;
            else b += V * sb + Din / 2 + D + V * sb + 2 * V * 2 * sb;
            add_traffic(M * b);
        }
        WDR_HIP(hipMemcpyAsync(per.data(), pr.as<double>(), (size_t)g.nblk * M * sizeof(double), hipMemcpyDeviceToHost,
                               s));
        WDR_HIP(hipStreamSynchronize(s));
        for (int j = 0; j < M; ++j) {
            const double *ps = per.data() + (size_t)j * g.nblk;
            double *dst = samples.data() + (size_t)(m0 + j) * nout;
            if (op == WDR_OP_BLOCKS) {
                for (int b = 0; b < g.nblk; ++b) dst[b] = ps[c->slot_of_block[b]];
            } else {
                double sum = 0;  // fixed order over slots
                for (int sl = 0; sl < g.nblk; ++sl) sum += ps[sl];
                dst[0] = sum;
            }
        }
    }
    st = summarize(all_stats);
    return status;
}

// a second context of the same geometry with its own workspace pool, solver
// read-back buffers and stream (for running two estimates concurrently)
static wdr_ctx *twin_of(wdr_ctx *c)
{
    if (!c->twin) {
        wdr_ctx *t = new wdr_ctx();
        t->device = c->device;
        t->geom = c->geom;
        t->g = c->g;  // shares the parent's geometry tables (tables = NULL: not owned)
        t->slot_of_block = c->slot_of_block;
        c->twin = t;
    }
    return c->twin;
}

wdr_status logdet_ratio(wdr_ctx *c, const std::vector<Proposal> &props, const wdr_est_params &p,
                        double *host_samples, double *host_log_ratios, Stats &st, hipStream_t s)
{
    const auto &g = c->g;
    const int P = (int)props.size(), N = p.n_steps, K = p.n_noise, per_prop = N * K, total = P * per_prop;
    Path path;
    wdr_status e = build_path(c, props, p, path, s);
    if (e != WDR_OK) return e;
    std::vector<double> samples;
    int nout;
    wdr_status status = WDR_OK;
    if (p.op != WDR_OP_DD) {
        nout = p.op == WDR_OP_BLOCKS ? g.nblk : 1;
        status = run_op(c, path, props, p.op, p, samples, st, s);
        if (status != WDR_OK && status != WDR_ENOCONV) return status;
    } else {
        // the block ratios here and the Schur ratio on the twin context's
        // stream, concurrently; both read the one path
        nout = g.nblk + 1;
        wdr_ctx *t = twin_of(c);
        hipEvent_t fork;
        WDR_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        WDR_HIP(hipEventRecord(fork, s));
        if (!t->aux && hipStreamCreateWithFlags(&t->aux, hipStreamNonBlocking) != hipSuccess) {
            (void)hipEventDestroy(fork);
            set_error("stream creation failed");
            return WDR_EDEVICE;
        }
        (void)hipStreamWaitEvent(t->aux, fork, 0);
        std::vector<double> sb, ss;
        Stats stb, sts;
        wdr_status es = WDR_OK;
        std::string msg;
        std::thread th([&] {
            (void)hipSetDevice(t->device);
            es = run_op(t, path, props, WDR_OP_SCHUR, p, ss, sts, t->aux);
            (void)hipStreamSynchronize(t->aux);
            if (es != WDR_OK) msg = wdr_last_error();
        });
        const wdr_status eb = run_op(c, path, props, WDR_OP_BLOCKS, p, sb, stb, s);
        th.join();
        (void)hipEventDestroy(fork);
        for (wdr_status x : {eb, es}) {
            if (x != WDR_OK && x != WDR_ENOCONV) {
                if (x == es) set_error(msg);
                return x;
            }
            if (x == WDR_ENOCONV) status = x;
        }
        if (es == WDR_ENOCONV) set_error(msg);
        st = summarize({stb, sts});
        samples.assign((size_t)total * nout, 0.0);
        for (int m = 0; m < total; ++m) {
            std::copy(sb.begin() + (size_t)m * g.nblk, sb.begin() + (size_t)(m + 1) * g.nblk,
                      samples.begin() + (size_t)m * nout);
            samples[(size_t)m * nout + g.nblk] = ss[m];
        }
    }
    if (host_samples) std::copy(samples.begin(), samples.end(), host_samples);
    if (host_log_ratios) {
        // per proposal: sum_i log( (1/K) sum_k exp(s_ik) ), summed over the
        // separate ratios (blocks, and the Schur complement for DD)
        for (int q = 0; q < P; ++q) {
            const double *sq = samples.data() + (size_t)q * per_prop * nout;
            double tot = 0;
            for (int b = 0; b < nout; ++b)
                for (int i = 0; i < N; ++i) {
                    double mx = -INFINITY;
                    for (int k = 0; k < K; ++k) mx = std::max(mx, sq[((size_t)i * K + k) * nout + b]);
                    double acc = 0;
                    for (int k = 0; k < K; ++k) acc += std::exp(sq[((size_t)i * K + k) * nout + b] - mx);
                    tot += mx + std::log(acc / K);
                }
            host_log_ratios[q] = tot;
        }
    }
    return status;
}

}  // namespace wdr
