// Host runtime behind the C ABI: contexts, gauge handles, workspaces and
// the solver / estimator drivers.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "ops.h"

struct wdr_ctx {
    int device = 0;
    wdr_geom geom{};
    wdr::Geo g{};
    void *tables = nullptr;        // loc_coord, loc_index, slot_nbr, slot_blk
    struct Buf {
        size_t bytes;
        void *p;
    };
    std::vector<Buf> free_bufs;    // workspace pool
    std::vector<void *> owned;     // every pool allocation
    std::vector<int> slot_of_block;  // host copy: slot of each lexicographic block
    // pinned host copies of per-system solver flags (two slots, grown on
    // demand) and their events: solver loops poll them without stalling
    int32_t *poll_host = nullptr;
    size_t poll_cap = 0;
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
    // pinned copies of per-system residual norms read with the flags (two
    // slots of M, then M reference norms)
    double2 *poll_val = nullptr;
    size_t poll_val_cap = 0;
    // stream of this context's group in a batch over several contexts
    // (created on first use, default priority)
    hipStream_t aux = nullptr;
    // a context of the same geometry with its own pool, read-back buffers and
    // stream, for the concurrent half of a DD estimate (created on first use;
    // shares this context's geometry tables)
    wdr_ctx *twin = nullptr;
    // stream on which solver periods are captured into HIP graphs (created on first use)
    hipStream_t cap = nullptr;
    // autotuned solver schedules and launch forms (wdr_stencil, wdr_mr_form),
    // keyed by (ratio, solver, inner and middle precision, kappa)
    std::map<std::string, wdr_solver_params> tuned;
    std::map<std::string, std::pair<int, int>> tuned_forms;
};

struct wdr_gauge {
    wdr_ctx *ctx = nullptr;  // identity check only: a gauge may outlive its context
    int device = 0;
    double2 *u64 = nullptr;  // internal FP64 links, boundary phases folded in
    float2 *u32 = nullptr;   // internal FP32 copy
    wdr::h2 *u16 = nullptr;  // FP16 copy of the first two rows (SU(3) fields only)
    wdr::h2 *e16 = nullptr;  // the same in the even-odd CG's layout (SU(3) fields, 4^4 blocks)
    // clover term (wdr_gauge_set_clover): A and A^-1 in FP64 and FP32, the
    // coefficient and the hopping parameter they were built with (csw = 0:
    // none)
    double *c64 = nullptr;
    float *c32 = nullptr;
    double csw = 0, ckappa = 0;
    void **tab = nullptr;    // device table {u64, u32, u16, e16, c64, c32} for single-system launches
    int su3 = 0;             // every link is SU(3) to SU3_TOL (checked at upload)
    // the same four pointers repeated for launches of several systems on this
    // field: rep + k * rep_cap holds rep_cap copies of entry k of tab
    void **rep = nullptr;
    int rep_cap = 0;
};

namespace wdr {
// device address of wdr_apply_D_noalloc's static staging array on `device`
// (the current device), looked up once per device
wdr_status init_scratch(int device);
}  // namespace wdr

// largest |U U^+ - 1| and |det U - 1| entry for which a gauge field counts as
// SU(3), so that kernels may rebuild the third row of its links
constexpr double SU3_TOL = 1e-10;

namespace wdr {


// workspace buffers, returned to the context pool on destruction
class Work {
  public:
    Work(wdr_ctx *c, size_t bytes);
    ~Work();
    Work(const Work &) = delete;
    Work &operator=(const Work &) = delete;
    template <typename P> P *as() const { return static_cast<P *>(p_); }
    bool ok() const { return p_ != nullptr; }

  private:
    wdr_ctx *c_;
    size_t bytes_;
    void *p_;
};

inline size_t field_bytes(const wdr_ctx *c, int prec)
{
    return (size_t)c->g.V * 12 * (prec == WDR_F64 ? sizeof(double2) : prec == WDR_F32 ? sizeof(float2) : 4);
}
inline long field_n(const wdr_ctx *c) { return (long)c->g.V * 12; }
// an FP16 field of the C ABI: 12 V FP16 complex values (internal layout),
// then one float scale per block slot
inline size_t f16_field_bytes(const wdr_ctx *c) { return (size_t)c->g.V * 12 * 4 + (size_t)c->g.nblk * 4; }
inline wdr::H16 f16_field(const wdr_ctx *c, void *p)
{
    wdr::h2 *v = static_cast<wdr::h2 *>(p);
    return wdr::H16{v, reinterpret_cast<float *>(v + (size_t)c->g.V * 12)};
}

// device table of nsys copies of entry k (0 u64, 1 u32, 2 u16, 3 e16) of the
// gauge's pointers (grown, and the stream synchronised, when too short);
// NULL if the allocation fails
const void *const *replicated(wdr_gauge *g, int k, int nsys, hipStream_t s);

// per-system gauge tables (device arrays of M pointers)
struct GaugeTab {
    Links<double> u64;
    Links<float> u32;
    Links16 u16;  // tab NULL when the fields are not SU(3)
    Links16 e16;  // E16 links of the FP16 even-odd CG; tab NULL when absent
};
inline GaugeTab view(const wdr_gauge *g)
{
    GaugeTab t{{reinterpret_cast<UTab<double>>(g->tab), g->su3},
               {reinterpret_cast<UTab<float>>(g->tab + 1), g->su3},
               {g->u16 ? reinterpret_cast<const h2 *const *>(g->tab + 2) : nullptr},
               {g->e16 ? reinterpret_cast<const h2 *const *>(g->tab + 3) : nullptr}};
    if (g->c64) {
        t.u64.ctab = reinterpret_cast<const double *const *>(g->tab + 4);
        t.u32.ctab = reinterpret_cast<const float *const *>(g->tab + 5);
    }
    return t;
}

// bytes per site of one clover block pair (A or A^-1) in precision T
template <typename T> constexpr double clov_b() { return 72.0 * sizeof(T); }

// ---- algorithmic traffic: the compulsory device-memory bytes of the work
// done (every operand of a kernel read or written once: spinors of the sites
// a kernel covers, each link and each neighbour counted once), summed over
// the process and read by wdr_traffic.  The drivers add their totals from
// the exact work counts (iterations, updates, rounds) of every system, so
// launches that skip converged systems add nothing.
void add_traffic(double bytes);
// bytes per lattice site: a spinor of precision T (24 reals), the two-row
// links of a site (4 links x 12 reals), an FP16 half-field site (48 bytes)
template <typename T> constexpr double spin_b() { return 24.0 * sizeof(T); }
template <typename T> constexpr double link_b() { return 48.0 * sizeof(T); }
// one even-odd half of the stencil over V sites (V / 2 outputs, V / 2
// inputs, every link of the lattice), with or without a diagonal term
template <typename T> constexpr double half_b(double V, bool diag)
{
    return V / 2 * (diag ? 3 : 2) * spin_b<T>() + V * link_b<T>();
}

struct Stats {
    int iters = 0;
    int converged = 1;
    double rel = 0;
    long total = 0;
};
// summary over the systems of a batch: max iterations, all converged, max
// residual, summed iterations
Stats summarize(const std::vector<Stats> &v);

inline Sys all_sys(const wdr_ctx *c, int M) { return Sys{M, nullptr, field_n(c)}; }

// slot ranges of the block colours
inline void colour_slots(const wdr_ctx *c, int colour, int &slot0, int &n)
{
    if (colour == 0) { slot0 = 0; n = c->g.nblack; }
    else if (colour == 1) { slot0 = c->g.nblack; n = c->g.nblk - c->g.nblack; }
    else { slot0 = 0; n = c->g.nblk; }
}

// ---- drivers: batches of M systems, internal FP64 fields [M][12 V] ----
void apply_D64(wdr_ctx *c, const Sys &sy, const GaugeTab &U, double kappa, const double2 *in, double2 *out,
               hipStream_t s);
wdr_status sap64(wdr_ctx *c, const Sys &sy, const GaugeTab &U, double kappa, const wdr_solver_params &sp,
                 const double2 *in, double2 *out, hipStream_t s);
wdr_status solve64(wdr_ctx *c, int M, const GaugeTab &U, double kappa, const wdr_solver_params &sp, double tol,
                   const double2 *b, double2 *x, std::vector<Stats> &st, hipStream_t s);
wdr_status block_solve64(wdr_ctx *c, int M, const GaugeTab &U, double kappa, int colour, const wdr_solver_params &sp,
                         double tol, const double2 *b, double2 *x, std::vector<Stats> &st, hipStream_t s);
wdr_status schur64(wdr_ctx *c, int M, const GaugeTab &U, double kappa, const wdr_solver_params &sp,
                   const double2 *in, double2 *out, std::vector<Stats> &st, hipStream_t s);
// one proposal U -> U' of an estimate (links on the estimate's context)
struct Proposal {
    const wdr_gauge *U, *Up;
    double kappa;
    uint64_t seed;
};
// every (proposal, step, noise) sample of the proposals is one system of the
// batched launches; samples [proposal][step][noise](x nblk for BLOCKS),
// log ratios per proposal
// log det(D_b^+ D_b) of every block for U0 (and U1 when not null): out[f *
// nblk + b] by lexicographic block id b
wdr_status block_logdet(wdr_ctx *c, const wdr_gauge *U0, const wdr_gauge *U1, double kappa, int max_blocks,
                        double *out, hipStream_t s);
// heat-bath sweep of the masked links of the canonical field U (8 launches)
void launch_heatbath(const wdr_ctx *c, double beta, const uint8_t *mask, uint64_t seed, int sweep, double2 *U,
                     hipStream_t s);
// relative gauge fixing of the canonical field Up to U, in place
void launch_relgauge(const wdr_ctx *c, const double2 *U, double2 *Up, int sweeps, hipStream_t s);
// over-relaxation sweep of the masked links of the canonical field U
void launch_overrelax(const wdr_ctx *c, const uint8_t *mask, double2 *U, hipStream_t s);
// one step of the hierarchical filter on the canonical field U (in place)
// (p == nullptr: block steps only)
wdr_status filter_step(wdr_ctx *c, double beta, double kappa, const uint8_t *mask, int n_block_steps,
                       const wdr_est_params *p, uint64_t seed, double2 *U, uint8_t *accepts, wdr_filter_info &info,
                       hipStream_t s);
wdr_status logdet_ratio(wdr_ctx *c, const std::vector<Proposal> &props, const wdr_est_params &p,
                        double *host_samples, double *host_log_ratios, Stats &st, hipStream_t s);

// validation helpers
wdr_status check_ctx(const wdr_ctx *c);
wdr_status check_blocks_usable(const wdr_ctx *c, bool solver);
wdr_status check_params(const wdr_ctx *c, const wdr_solver_params &sp, bool needs_blocks);

}  // namespace wdr
