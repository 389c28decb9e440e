// Host runtime behind the C ABI: contexts, gauge handles, workspaces and
// the solver / estimator drivers.
#pragma once

#include <vector>

#include "ops.h"

struct wdr_ctx {
    int device = 0;
    wdr_geom geom{};
    wdr::Geo g{};
    void *tables = nullptr;        // loc_coord, loc_index, slot_nbr, slot_blk
    double *red = nullptr;         // reduction scratch (RED_SCRATCH doubles)
    double2 *scal = nullptr;       // device scalars (SCAL_N complex)
    const void **ptrs = nullptr;   // device array of field pointers (PTRS_N)
    struct Buf {
        size_t bytes;
        void *p;
    };
    std::vector<Buf> free_bufs;    // workspace pool
    std::vector<void *> owned;     // every pool allocation
    std::vector<int> slot_of_block;  // host copy: slot of each lexicographic block
};

struct wdr_gauge {
    wdr_ctx *ctx = nullptr;  // identity check only: a gauge may outlive its context
    int device = 0;
    double2 *u64 = nullptr;  // internal FP64 links, boundary phases folded in
    float2 *u32 = nullptr;   // internal FP32 copy
};

namespace wdr {

constexpr int SCAL_N = 512;
constexpr int PTRS_N = 64;

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

// a gauge field in the internal layout, FP64 with an FP32 copy
struct GaugeView {
    const double2 *u64;
    const float2 *u32;
};
inline GaugeView view(const wdr_gauge *g) { return {g->u64, g->u32}; }

struct Stats {
    int iters = 0;
    int converged = 1;
    double rel = 0;
    long total = 0;
    void merge(const Stats &o)
    {
        iters = o.iters;
        converged = converged && o.converged;
        rel = o.rel;
        total += o.total;
    }
};

// slot ranges of the block colours
inline void colour_slots(const wdr_ctx *c, int colour, int &slot0, int &n)
{
    if (colour == 0) { slot0 = 0; n = c->g.nblack; }
    else if (colour == 1) { slot0 = c->g.nblack; n = c->g.nblk - c->g.nblack; }
    else { slot0 = 0; n = c->g.nblk; }
}

// ---- drivers (internal FP64 fields) ----
// D, Dirichlet blocks of a colour, or cross-block hops from a colour
void apply_D64(wdr_ctx *c, GaugeView U, double kappa, const double2 *in, double2 *out, hipStream_t s);
wdr_status sap64(wdr_ctx *c, GaugeView U, double kappa, const wdr_solver_params &sp, const double2 *in,
                 double2 *out, hipStream_t s);
wdr_status solve64(wdr_ctx *c, GaugeView U, double kappa, const wdr_solver_params &sp, double tol,
                   const double2 *b, double2 *x, Stats &st, hipStream_t s);
wdr_status block_solve64(wdr_ctx *c, GaugeView U, double kappa, int colour, const wdr_solver_params &sp,
                         double tol, const double2 *b, double2 *x, Stats &st, hipStream_t s);
wdr_status schur64(wdr_ctx *c, GaugeView U, double kappa, const wdr_solver_params &sp, const double2 *in,
                   double2 *out, Stats &st, hipStream_t s);
wdr_status logdet_ratio(wdr_ctx *c, const wdr_gauge *U, const wdr_gauge *Up, double kappa, const wdr_est_params &p,
                        double *host_samples, double *host_log_ratio, Stats &st, hipStream_t s);

// validation helpers
wdr_status check_ctx(const wdr_ctx *c);
wdr_status check_blocks_usable(const wdr_ctx *c, bool solver);
wdr_status check_params(const wdr_ctx *c, const wdr_solver_params &sp, bool needs_blocks);

}  // namespace wdr
