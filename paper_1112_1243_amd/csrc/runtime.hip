// Contexts, geometry tables, workspace pool and gauge handles.
#include <algorithm>
#include <cstring>
#include <memory>
#include <string>

#include <atomic>
#include <cmath>

#include "runtime.h"

namespace wdr {

static thread_local std::string g_last_error = "no error";
void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error() { return g_last_error.c_str(); }

Work::Work(wdr_ctx *c, size_t bytes) : c_(c), bytes_(bytes), p_(nullptr)
{
    auto &fb = c->free_bufs;
    for (size_t i = 0; i < fb.size(); ++i)
        if (fb[i].bytes == bytes) {
            p_ = fb[i].p;
            fb.erase(fb.begin() + i);
            return;
        }
    if (hipMalloc(&p_, bytes) != hipSuccess) {
        p_ = nullptr;
        set_error("workspace allocation of " + std::to_string(bytes) + " bytes failed");
        return;
    }
    c->owned.push_back(p_);
}

Work::~Work()
{
    if (p_) c_->free_bufs.push_back({bytes_, p_});
}

Stats summarize(const std::vector<Stats> &v)
{
    Stats r;
    for (const Stats &x : v) {
        r.iters = std::max(r.iters, x.iters);
        r.converged = r.converged && x.converged;
        r.rel = std::max(r.rel, x.rel);
        r.total += x.total;
    }
    return r;
}

wdr_status check_ctx(const wdr_ctx *c)
{
    if (!c) {
        set_error("null context");
        return WDR_EINVAL;
    }
    return WDR_OK;
}

wdr_status check_blocks_usable(const wdr_ctx *c, bool solver)
{
    if (!c->g.colourable) {
        set_error("block operations need L[mu]/B[mu] even in every direction");
        return WDR_EINVAL;
    }
    if (solver && c->g.Vb > 256) {
        set_error("block solvers support blocks of at most 256 sites");
        return WDR_EINVAL;
    }
    return WDR_OK;
}

wdr_status check_params(const wdr_ctx *c, const wdr_solver_params &sp, bool needs_blocks)
{
    if (!(sp.tol > 0) || !(sp.block_tol > 0) || !(sp.adj_tol > 0) || sp.max_iter <= 0) {
        set_error("solver tolerances must be positive and max_iter >= 1");
        return WDR_EINVAL;
    }
    if (sp.block_mr_steps < 1 || sp.block_mr_steps > 1000) {
        set_error("block_mr_steps must be in [1, 1000]");
        return WDR_EINVAL;
    }
    if (sp.update_every < 1 || sp.update_every > 64 || (sp.graph != 0 && sp.graph != 1)) {
        set_error("update_every must be in [1, 64] and graph 0 or 1");
        return WDR_EINVAL;
    }
    if (sp.solver != WDR_SOLVER_FGCR_SAP && sp.solver != WDR_SOLVER_CGNE) {
        set_error("unknown solver");
        return WDR_EINVAL;
    }
    if (sp.inner != WDR_F64 && sp.inner != WDR_F32 && sp.inner != WDR_F16) {
        set_error("inner precision must be F64, F32 or F16");
        return WDR_EINVAL;
    }
    if (sp.middle != WDR_F64 && sp.middle != WDR_F32) {
        set_error("middle precision must be F64 or F32");
        return WDR_EINVAL;
    }
    if (sp.middle == WDR_F32 && (sp.solver != WDR_SOLVER_CGNE || sp.inner != WDR_F16)) {
        set_error("an F32 middle level needs CGNE with F16 inner iterations");
        return WDR_EINVAL;
    }
    if (sp.inner == WDR_F16) {
        // FP16 storage is implemented for 4^4 blocks: the Schwarz / block
        // solver and the even-odd CG (which also needs a 2-colourable
        // checkerboard of blocks)
        for (int mu = 0; mu < 4; ++mu)
            if (c->g.B[mu] != 4) {
                set_error("FP16 inner precision needs 4^4 blocks");
                return WDR_EINVAL;
            }
        if (sp.solver == WDR_SOLVER_CGNE && !c->g.colourable) {
            set_error("the FP16 even-odd CG needs L[mu]/B[mu] even in every direction");
            return WDR_EINVAL;
        }
    }
    if (sp.solver == WDR_SOLVER_FGCR_SAP || needs_blocks) {
        if (sp.restart < 1 || sp.restart > 16 || sp.sap_cycles < 1 || sp.mr_steps < 1) {
            set_error("FGCR restart must be in [1, 16], SAP cycles and MR steps >= 1");
            return WDR_EINVAL;
        }
        wdr_status st = check_blocks_usable(c, true);
        if (st != WDR_OK) return st;
    }
    return WDR_OK;
}

}  // namespace wdr

using namespace wdr;

namespace wdr {
const void *const *replicated(wdr_gauge *g, int k, int nsys, hipStream_t s)
{
    if (nsys > g->rep_cap) {
        int cap = 64;
        while (cap < nsys) cap *= 2;
        if (hipStreamSynchronize(s) != hipSuccess) return nullptr;  // launches may still read the old table
        void **rep = nullptr;
        if (hipMalloc(&rep, sizeof(void *) * 4 * cap) != hipSuccess) return nullptr;
        std::vector<void *> h(4 * (size_t)cap);
        void *src[4] = {g->u64, g->u32, g->u16, g->e16};
        for (int j = 0; j < 4; ++j)
            for (int m = 0; m < cap; ++m) h[(size_t)j * cap + m] = src[j];
        if (hipMemcpy(rep, h.data(), sizeof(void *) * h.size(), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(rep);
            return nullptr;
        }
        if (g->rep) (void)hipFree(g->rep);
        g->rep = rep;
        g->rep_cap = cap;
    }
    return g->rep + (size_t)k * g->rep_cap;
}
}  // namespace wdr

namespace wdr {
static std::atomic<long long> g_traffic{0};
void add_traffic(double bytes) { g_traffic.fetch_add((long long)bytes, std::memory_order_relaxed); }
}  // namespace wdr

extern "C" {

const char *wdr_last_error(void) { return wdr::last_error(); }

const char *wdr_status_str(wdr_status s)
{
    switch (s) {
    case WDR_OK: return "ok";
    case WDR_EINVAL: return "invalid argument";
    case WDR_ENOMEM: return "out of device memory";
    case WDR_EDEVICE: return "device error";
    case WDR_ENOCONV: return "solver did not converge";
    case WDR_ESTATE: return "handles do not belong together";
    }
    return "unknown status";
}

void wdr_default_solver_params(wdr_solver_params *out)
{
    if (!out) return;
    out->solver = WDR_SOLVER_FGCR_SAP;
    out->restart = 16;
    out->max_iter = 2000;
    out->sap_cycles = 4;
    out->mr_steps = 5;
    out->tol = 1e-10;
    out->block_tol = 1e-13;
    out->adj_tol = 1e-7;
    out->inner = WDR_F32;
    out->middle = WDR_F64;
    out->block_mr_steps = 16;
    out->update_every = 4;
    out->graph = 1;
}

wdr_status wdr_ctx_create(const wdr_geom *geom, int device, wdr_ctx **out)
{
    if (!geom || !out) {
        set_error("null argument");
        return WDR_EINVAL;
    }
    *out = nullptr;
    long V = 1, Vb = 1;
    for (int mu = 0; mu < 4; ++mu) {
        const int L = geom->L[mu], B = geom->B[mu];
        if (L <= 0 || B <= 0 || L % B != 0 || B % 2 != 0 || B > 255) {
            set_error("need 0 < B[mu] <= 255, B[mu] even and dividing L[mu]");
            return WDR_EINVAL;
        }
        if (geom->bc[mu] < -1 || geom->bc[mu] > 1) {
            set_error("bc[mu] must be -1, 0 or +1");
            return WDR_EINVAL;
        }
        V *= L;
        Vb *= B;
    }
    if (Vb > 65535 || V > (1L << 30)) {
        set_error("lattice or block too large");
        return WDR_EINVAL;
    }
    int ndev = 0;
    WDR_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) {
        set_error("no such device");
        return WDR_EINVAL;
    }
    WDR_HIP(hipSetDevice(device));
    {
        const wdr_status se = init_scratch(device);
        if (se != WDR_OK) return se;
    }

    wdr_ctx *c = new wdr_ctx();
    c->device = device;
    c->geom = *geom;
    Geo &g = c->g;
    int nblk = 1, colourable = 1;
    for (int mu = 0; mu < 4; ++mu) {
        g.L[mu] = geom->L[mu];
        g.B[mu] = geom->B[mu];
        g.NB[mu] = geom->L[mu] / geom->B[mu];
        g.bc[mu] = geom->bc[mu];
        nblk *= g.NB[mu];
        if (g.NB[mu] % 2) colourable = 0;
    }
    g.V = (int)V;
    g.Vb = (int)Vb;
    g.Vh = (int)Vb / 2;
    g.nblk = nblk;
    g.colourable = colourable;
    g.stencil = WDR_STENCIL_AUTO;
    g.mr_form = WDR_MR_AUTO;
    g.cg_form = WDR_CG_LAUNCHES;

    // in-block order: even sites then odd sites, lexicographic within each
    std::vector<uint32_t> loc_coord(Vb);
    std::vector<uint16_t> loc_index(Vb);
    {
        int ne = 0, no = (int)Vb / 2;
        for (int lex = 0; lex < Vb; ++lex) {
            int x[4], r = lex;
            for (int mu = 0; mu < 4; ++mu) {
                x[mu] = r % g.B[mu];
                r /= g.B[mu];
            }
            const int par = (x[0] + x[1] + x[2] + x[3]) & 1;
            const int l = par ? no++ : ne++;
            loc_coord[l] = (uint32_t)x[0] | ((uint32_t)x[1] << 8) | ((uint32_t)x[2] << 16) | ((uint32_t)x[3] << 24);
            loc_index[lex] = (uint16_t)l;
        }
    }
    // block slots: black blocks first (lexicographic), then white (paper Sec. 3)
    std::vector<int32_t> slot_blk(nblk), slot_nbr(8L * nblk);
    c->slot_of_block.assign(nblk, 0);
    {
        int nb = 0;
        for (int colour = 0; colour < 2; ++colour)
            for (int b = 0; b < nblk; ++b) {
                int r = b, sum = 0;
                for (int mu = 0; mu < 4; ++mu) {
                    sum += r % g.NB[mu];
                    r /= g.NB[mu];
                }
                if ((colourable ? (sum & 1) : 0) == colour) {
                    c->slot_of_block[b] = nb;
                    slot_blk[nb++] = b;
                }
            }
        g.nblack = 0;
        for (int b = 0; b < nblk; ++b) {
            int r = b, sum = 0;
            for (int mu = 0; mu < 4; ++mu) {
                sum += r % g.NB[mu];
                r /= g.NB[mu];
            }
            if (!colourable || (sum & 1) == 0) g.nblack++;
        }
        if (!colourable) g.nblack = nblk;
        for (int s = 0; s < nblk; ++s) {
            int n[4], r = slot_blk[s];
            for (int mu = 0; mu < 4; ++mu) {
                n[mu] = r % g.NB[mu];
                r /= g.NB[mu];
            }
            for (int mu = 0; mu < 4; ++mu)
                for (int d = 0; d < 2; ++d) {
                    int m[4] = {n[0], n[1], n[2], n[3]};
                    m[mu] = (m[mu] + (d == 0 ? 1 : g.NB[mu] - 1)) % g.NB[mu];
                    const int bl = m[0] + g.NB[0] * (m[1] + g.NB[1] * (m[2] + g.NB[2] * m[3]));
                    slot_nbr[8 * s + 2 * mu + d] = bl;  // block id for now, slot below
                }
        }
        for (auto &v : slot_nbr) v = c->slot_of_block[v];
    }

    // XCD-aware schedules: the slots of a range in lexicographic block order
    // (mu = 0 fastest), cut into 8 contiguous chunks; workgroup i (on XCD
    // i % 8) takes the (i / 8)-th block of chunk i % 8.  For a lattice of 8
    // blocks in time each XCD then owns one time slab, whose x and y
    // neighbours run close in time and meet in its L2 (a Morton order was
    // measured to miss L2 more often: its regions cut x and y faces, whose
    // sites spread over every cache line of a block).
    std::vector<int32_t> sched[3];
    for (int r = 0; r < 3; ++r) {
        std::vector<int32_t> order;
        for (int b = 0; b < nblk; ++b) {
            const int sl = c->slot_of_block[b];
            const bool black = sl < g.nblack;
            if (r == 2 || (r == 0 && black) || (r == 1 && !black)) order.push_back(sl);
        }
        const int n = (int)order.size(), q = n / 8, rem = n % 8;
        sched[r].assign(n, 0);
        for (int i = 0; i < n; ++i) {
            const int xcd = i % 8, t = i / 8;
            const int start = xcd * q + std::min(xcd, rem);
            sched[r][i] = order[start + t];
        }
    }

    const size_t b1 = Vb * sizeof(uint32_t), b2 = Vb * sizeof(uint16_t), b3 = 8L * nblk * sizeof(int32_t),
                 b4 = nblk * sizeof(int32_t);
    const size_t o2 = (b1 + 255) & ~255ul, o3 = o2 + ((b2 + 255) & ~255ul), o4 = o3 + ((b3 + 255) & ~255ul);
    const size_t o5 = o4 + ((b4 + 255) & ~255ul), o6 = o5 + ((sched[0].size() * 4 + 255) & ~255ul),
                 o7 = o6 + ((sched[1].size() * 4 + 255) & ~255ul);
    const size_t total = o7 + sched[2].size() * 4 + 256;
    if (hipMalloc(&c->tables, total) != hipSuccess) {
        set_error("context allocation failed");
        wdr_ctx_destroy(c);
        return WDR_ENOMEM;
    }
    char *t = static_cast<char *>(c->tables);
    if (hipMemcpy(t, loc_coord.data(), b1, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t + o2, loc_index.data(), b2, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t + o3, slot_nbr.data(), b3, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t + o4, slot_blk.data(), b4, hipMemcpyHostToDevice) != hipSuccess ||
        (sched[0].size() && hipMemcpy(t + o5, sched[0].data(), sched[0].size() * 4, hipMemcpyHostToDevice) != hipSuccess) ||
        (sched[1].size() && hipMemcpy(t + o6, sched[1].data(), sched[1].size() * 4, hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemcpy(t + o7, sched[2].data(), sched[2].size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
        set_error("context upload failed");
        wdr_ctx_destroy(c);
        return WDR_EDEVICE;
    }
    g.loc_coord = reinterpret_cast<const uint32_t *>(t);
    g.loc_index = reinterpret_cast<const uint16_t *>(t + o2);
    g.slot_nbr = reinterpret_cast<const int32_t *>(t + o3);
    g.slot_blk = reinterpret_cast<const int32_t *>(t + o4);
    g.sched[0] = reinterpret_cast<const int32_t *>(t + o5);
    g.sched[1] = reinterpret_cast<const int32_t *>(t + o6);
    g.sched[2] = reinterpret_cast<const int32_t *>(t + o7);
    *out = c;
    return WDR_OK;
}

wdr_status wdr_ctx_destroy(wdr_ctx *c)
{
    if (!c) return WDR_OK;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    if (c->twin) wdr_ctx_destroy(c->twin);  // tables NULL: the twin frees only its own pool
    for (void *p : c->owned) (void)hipFree(p);
    if (c->tables) (void)hipFree(c->tables);
    if (c->poll_host) (void)hipHostFree(c->poll_host);
    if (c->poll_val) (void)hipHostFree(c->poll_val);
    for (hipEvent_t e : c->poll_ev)
        if (e) (void)hipEventDestroy(e);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
    return WDR_OK;
}

int64_t wdr_ctx_volume(const wdr_ctx *c) { return c ? c->g.V : 0; }

int64_t wdr_traffic(int32_t reset)
{
    return reset ? (int64_t)g_traffic.exchange(0) : (int64_t)g_traffic.load();
}
int32_t wdr_ctx_nblocks(const wdr_ctx *c) { return c ? c->g.nblk : 0; }

wdr_status wdr_ctx_set_stencil(wdr_ctx *c, int32_t choice)
{
    if (!c) {
        set_error("null context");
        return WDR_EINVAL;
    }
    if (choice < WDR_STENCIL_AUTO || choice > WDR_STENCIL_BLK) {
        set_error("stencil choice must be WDR_STENCIL_AUTO, WDR_STENCIL_DIR or WDR_STENCIL_BLK");
        return WDR_EINVAL;
    }
    c->g.stencil = choice;
    if (c->twin) c->twin->g.stencil = choice;
    return WDR_OK;
}

wdr_status wdr_ctx_set_mr_form(wdr_ctx *c, int32_t choice)
{
    if (!c) {
        set_error("null context");
        return WDR_EINVAL;
    }
    if (choice < WDR_MR_AUTO || choice > WDR_MR_TWO_PER_CU) {
        set_error("block-MR form must be WDR_MR_AUTO, WDR_MR_ONE_PER_CU or WDR_MR_TWO_PER_CU");
        return WDR_EINVAL;
    }
    c->g.mr_form = choice;
    if (c->twin) c->twin->g.mr_form = choice;
    return WDR_OK;
}

wdr_status wdr_ctx_set_cg_form(wdr_ctx *c, int32_t choice)
{
    if (!c) {
        set_error("null context");
        return WDR_EINVAL;
    }
    if (choice != WDR_CG_LAUNCHES && choice != WDR_CG_PERSISTENT) {
        set_error("CG form must be WDR_CG_LAUNCHES or WDR_CG_PERSISTENT");
        return WDR_EINVAL;
    }
    c->g.cg_form = choice;
    if (c->twin) c->twin->g.cg_form = choice;
    return WDR_OK;
}

wdr_status wdr_gauge_create(wdr_ctx *c, const double *dev_U, wdr_gauge **out, void *stream)
{
    if (check_ctx(c) != WDR_OK) return WDR_EINVAL;
    if (!dev_U || !out) {
        set_error("null argument");
        return WDR_EINVAL;
    }
    WDR_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<wdr_gauge, wdr_status (*)(wdr_gauge *)> g(new wdr_gauge(), wdr_gauge_destroy);
    g->ctx = c;
    g->device = c->device;
    const size_t n = (size_t)c->g.V * 36;
    if (hipMalloc(&g->u64, n * sizeof(double2)) != hipSuccess || hipMalloc(&g->u32, n * sizeof(float2)) != hipSuccess ||
        hipMalloc(&g->tab, 6 * sizeof(void *)) != hipSuccess) {
        set_error("gauge allocation failed");
        return WDR_ENOMEM;
    }
    launch_pack_gauge<double>(c->g, c->geom.bc, reinterpret_cast<const double2 *>(dev_U), g->u64, s);
    launch_convert_gauge_f32(c->g, g->u64, g->u32, s);
    {
        // kernels that rebuild the third row of a link need SU(3) links
        Work part(c, sizeof(double) * ((size_t)c->g.V * 4 / 256 + 2));
        if (!part.ok()) return WDR_ENOMEM;
        launch_su3_deviation(c->g, reinterpret_cast<const double2 *>(dev_U), part.as<double>(),
                             part.as<double>() + ((size_t)c->g.V * 4 + 255) / 256, s);
        double dev = 1e300;
        WDR_HIP(hipMemcpyAsync(&dev, part.as<double>() + ((size_t)c->g.V * 4 + 255) / 256, sizeof(double),
                               hipMemcpyDeviceToHost, s));
        WDR_HIP(hipStreamSynchronize(s));
        g->su3 = dev <= SU3_TOL;
    }
    if (g->su3) {  // FP16 two-row copy for the FP16 inner solver
        if (hipMalloc(&g->u16, (size_t)c->g.V * 24 * sizeof(h2)) != hipSuccess) {
            set_error("gauge allocation failed");
            return WDR_ENOMEM;
        }
        launch_pack_links_h16(c->g, g->u64, g->u16, s);
        if (e16_geometry(c->g)) {
            if (hipMalloc(&g->e16, (size_t)c->g.V * 24 * sizeof(h2)) != hipSuccess) {
                set_error("gauge allocation failed");
                return WDR_ENOMEM;
            }
            launch_pack_links_e16(c->g, g->u64, g->e16, s);
        }
    }
    void *tab[6] = {g->u64, g->u32, g->u16, g->e16, nullptr, nullptr};
    WDR_HIP(hipMemcpyAsync(g->tab, tab, sizeof(tab), hipMemcpyHostToDevice, s));
    WDR_HIP(hipStreamSynchronize(s));
    WDR_HIP(hipGetLastError());
    *out = g.release();
    return WDR_OK;
}

int32_t wdr_gauge_is_su3(const wdr_gauge *g) { return g && g->su3 ? 1 : 0; }

wdr_status wdr_gauge_set_clover(wdr_ctx *c, wdr_gauge *U, double csw, double kappa, void *stream)
{
    if (check_ctx(c) != WDR_OK) return WDR_EINVAL;
    if (!U) {
        set_error("null gauge handle");
        return WDR_EINVAL;
    }
    if (U->ctx != c) {
        set_error("gauge handle belongs to another context");
        return WDR_ESTATE;
    }
    if (!std::isfinite(csw) || !std::isfinite(kappa) || (csw != 0 && !(kappa > 0))) {
        set_error("csw must be finite and kappa positive");
        return WDR_EINVAL;
    }
    for (int mu = 0; mu < 4; ++mu)
        if (csw != 0 && c->geom.bc[mu] == 0) {
            set_error("the clover term needs periodic or antiperiodic boundaries (bc = +1 / -1) in every direction");
            return WDR_EINVAL;
        }
    WDR_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    // launches already queued may read the old term
    WDR_HIP(hipStreamSynchronize(s));
    WDR_HIP(hipDeviceSynchronize());
    if (U->c64) (void)hipFree(U->c64);
    if (U->c32) (void)hipFree(U->c32);
    U->c64 = nullptr;
    U->c32 = nullptr;
    U->csw = U->ckappa = 0;
    void *none[2] = {nullptr, nullptr};
    WDR_HIP(hipMemcpy(U->tab + 4, none, sizeof(none), hipMemcpyHostToDevice));
    if (csw == 0) return WDR_OK;
    const size_t n = (size_t)c->g.V * 144;
    if (hipMalloc(&U->c64, n * sizeof(double)) != hipSuccess || hipMalloc(&U->c32, n * sizeof(float)) != hipSuccess) {
        set_error("clover allocation failed");
        return WDR_ENOMEM;
    }
    {
        Work w(c, clover_work_bytes(c->g) + sizeof(double));
        if (!w.ok()) return WDR_ENOMEM;
        double *worst = reinterpret_cast<double *>(w.as<char>() + clover_work_bytes(c->g));
        launch_clover_build(c->g, U->u64, csw, kappa, w.as<void>(), U->c64, U->c32, worst, s);
        double h = 0;
        WDR_HIP(hipMemcpyAsync(&h, worst, sizeof(double), hipMemcpyDeviceToHost, s));
        WDR_HIP(hipStreamSynchronize(s));
        WDR_HIP(hipGetLastError());
        if (!(h < 1e8)) {
            (void)hipFree(U->c64);
            (void)hipFree(U->c32);
            U->c64 = nullptr;
            U->c32 = nullptr;
            set_error("the clover term has a (nearly) singular block: largest 1/|pivot| " + std::to_string(h));
            return WDR_EINVAL;
        }
    }
    void *ct[2] = {U->c64, U->c32};
    WDR_HIP(hipMemcpy(U->tab + 4, ct, sizeof(ct), hipMemcpyHostToDevice));
    U->csw = csw;
    U->ckappa = kappa;
    return WDR_OK;
}

wdr_status wdr_gauge_destroy(wdr_gauge *g)
{
    if (!g) return WDR_OK;
    (void)hipSetDevice(g->device);
    (void)hipDeviceSynchronize();
    if (g->u64) (void)hipFree(g->u64);
    if (g->u32) (void)hipFree(g->u32);
    if (g->u16) (void)hipFree(g->u16);
    if (g->e16) (void)hipFree(g->e16);
    if (g->c64) (void)hipFree(g->c64);
    if (g->c32) (void)hipFree(g->c32);
    if (g->rep) (void)hipFree(g->rep);
    if (g->tab) (void)hipFree(g->tab);
    delete g;
    return WDR_OK;
}

}  // extern "C"
