// extern "C" entry points of include/wdr.h: argument checks, canonical <->
// internal layout conversion, and dispatch to the drivers.
#include <algorithm>
#include <thread>
#include <chrono>
#include <cmath>
#include <mutex>

#include "runtime.h"

using namespace wdr;

namespace {

// Staging area of wdr_apply_D_noalloc: the two internal-layout fields of a
// call live in this static device array, which every device the library runs
// on holds until the process ends.  Host code never passes the array's name
// to a kernel or a copy (on the host it is only a stand-in): scratch_dev[d]
// holds device d's address of its copy, taken by init_scratch.
constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;
constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
std::mutex scratch_mu;
void *scratch_dev[MAX_DEVICES];

hipStream_t S(void *stream) { return (hipStream_t)stream; }

wdr_status pre(wdr_ctx *c, const void *a, const void *b)
{
    if (check_ctx(c) != WDR_OK) return WDR_EINVAL;
    if (!a || !b) {
        set_error("null field pointer");
        return WDR_EINVAL;
    }
    if (hipSetDevice(c->device) != hipSuccess) {
        set_error("hipSetDevice failed");
        return WDR_EDEVICE;
    }
    return WDR_OK;
}

// clover_ok: the call supports gauge fields that carry a clover term, whose
// hopping parameter must then be kappa; every other call refuses them
wdr_status check_gauge(const wdr_ctx *c, const wdr_gauge *U, bool clover_ok = false, double kappa = 0)
{
    if (!U) {
        set_error("null gauge handle");
        return WDR_EINVAL;
    }
    if (U->ctx != c) {
        set_error("gauge handle belongs to another context");
        return WDR_ESTATE;
    }
    if (U->c64) {
        if (!clover_ok) {
            set_error("this call does not support a gauge field with a clover term (supported: D, D_b, the block "
                      "hops and D_ee in F64 / F32; CGNE and FGCR solves and the Schwarz procedure; block solves "
                      "and the Schur complement; FULL, BLOCKS, SCHUR and DD estimates; exact block "
                      "determinants)");
            return WDR_EINVAL;
        }
        if (kappa != U->ckappa) {
            set_error("kappa differs from the hopping parameter the clover term was built with");
            return WDR_EINVAL;
        }
    }
    return WDR_OK;
}

wdr_status check_pair(const wdr_gauge *U, const wdr_gauge *Up)
{
    if (U->csw != Up->csw) {
        set_error("the two gauge fields of a ratio must carry the same clover coefficient");
        return WDR_EINVAL;
    }
    return WDR_OK;
}

wdr_status check_kappa(double kappa)
{
    if (!(kappa > 0) || !std::isfinite(kappa)) {
        set_error("kappa must be positive");
        return WDR_EINVAL;
    }
    return WDR_OK;
}

wdr_status finish(hipStream_t s)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
        return WDR_EDEVICE;
    }
    (void)s;
    return WDR_OK;
}

// runs op(in_internal, out_internal) in precision T on canonical FP64 fields
template <typename T, class F>
wdr_status with_fields(wdr_ctx *c, const double *in, double *out, hipStream_t s, F &&op)
{
    const int prec = sizeof(T) == 8 ? WDR_F64 : WDR_F32;
    Work a(c, field_bytes(c, prec)), b(c, field_bytes(c, prec));
    if (!a.ok() || !b.ok()) return WDR_ENOMEM;
    typedef typename C2<T>::type T2;
    launch_pack_spinor<T>(c->g, reinterpret_cast<const double2 *>(in), a.as<T2>(), s);
    launch_zero<T>(b.as<T2>(), field_n(c), s);
    op(a.as<T2>(), b.as<T2>());
    launch_unpack_spinor<T>(c->g, b.as<T2>(), reinterpret_cast<double2 *>(out), s);
    return finish(s);
}

// the links of U in precision T, with clover mode cmode for a clover term
template <typename T> Links<T> links(const wdr_gauge *U, int cmode = CLOV_DIAG);
template <> Links<double> links<double>(const wdr_gauge *U, int cmode)
{
    Links<double> L = view(U).u64;
    L.cmode = cmode;
    return L;
}
template <> Links<float> links<float>(const wdr_gauge *U, int cmode)
{
    Links<float> L = view(U).u32;
    L.cmode = cmode;
    return L;
}

template <typename T>
wdr_status stencil_call(wdr_ctx *c, const wdr_gauge *U, double kappa, int kind, int arg, const double *in,
                        double *out, hipStream_t s)
{
    typedef typename C2<T>::type T2;
    const Geo &g = c->g;
    Sys one = all_sys(c, 1);
    return with_fields<T>(c, in, out, s, [&](T2 *a, T2 *b) {
        const T k = (T)kappa;
        if (kind == 0) {  // D
            launch_dslash<T>(g, one, links<T>(U), HOPS_ALL, -1, 0, a, a, b, k, 0, g.nblk, s);
        } else if (kind == 1) {  // Dirichlet blocks of colour arg
            int s0, n;
            colour_slots(c, arg, s0, n);
            launch_dslash<T>(g, one, links<T>(U), HOPS_IN, -1, 0, a, a, b, k, s0, n, s);
        } else if (kind == 2) {  // hops from colour arg to the other colour
            int s0, n;
            colour_slots(c, 1 - arg, s0, n);
            launch_dslash<T>(g, one, links<T>(U), HOPS_CROSS, -1, 0, a, nullptr, b, k, s0, n, s);
        } else {  // even-odd reduced, blocked = arg: A_ee - kappa^2 H_eo A_oo^-1 H_oe
            Work t(c, field_bytes(c, sizeof(T) == 8 ? WDR_F64 : WDR_F32));
            const int hops = arg ? HOPS_IN : HOPS_ALL;
            launch_dslash<T>(g, one, links<T>(U, CLOV_INV), hops, 1, 0, a, nullptr, t.as<T2>(), k, 0, g.nblk, s);
            launch_dslash<T>(g, one, links<T>(U), hops, 0, 0, t.as<T2>(), a, b, (T)(-kappa), 0, g.nblk, s);
        }
    });
}

wdr_status stencil_entry(wdr_ctx *c, const wdr_gauge *U, double kappa, wdr_prec prec, int kind, int arg,
                         const double *in, double *out, void *stream)
{
    wdr_status e = pre(c, in, out);
    if (e != WDR_OK) return e;
    if ((e = check_gauge(c, U, prec == WDR_F64 || prec == WDR_F32, kappa)) != WDR_OK) return e;
    if ((e = check_kappa(kappa)) != WDR_OK) return e;
    if ((kind == 1 || kind == 2) && (e = check_blocks_usable(c, false)) != WDR_OK) return e;
    if (prec == WDR_F64) return stencil_call<double>(c, U, kappa, kind, arg, in, out, S(stream));
    if (prec == WDR_F32) return stencil_call<float>(c, U, kappa, kind, arg, in, out, S(stream));
    if (prec == WDR_F16 && kind == 0) {  // D on FP16 fields with per-block scales
        Work a(c, f16_field_bytes(c)), b(c, f16_field_bytes(c));
        if (!a.ok() || !b.ok()) return WDR_ENOMEM;
        if ((e = wdr_pack(c, WDR_F16, in, a.as<void>(), stream)) != WDR_OK) return e;
        if ((e = wdr_apply_D_internal(c, U, kappa, WDR_F16, a.as<void>(), b.as<void>(), stream)) != WDR_OK) return e;
        return wdr_unpack(c, WDR_F16, b.as<void>(), out, stream);
    }
    set_error(prec == WDR_F16 ? "FP16 is available for D only" : "precision must be F64, F32 or F16");
    return WDR_EINVAL;
}

void fill_info(wdr_solve_info *info, const Stats &st, double secs)
{
    if (!info) return;
    info->iters = st.iters;
    info->converged = st.converged;
    info->true_rel_resid = st.rel;
    info->seconds = secs;
    info->total_iters = st.total;
}

double now()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

namespace wdr {
// the address of the staging array on `device` (the current device), once
// per device; called by wdr_ctx_create
wdr_status init_scratch(int device)
{
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (device < 0 || device >= MAX_DEVICES) {
        set_error("device index beyond the staging table");
        return WDR_EINVAL;
    }
    if (scratch_dev[device]) return WDR_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        set_error(std::string("hipGetSymbolAddress of the staging array: ") + hipGetErrorString(e));
        return WDR_EDEVICE;
    }
    scratch_dev[device] = p;
    return WDR_OK;
}
}  // namespace wdr

extern "C" {

wdr_status wdr_site_maps(wdr_ctx *c, int32_t *bid, int32_t *col, int32_t *par, int32_t *pos, void *stream)
{
    if (check_ctx(c) != WDR_OK) return WDR_EINVAL;
    WDR_HIP(hipSetDevice(c->device));
    launch_site_maps(c->g, bid, col, par, pos, S(stream));
    return finish(S(stream));
}

wdr_status wdr_active_links(wdr_ctx *c, int32_t lo, int32_t hi, uint8_t *mask, void *stream)
{
    if (check_ctx(c) != WDR_OK) return WDR_EINVAL;
    if (!mask) {
        set_error("null mask");
        return WDR_EINVAL;
    }
    for (int mu = 0; mu < 4; ++mu)
        if (lo < 0 || hi >= c->g.B[mu] || hi - lo < 2) {
            set_error("need 0 <= lo, hi - lo >= 2 and hi < B[mu]");
            return WDR_EINVAL;
        }
    WDR_HIP(hipSetDevice(c->device));
    launch_active_links(c->g, lo, hi, mask, S(stream));
    return finish(S(stream));
}

wdr_status wdr_interpolate(wdr_ctx *c, const double *U, const double *Up, int32_t i, int32_t N, double *out,
                           void *stream)
{
    wdr_status e = pre(c, U, out);
    if (e != WDR_OK) return e;
    if (!Up || N < 1 || i < 0 || i > N) {
        set_error("need 0 <= i <= N, N >= 1 and non-null fields");
        return WDR_EINVAL;
    }
    hipStream_t s = S(stream);
    const size_t n = (size_t)c->g.V * 36;
    if (i == 0 || i == N) {
        WDR_HIP(hipMemcpyAsync(out, i == 0 ? U : Up, n * sizeof(double2), hipMemcpyDeviceToDevice, s));
        return WDR_OK;
    }
    Work a(c, n * sizeof(double2)), b(c, n * sizeof(double2)), o(c, n * sizeof(double2));
    if (!a.ok() || !b.ok() || !o.ok()) return WDR_ENOMEM;
    // the path of canonical links does not depend on the boundary phases
    // (folding a sign in and out commutes with it; an open boundary would
    // zero the wrapping links), so none are applied here
    const int unit[4] = {1, 1, 1, 1};
    launch_pack_gauge<double>(c->g, unit, reinterpret_cast<const double2 *>(U), a.as<double2>(), s);
    launch_pack_gauge<double>(c->g, unit, reinterpret_cast<const double2 *>(Up), b.as<double2>(), s);
    launch_interpolate(c->g, a.as<double2>(), b.as<double2>(), (double)i / N, o.as<double2>(), s);
    launch_unpack_gauge(c->g, unit, o.as<double2>(), reinterpret_cast<double2 *>(out), s);
    return finish(s);
}

wdr_status wdr_noise(wdr_ctx *c, wdr_noise_kind kind, uint64_t seed, int32_t step, int32_t k, int32_t black_only,
                     double *out, void *stream)
{
    wdr_status e = pre(c, out, out);
    if (e != WDR_OK) return e;
    if (kind != WDR_NOISE_Z2 && kind != WDR_NOISE_GAUSS) {
        set_error("unknown noise kind");
        return WDR_EINVAL;
    }
    if (black_only && (e = check_blocks_usable(c, false)) != WDR_OK) return e;
    Work a(c, field_bytes(c, WDR_F64)), idx(c, 2 * sizeof(int32_t));
    if (!a.ok() || !idx.ok()) return WDR_ENOMEM;
    const int32_t sk[2] = {step, k};
    WDR_HIP(hipMemcpyAsync(idx.as<void>(), sk, sizeof(sk), hipMemcpyHostToDevice, S(stream)));
    launch_noise(c->g, all_sys(c, 1), kind, seed, nullptr, idx.as<int32_t>(), idx.as<int32_t>() + 1, black_only,
                 a.as<double2>(), S(stream));
    launch_unpack_spinor<double>(c->g, a.as<double2>(), reinterpret_cast<double2 *>(out), S(stream));
    return finish(S(stream));
}

int64_t wdr_field_bytes(const wdr_ctx *c, wdr_prec prec)
{
    if (!c || (prec != WDR_F64 && prec != WDR_F32 && prec != WDR_F16)) return 0;
    if (prec == WDR_F16) return (int64_t)f16_field_bytes(c);
    return (int64_t)field_bytes(c, prec);
}

int64_t wdr_halo_bytes(const wdr_ctx *c, wdr_prec prec)
{
    if (!c || (prec != WDR_F64 && prec != WDR_F32)) return 0;
    const int64_t F = (int64_t)c->g.L[0] * c->g.L[1] * c->g.L[2];
    return 6 * F * (prec == WDR_F64 ? 16 : 8);
}

// shared checks of the halo calls: an open t boundary and F64 / F32
static wdr_status halo_ok(wdr_ctx *c, const void *U, const void *a, const void *b, const void *f, wdr_prec prec)
{
    wdr_status e = pre(c, U, a);
    if (e != WDR_OK) return e;
    if (!b || !f) {
        set_error("null field pointer");
        return WDR_EINVAL;
    }
    if (c->g.bc[3] != 0) {
        set_error("the halo calls need a context whose t boundary is open (bc[3] = 0): the slab of one GPU");
        return WDR_EINVAL;
    }
    if (prec != WDR_F64 && prec != WDR_F32) {
        set_error("the halo calls take F64 or F32 fields");
        return WDR_EINVAL;
    }
    return WDR_OK;
}

wdr_status wdr_halo_pack(wdr_ctx *c, const double *U, wdr_prec prec, const void *in, void *send_lo, void *send_hi,
                         void *stream)
{
    wdr_status e = halo_ok(c, U, in, send_lo, send_hi, prec);
    if (e != WDR_OK) return e;
    const double2 *u = reinterpret_cast<const double2 *>(U);
    if (prec == WDR_F64)
        launch_halo_pack<double>(c->g, u, static_cast<const double2 *>(in), static_cast<double2 *>(send_lo),
                                 static_cast<double2 *>(send_hi), S(stream));
    else
        launch_halo_pack<float>(c->g, u, static_cast<const float2 *>(in), static_cast<float2 *>(send_lo),
                                static_cast<float2 *>(send_hi), S(stream));
    return finish(S(stream));
}

wdr_status wdr_halo_unpack(wdr_ctx *c, const double *U, double kappa, wdr_prec prec, const void *recv_lo,
                           const void *recv_hi, int32_t sign_lo, int32_t sign_hi, void *out, void *stream)
{
    wdr_status e = halo_ok(c, U, recv_lo, recv_hi, out, prec);
    if (e != WDR_OK) return e;
    if ((e = check_kappa(kappa)) != WDR_OK) return e;
    if ((sign_lo != 1 && sign_lo != -1) || (sign_hi != 1 && sign_hi != -1)) {
        set_error("the boundary signs must be 1 or -1");
        return WDR_EINVAL;
    }
    const double2 *u = reinterpret_cast<const double2 *>(U);
    if (prec == WDR_F64)
        launch_halo_unpack<double>(c->g, u, kappa, static_cast<const double2 *>(recv_lo),
                                   static_cast<const double2 *>(recv_hi), (double)sign_lo, (double)sign_hi,
                                   static_cast<double2 *>(out), S(stream));
    else
        launch_halo_unpack<float>(c->g, u, (float)kappa, static_cast<const float2 *>(recv_lo),
                                  static_cast<const float2 *>(recv_hi), (float)sign_lo, (float)sign_hi,
                                  static_cast<float2 *>(out), S(stream));
    return finish(S(stream));
}

wdr_status wdr_pack(wdr_ctx *c, wdr_prec prec, const double *canon, void *internal, void *stream)
{
    wdr_status e = pre(c, canon, internal);
    if (e != WDR_OK) return e;
    if (prec == WDR_F64)
        launch_pack_spinor<double>(c->g, reinterpret_cast<const double2 *>(canon), static_cast<double2 *>(internal),
                                   S(stream));
    else if (prec == WDR_F32)
        launch_pack_spinor<float>(c->g, reinterpret_cast<const double2 *>(canon), static_cast<float2 *>(internal),
                                  S(stream));
    else if (prec == WDR_F16) {
        Work t(c, field_bytes(c, WDR_F64));
        if (!t.ok()) return WDR_ENOMEM;
        launch_pack_spinor<double>(c->g, reinterpret_cast<const double2 *>(canon), t.as<double2>(), S(stream));
        launch_to_h16<double>(c->g, all_sys(c, 1), t.as<double2>(), f16_field(c, internal), 0, c->g.nblk, S(stream));
    } else {
        set_error("precision must be F64, F32 or F16");
        return WDR_EINVAL;
    }
    return finish(S(stream));
}

wdr_status wdr_unpack(wdr_ctx *c, wdr_prec prec, const void *internal, double *canon, void *stream)
{
    wdr_status e = pre(c, internal, canon);
    if (e != WDR_OK) return e;
    if (prec == WDR_F64)
        launch_unpack_spinor<double>(c->g, static_cast<const double2 *>(internal), reinterpret_cast<double2 *>(canon),
                                     S(stream));
    else if (prec == WDR_F32)
        launch_unpack_spinor<float>(c->g, static_cast<const float2 *>(internal), reinterpret_cast<double2 *>(canon),
                                    S(stream));
    else if (prec == WDR_F16) {
        Work t(c, field_bytes(c, WDR_F64));
        if (!t.ok()) return WDR_ENOMEM;
        const H16 f = f16_field(c, const_cast<void *>(internal));
        launch_from_h16(c->g, all_sys(c, 1), H16c{f.v, f.s}, t.as<double2>(), 0, 0, c->g.nblk, S(stream));
        launch_unpack_spinor<double>(c->g, t.as<double2>(), reinterpret_cast<double2 *>(canon), S(stream));
    } else {
        set_error("precision must be F64, F32 or F16");
        return WDR_EINVAL;
    }
    return finish(S(stream));
}

int64_t wdr_eo16_field_bytes(const wdr_ctx *c)
{
    if (!c || !e16_geometry(c->g)) return 0;
    return (int64_t)e16_field_bytes(c->g, 1);
}

wdr_status wdr_pack_eo16(wdr_ctx *c, int32_t parity, const double *canon, void *eo16, void *stream)
{
    wdr_status e = pre(c, canon, eo16);
    if (e != WDR_OK) return e;
    if (!e16_geometry(c->g) || (parity != 0 && parity != 1)) {
        set_error("FP16 half fields need 4^4 blocks in a 2-colourable checkerboard; parity 0 or 1");
        return WDR_EINVAL;
    }
    Work t(c, field_bytes(c, WDR_F64));
    if (!t.ok()) return WDR_ENOMEM;
    launch_pack_spinor<double>(c->g, reinterpret_cast<const double2 *>(canon), t.as<double2>(), S(stream));
    launch_e16_from64(c->g, 1, parity, t.as<double2>(), e16_field(c->g, 1, eo16), S(stream));
    return finish(S(stream));
}

wdr_status wdr_unpack_eo16(wdr_ctx *c, int32_t parity, const void *eo16, double *canon, void *stream)
{
    wdr_status e = pre(c, eo16, canon);
    if (e != WDR_OK) return e;
    if (!e16_geometry(c->g) || (parity != 0 && parity != 1)) {
        set_error("FP16 half fields need 4^4 blocks in a 2-colourable checkerboard; parity 0 or 1");
        return WDR_EINVAL;
    }
    Work t(c, field_bytes(c, WDR_F64));
    if (!t.ok()) return WDR_ENOMEM;
    launch_e16_to64(c->g, 1, parity, cref(e16_field(c->g, 1, const_cast<void *>(eo16))), t.as<double2>(), S(stream));
    launch_unpack_spinor<double>(c->g, t.as<double2>(), reinterpret_cast<double2 *>(canon), S(stream));
    return finish(S(stream));
}

wdr_status wdr_apply_hop_eo_internal(wdr_ctx *c, const wdr_gauge *U, double kappa, wdr_prec prec, int32_t parity,
                                     int32_t dag, int32_t nsys, const void *in, const void *diag, void *out,
                                     void *stream)
{
    wdr_status e = pre(c, in, out);
    if (e != WDR_OK) return e;
    if ((e = check_gauge(c, U)) != WDR_OK || (e = check_kappa(kappa)) != WDR_OK) return e;
    if ((parity != 0 && parity != 1) || (dag != 0 && dag != 1) || nsys < 1) {
        set_error("parity and dag must be 0 or 1, nsys >= 1");
        return WDR_EINVAL;
    }
    if (in == out || diag == out || diag == in) {
        set_error("in, diag and out must not alias");
        return WDR_EINVAL;
    }
    const Geo &g = c->g;
    GaugeTab tab = view(U);
    Sys sy = all_sys(c, nsys);
    if (prec == WDR_F16) {
        if (!e16_geometry(g) || !tab.e16.tab) {
            set_error("FP16 half fields need 4^4 blocks in a 2-colourable checkerboard and an SU(3) field");
            return WDR_EINVAL;
        }
        // one gauge pointer for every system of the launch (a table the handle keeps)
        const void *const *t = replicated(const_cast<wdr_gauge *>(U), 3, nsys, S(stream));
        if (!t) {
            set_error("gauge table allocation failed");
            return WDR_ENOMEM;
        }
        const Links16 L{reinterpret_cast<const h2 *const *>(t), nullptr};
        const E16c din = cref(e16_field(g, nsys, const_cast<void *>(in)));
        const E16c ddg = diag ? cref(e16_field(g, nsys, const_cast<void *>(diag))) : E16c{nullptr, nullptr};
        launch_eo16(g, sy, L, -1.f, -(float)kappa, parity, dag, din, ddg, e16_field(g, nsys, out), nullptr,
                    S(stream));
        return finish(S(stream));
    }
    if (prec != WDR_F64 && prec != WDR_F32) {
        set_error("precision must be F64, F32 or F16");
        return WDR_EINVAL;
    }
    const void *const *t = replicated(const_cast<wdr_gauge *>(U), prec == WDR_F64 ? 0 : 1, nsys, S(stream));
    if (!t) {
        set_error("gauge table allocation failed");
        return WDR_ENOMEM;
    }
    if (prec == WDR_F64)
        launch_dslash<double>(g, sy, Links<double>{reinterpret_cast<UTab<double>>(t), U->su3}, HOPS_ALL, parity,
                              dag, static_cast<const double2 *>(in), static_cast<const double2 *>(diag),
                              static_cast<double2 *>(out), kappa, 0, g.nblk, S(stream));
    else
        launch_dslash<float>(g, sy, Links<float>{reinterpret_cast<UTab<float>>(t), U->su3}, HOPS_ALL, parity, dag,
                             static_cast<const float2 *>(in), static_cast<const float2 *>(diag),
                             static_cast<float2 *>(out), (float)kappa, 0, g.nblk, S(stream));
    return finish(S(stream));
}

wdr_status wdr_apply_D_internal(wdr_ctx *c, const wdr_gauge *U, double kappa, wdr_prec prec, const void *in,
                                void *out, void *stream)
{
    wdr_status e = pre(c, in, out);
    if (e != WDR_OK) return e;
    if ((e = check_gauge(c, U, prec == WDR_F64 || prec == WDR_F32, kappa)) != WDR_OK ||
        (e = check_kappa(kappa)) != WDR_OK)
        return e;
    if (in == out) {
        set_error("in and out must not alias");
        return WDR_EINVAL;
    }
    const Geo &g = c->g;
    Sys one = all_sys(c, 1);
    if (prec == WDR_F64)
        launch_dslash<double>(g, one, links<double>(U), HOPS_ALL, -1, 0, static_cast<const double2 *>(in),
                              static_cast<const double2 *>(in), static_cast<double2 *>(out), kappa, 0, g.nblk,
                              S(stream));
    else if (prec == WDR_F32)
        launch_dslash<float>(g, one, links<float>(U), HOPS_ALL, -1, 0, static_cast<const float2 *>(in),
                             static_cast<const float2 *>(in), static_cast<float2 *>(out), (float)kappa, 0, g.nblk,
                             S(stream));
    else if (prec == WDR_F16) {
        const H16 a = f16_field(c, const_cast<void *>(in)), b = f16_field(c, out);
        if (!launch_dslash_h16(g, U->u16, H16c{a.v, a.s}, b, (float)kappa, S(stream))) {
            set_error("the FP16 stencil needs 4^4 blocks and an SU(3) gauge field");
            return WDR_EINVAL;
        }
    } else {
        set_error("precision must be F64, F32 or F16");
        return WDR_EINVAL;
    }
    return finish(S(stream));
}

wdr_status wdr_apply_D(wdr_ctx *c, const wdr_gauge *U, double kappa, wdr_prec prec, const double *in, double *out,
                       void *stream)
{
    return stencil_entry(c, U, kappa, prec, 0, 0, in, out, stream);
}

wdr_status wdr_apply_D_noalloc(wdr_ctx *c, const wdr_gauge *U, double kappa, wdr_prec prec, const double *in,
                               double *out, void *stream)
{
    wdr_status e = pre(c, in, out);
    if (e != WDR_OK) return e;
    if ((e = check_gauge(c, U, prec == WDR_F64 || prec == WDR_F32, kappa)) != WDR_OK ||
        (e = check_kappa(kappa)) != WDR_OK)
        return e;
    if (prec != WDR_F64 && prec != WDR_F32) {
        set_error("wdr_apply_D_noalloc computes in F64 or F32");
        return WDR_EINVAL;
    }
    const size_t fb = (field_bytes(c, prec) + 255) / 256 * 256;
    if (2 * fb > NOALLOC_BYTES) {
        set_error("wdr_apply_D_noalloc needs " + std::to_string(2 * fb) + " bytes of staging, more than its " +
                  std::to_string(NOALLOC_BYTES) + "-byte static array");
        return WDR_EINVAL;
    }
    void *base;
    {
        std::lock_guard<std::mutex> lock(scratch_mu);
        base = c->device >= 0 && c->device < MAX_DEVICES ? scratch_dev[c->device] : nullptr;
    }
    if (!base) {
        set_error("the staging array of this device was not set up");
        return WDR_ESTATE;
    }
    unsigned char *a = static_cast<unsigned char *>(base), *b = a + fb;
    const hipStream_t s = S(stream);
    const Geo &g = c->g;
    const Sys one = all_sys(c, 1);
    // the output field starts at zero (a kernel clears it, like the pooled
    // form); the input field is written in full by the pack
    if (prec == WDR_F64) {
        launch_pack_spinor<double>(g, reinterpret_cast<const double2 *>(in), reinterpret_cast<double2 *>(a), s);
        launch_zero<double>(reinterpret_cast<double2 *>(b), field_n(c), s);
        launch_dslash<double>(g, one, links<double>(U), HOPS_ALL, -1, 0, reinterpret_cast<const double2 *>(a),
                              reinterpret_cast<const double2 *>(a), reinterpret_cast<double2 *>(b), kappa, 0, g.nblk,
                              s);
        launch_unpack_spinor<double>(g, reinterpret_cast<const double2 *>(b), reinterpret_cast<double2 *>(out), s);
    } else {
        launch_pack_spinor<float>(g, reinterpret_cast<const double2 *>(in), reinterpret_cast<float2 *>(a), s);
        launch_zero<float>(reinterpret_cast<float2 *>(b), field_n(c), s);
        launch_dslash<float>(g, one, links<float>(U), HOPS_ALL, -1, 0, reinterpret_cast<const float2 *>(a),
                             reinterpret_cast<const float2 *>(a), reinterpret_cast<float2 *>(b), (float)kappa, 0,
                             g.nblk, s);
        launch_unpack_spinor<float>(g, reinterpret_cast<const float2 *>(b), reinterpret_cast<double2 *>(out), s);
    }
    return finish(s);
}

wdr_status wdr_apply_Dblock(wdr_ctx *c, const wdr_gauge *U, double kappa, wdr_prec prec, int32_t colour,
                            const double *in, double *out, void *stream)
{
    if (colour < 0 || colour > 2) {
        set_error("colour must be 0, 1 or 2");
        return WDR_EINVAL;
    }
    return stencil_entry(c, U, kappa, prec, 1, colour, in, out, stream);
}

wdr_status wdr_apply_Dhop(wdr_ctx *c, const wdr_gauge *U, double kappa, wdr_prec prec, int32_t from_colour,
                          const double *in, double *out, void *stream)
{
    if (from_colour < 0 || from_colour > 1) {
        set_error("from_colour must be 0 or 1");
        return WDR_EINVAL;
    }
    return stencil_entry(c, U, kappa, prec, 2, from_colour, in, out, stream);
}

wdr_status wdr_apply_Dee(wdr_ctx *c, const wdr_gauge *U, double kappa, wdr_prec prec, int32_t blocked,
                         const double *in, double *out, void *stream)
{
    return stencil_entry(c, U, kappa, prec, 3, blocked ? 1 : 0, in, out, stream);
}

wdr_status wdr_sap(wdr_ctx *c, const wdr_gauge *U, double kappa, const wdr_solver_params *sp, const double *in,
                   double *out, void *stream)
{
    wdr_status e = pre(c, in, out);
    if (e != WDR_OK) return e;
    if ((e = check_gauge(c, U, true, kappa)) != WDR_OK || (e = check_kappa(kappa)) != WDR_OK) return e;
    if (!sp) {
        set_error("null solver parameters");
        return WDR_EINVAL;
    }
    wdr_solver_params p = *sp;
    p.solver = WDR_SOLVER_FGCR_SAP;
    if ((e = check_params(c, p, true)) != WDR_OK) return e;
    wdr_status se = WDR_OK;
    e = with_fields<double>(c, in, out, S(stream), [&](double2 *a, double2 *b) {
        se = sap64(c, all_sys(c, 1), view(U), kappa, p, a, b, S(stream));
    });
    return e != WDR_OK ? e : se;
}

wdr_status wdr_solve(wdr_ctx *c, const wdr_gauge *U, double kappa, const wdr_solver_params *sp, const double *b,
                     double *x, wdr_solve_info *info, void *stream)
{
    wdr_status e = pre(c, b, x);
    if (e != WDR_OK) return e;
    if (!sp) {
        set_error("null solver parameters");
        return WDR_EINVAL;
    }
    if ((e = check_gauge(c, U, true, kappa)) != WDR_OK || (e = check_kappa(kappa)) != WDR_OK) return e;
    if ((e = check_params(c, *sp, false)) != WDR_OK) return e;
    const double t0 = now();
    std::vector<Stats> st;
    wdr_status se = WDR_OK;
    e = with_fields<double>(c, b, x, S(stream), [&](double2 *a, double2 *o) {
        se = solve64(c, 1, view(U), kappa, *sp, sp->tol, a, o, st, S(stream));
    });
    (void)hipStreamSynchronize(S(stream));
    fill_info(info, summarize(st), now() - t0);
    return e != WDR_OK ? e : se;
}

wdr_status wdr_block_solve(wdr_ctx *c, const wdr_gauge *U, double kappa, int32_t colour, const wdr_solver_params *sp,
                           const double *b, double *x, wdr_solve_info *info, void *stream)
{
    wdr_status e = pre(c, b, x);
    if (e != WDR_OK) return e;
    if ((e = check_gauge(c, U, sp != nullptr, kappa)) != WDR_OK || (e = check_kappa(kappa)) != WDR_OK) return e;
    if (!sp || colour < 0 || colour > 2) {
        set_error("null solver parameters or colour not in 0..2");
        return WDR_EINVAL;
    }
    if ((e = check_params(c, *sp, true)) != WDR_OK) return e;
    const double t0 = now();
    std::vector<Stats> st;
    wdr_status se = WDR_OK;
    e = with_fields<double>(c, b, x, S(stream), [&](double2 *a, double2 *o) {
        se = block_solve64(c, 1, view(U), kappa, colour, *sp, sp->block_tol, a, o, st, S(stream));
    });
    (void)hipStreamSynchronize(S(stream));
    fill_info(info, summarize(st), now() - t0);
    return e != WDR_OK ? e : se;
}

wdr_status wdr_apply_schur(wdr_ctx *c, const wdr_gauge *U, double kappa, const wdr_solver_params *sp,
                           const double *in, double *out, void *stream)
{
    wdr_status e = pre(c, in, out);
    if (e != WDR_OK) return e;
    if ((e = check_gauge(c, U, sp != nullptr, kappa)) != WDR_OK || (e = check_kappa(kappa)) != WDR_OK) return e;
    if (!sp) {
        set_error("null solver parameters");
        return WDR_EINVAL;
    }
    if ((e = check_params(c, *sp, true)) != WDR_OK) return e;
    std::vector<Stats> st;
    wdr_status se = WDR_OK;
    e = with_fields<double>(c, in, out, S(stream), [&](double2 *a, double2 *o) {
        // white sites of the input are ignored
        launch_keep_slots(c->g, all_sys(c, 1), a, 0, c->g.nblack, S(stream));
        se = schur64(c, 1, view(U), kappa, *sp, a, o, st, S(stream));
    });
    return e != WDR_OK ? e : se;
}

static wdr_status check_est(const wdr_ctx *c, const wdr_est_params *p)
{
    if (!p || p->n_steps < 1 || p->n_noise < 1 || p->max_batch < 0 ||
        (p->op != WDR_OP_FULL && p->op != WDR_OP_SCHUR && p->op != WDR_OP_BLOCKS && p->op != WDR_OP_DD) ||
        (p->noise != WDR_NOISE_Z2 && p->noise != WDR_NOISE_GAUSS)) {
        set_error("invalid estimator parameters");
        return WDR_EINVAL;
    }
    return check_params(c, p->sp, p->op != WDR_OP_FULL);
}

wdr_status wdr_logdet_ratio(wdr_ctx *c, const wdr_gauge *U, const wdr_gauge *Up, double kappa,
                            const wdr_est_params *p, double *samples, double *log_ratio, wdr_solve_info *info,
                            void *stream)
{
    if (check_ctx(c) != WDR_OK) return WDR_EINVAL;
    wdr_status e;
    if ((e = check_est(c, p)) != WDR_OK) return e;
    if ((e = check_gauge(c, U, true, kappa)) != WDR_OK ||
        (e = check_gauge(c, Up, true, kappa)) != WDR_OK || (e = check_pair(U, Up)) != WDR_OK)
        return e;
    if ((e = check_kappa(kappa)) != WDR_OK) return e;
    WDR_HIP(hipSetDevice(c->device));
    const double t0 = now();
    Stats st;
    e = logdet_ratio(c, {Proposal{U, Up, kappa, p->seed}}, *p, samples, log_ratio, st, S(stream));
    (void)hipStreamSynchronize(S(stream));
    fill_info(info, st, now() - t0);
    if (e == WDR_OK) e = finish(S(stream));
    return e;
}

wdr_status wdr_logdet_ratio_batch(int32_t n, const wdr_proposal *props, const wdr_est_params *p, double *samples,
                                  double *log_ratios, wdr_solve_info *info, void *stream)
{
    if (n < 1 || !props) {
        set_error("need at least one proposal");
        return WDR_EINVAL;
    }
    // group the proposals by context, keeping their order inside a group
    std::vector<wdr_ctx *> ctxs;
    std::vector<std::vector<int>> members;
    for (int j = 0; j < n; ++j) {
        wdr_ctx *c = props[j].ctx;
        if (check_ctx(c) != WDR_OK) return WDR_EINVAL;
        wdr_status e;
        if ((e = check_gauge(c, props[j].U, true, props[j].kappa)) != WDR_OK ||
            (e = check_gauge(c, props[j].Up, true, props[j].kappa)) != WDR_OK ||
            (e = check_pair(props[j].U, props[j].Up)) != WDR_OK || (e = check_kappa(props[j].kappa)) != WDR_OK)
            return e;
        const size_t gi = std::find(ctxs.begin(), ctxs.end(), c) - ctxs.begin();
        if (gi == ctxs.size()) {
            if ((e = check_est(c, p)) != WDR_OK) return e;
            if (!ctxs.empty() && c->device != ctxs[0]->device) {
                set_error("all proposals of a batch must be on one device");
                return WDR_EINVAL;
            }
            ctxs.push_back(c);
            members.emplace_back();
        }
        members[gi].push_back(j);
    }
    WDR_HIP(hipSetDevice(ctxs[0]->device));
    // output offsets of every proposal
    const int per = p->n_steps * p->n_noise;
    std::vector<size_t> off(n + 1, 0);
    for (int j = 0; j < n; ++j) {
        const int nblk = props[j].ctx->g.nblk;
        off[j + 1] = off[j] + (size_t)per * (p->op == WDR_OP_BLOCKS ? nblk : p->op == WDR_OP_DD ? nblk + 1 : 1);
    }
    const size_t G = ctxs.size();
    std::vector<std::vector<double>> gs(G), gl(G);
    std::vector<Stats> gst(G);
    std::vector<wdr_status> ge(G, WDR_OK);
    std::vector<std::string> gmsg(G);
    const double t0 = now();
    auto run = [&](size_t gi, hipStream_t s) {
        (void)hipSetDevice(ctxs[gi]->device);
        std::vector<Proposal> pr;
        size_t ns = 0;
        for (int j : members[gi]) {
            pr.push_back(Proposal{props[j].U, props[j].Up, props[j].kappa, props[j].seed});
            ns += off[j + 1] - off[j];
        }
        gs[gi].resize(ns);
        gl[gi].resize(pr.size());
        ge[gi] = logdet_ratio(ctxs[gi], pr, *p, gs[gi].data(), gl[gi].data(), gst[gi], s);
        (void)hipStreamSynchronize(s);
        if (ge[gi] != WDR_OK) gmsg[gi] = wdr_last_error();
    };
    // contexts with the persistent CG form run one after another: two
    // cooperative launches sized to the whole GPU must never wait on each
    // other's workgroups
    bool coop = false;
    for (wdr_ctx *c : ctxs) coop = coop || c->g.cg_form == WDR_CG_PERSISTENT;
    if (G == 1 || coop) {
        for (size_t gi = 0; gi < G; ++gi) run(gi, S(stream));
    } else {
        // fork: each context's stream starts after the work queued on `stream`
        hipEvent_t fork;
        WDR_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        WDR_HIP(hipEventRecord(fork, S(stream)));
        for (wdr_ctx *c : ctxs) {
            if (!c->aux && hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess) {
                (void)hipEventDestroy(fork);
                set_error("stream creation failed");
                return WDR_EDEVICE;
            }
            (void)hipStreamWaitEvent(c->aux, fork, 0);
        }
        std::vector<std::thread> th;
        for (size_t gi = 0; gi < G; ++gi) th.emplace_back(run, gi, ctxs[gi]->aux);
        for (auto &t : th) t.join();
        (void)hipEventDestroy(fork);
    }
    // scatter the results back to proposal order
    Stats tot;
    wdr_status e = WDR_OK;
    for (size_t gi = 0; gi < G; ++gi) {
        size_t pos = 0;
        for (size_t q = 0; q < members[gi].size(); ++q) {
            const int j = members[gi][q];
            const size_t len = off[j + 1] - off[j];
            if (samples) std::copy(gs[gi].begin() + pos, gs[gi].begin() + pos + len, samples + off[j]);
            if (log_ratios) log_ratios[j] = gl[gi][q];
            pos += len;
        }
        tot.iters = std::max(tot.iters, gst[gi].iters);
        tot.converged = tot.converged && gst[gi].converged;
        tot.rel = std::max(tot.rel, gst[gi].rel);
        tot.total += gst[gi].total;
        // a hard error outranks non-convergence
        if (ge[gi] != WDR_OK && (e == WDR_OK || e == WDR_ENOCONV)) {
            e = ge[gi];
            set_error(gmsg[gi]);
        }
    }
    fill_info(info, tot, now() - t0);
    return e;
}

wdr_status wdr_block_logdet(wdr_ctx *c, const wdr_gauge *U, double kappa, int32_t max_blocks, double *out,
                            void *stream)
{
    return wdr_block_logdet_ratio(c, U, nullptr, kappa, max_blocks, out, stream);
}

wdr_status wdr_block_logdet_ratio(wdr_ctx *c, const wdr_gauge *U, const wdr_gauge *Up, double kappa,
                                  int32_t max_blocks, double *out, void *stream)
{
    if (check_ctx(c) != WDR_OK) return WDR_EINVAL;
    wdr_status e;
    if ((e = check_gauge(c, U, true, kappa)) != WDR_OK ||
        (Up && ((e = check_gauge(c, Up, true, kappa)) != WDR_OK || (e = check_pair(U, Up)) != WDR_OK)))
        return e;
    if ((e = check_kappa(kappa)) != WDR_OK) return e;
    if (!out || max_blocks < 0) {
        set_error("null output pointer or negative max_blocks");
        return WDR_EINVAL;
    }
    if ((e = check_blocks_usable(c, true)) != WDR_OK) return e;
    WDR_HIP(hipSetDevice(c->device));
    const int nb = c->g.nblk;
    if (!Up) return block_logdet(c, U, nullptr, kappa, max_blocks, out, S(stream));
    std::vector<double> both(2 * (size_t)nb);
    e = block_logdet(c, U, Up, kappa, max_blocks, both.data(), S(stream));
    for (int b = 0; b < nb; ++b) out[b] = both[nb + b] - both[b];
    return e;
}

wdr_status wdr_block_fields(wdr_ctx *c, const wdr_gauge *U, double *out, void *stream)
{
    wdr_status e = pre(c, U, out);
    if (e != WDR_OK) return e;
    if ((e = check_gauge(c, U, true, U->ckappa)) != WDR_OK) return e;
    launch_block_fields(c->g, c->geom.bc, U->u64, reinterpret_cast<double2 *>(out), S(stream));
    return finish(S(stream));
}

wdr_status wdr_clover_field(wdr_ctx *c, const wdr_gauge *U, int32_t inverse, double *out, void *stream)
{
    wdr_status e = pre(c, U, out);
    if (e != WDR_OK) return e;
    if ((e = check_gauge(c, U, true, U->ckappa)) != WDR_OK) return e;
    if (!U->c64 || (inverse != 0 && inverse != 1)) {
        set_error(U->c64 ? "inverse must be 0 or 1" : "the gauge field carries no clover term");
        return WDR_EINVAL;
    }
    launch_clover_canon(c->g, U->c64, inverse, reinterpret_cast<double2 *>(out), S(stream));
    return finish(S(stream));
}

wdr_status wdr_block_schur_ratio(wdr_ctx *c, const wdr_gauge *U, const wdr_gauge *Up, double kappa, wdr_ctx *sub,
                                 const wdr_est_params *p, double *samples, double *log_ratios, wdr_solve_info *info,
                                 void *stream)
{
    if (check_ctx(c) != WDR_OK || check_ctx(sub) != WDR_OK) return WDR_EINVAL;
    wdr_status e;
    if ((U && U->c64) || (Up && Up->c64)) {
        // the leaves at a block's face reach outside the block, which a
        // lattice of the block's extents with open boundaries does not hold
        set_error("the block Schur ratio does not support the clover term");
        return WDR_EINVAL;
    }
    if ((e = check_gauge(c, U)) != WDR_OK || (e = check_gauge(c, Up)) != WDR_OK) return e;
    if ((e = check_kappa(kappa)) != WDR_OK) return e;
    for (int mu = 0; mu < 4; ++mu)
        if (sub->geom.L[mu] != c->geom.B[mu] || sub->geom.bc[mu] != 0) {
            set_error("sub must have the block extents of ctx as its lattice and open boundaries");
            return WDR_EINVAL;
        }
    if (sub->device != c->device) {
        set_error("sub must live on the device of ctx");
        return WDR_EINVAL;
    }
    if (!p || p->op != WDR_OP_SCHUR) {
        set_error("the block Schur ratio needs op WDR_OP_SCHUR");
        return WDR_EINVAL;
    }
    if ((e = check_est(sub, p)) != WDR_OK) return e;
    WDR_HIP(hipSetDevice(c->device));
    hipStream_t s = S(stream);
    const double t0 = now();
    const int nb = c->g.nblk;
    const size_t per = (size_t)c->g.Vb * 36;
    Work fw(c, 2 * nb * per * sizeof(double2));
    if (!fw.ok()) return WDR_ENOMEM;
    double2 *f0 = fw.as<double2>(), *f1 = f0 + nb * per;
    launch_block_fields(c->g, c->geom.bc, U->u64, f0, s);
    launch_block_fields(c->g, c->geom.bc, Up->u64, f1, s);
    // one proposal per block on `sub`
    std::vector<wdr_gauge *> hs;
    auto release = [&] {
        for (wdr_gauge *h : hs) (void)wdr_gauge_destroy(h);
    };
    std::vector<Proposal> props;
    for (int b = 0; b < nb && e == WDR_OK; ++b) {
        wdr_gauge *hu = nullptr, *hp = nullptr;
        e = wdr_gauge_create(sub, reinterpret_cast<const double *>(f0 + b * per), &hu, stream);
        if (hu) hs.push_back(hu);
        if (e == WDR_OK) e = wdr_gauge_create(sub, reinterpret_cast<const double *>(f1 + b * per), &hp, stream);
        if (hp) hs.push_back(hp);
        if (e == WDR_OK) props.push_back(Proposal{hu, hp, kappa, p->seed + (uint64_t)b});
    }
    if (e != WDR_OK) {
        release();
        return e;
    }
    Stats st;
    e = logdet_ratio(sub, props, *p, samples, log_ratios, st, s);
    (void)hipStreamSynchronize(s);
    fill_info(info, st, now() - t0);
    release();
    if (e == WDR_OK) e = finish(s);
    return e;
}

wdr_status wdr_heatbath(wdr_ctx *c, double beta, const uint8_t *mask, uint64_t seed, int32_t sweep, double *U,
                        void *stream)
{
    wdr_status e = pre(c, mask, U);
    if (e != WDR_OK) return e;
    if (!(beta > 0) || !std::isfinite(beta) || sweep < 0) {
        set_error("need beta > 0 and sweep >= 0");
        return WDR_EINVAL;
    }
    launch_heatbath(c, beta, mask, seed, sweep, reinterpret_cast<double2 *>(U), S(stream));
    return finish(S(stream));
}

wdr_status wdr_relative_gauge(wdr_ctx *c, const double *U, double *Up, int32_t sweeps, double *F, void *stream)
{
    wdr_status e = pre(c, U, Up);
    if (e != WDR_OK) return e;
    if (sweeps < 0) {
        set_error("sweeps must be >= 0");
        return WDR_EINVAL;
    }
    hipStream_t s = S(stream);
    launch_relgauge(c, reinterpret_cast<const double2 *>(U), reinterpret_cast<double2 *>(Up), sweeps, s);
    if (F) {
        // F = sum Re tr(U' U^+) / 3 = Re <U, U'> / 3 over all 36 V entries,
        // reduced as three fields of 12 V entries
        Work part(c, sizeof(double) * red_scratch(3)), out(c, 3 * sizeof(double2));
        if (!part.ok() || !out.ok()) return WDR_ENOMEM;
        launch_dot<double>(all_sys(c, 3), reinterpret_cast<const double2 *>(U), reinterpret_cast<const double2 *>(Up),
                           part.as<double>(), out.as<double2>(), 1, s);
        double2 h[3];
        WDR_HIP(hipMemcpyAsync(h, out.as<void>(), sizeof(h), hipMemcpyDeviceToHost, s));
        WDR_HIP(hipStreamSynchronize(s));
        *F = (h[0].x + h[1].x + h[2].x) / 3.0;
    }
    return finish(s);
}

wdr_status wdr_overrelax(wdr_ctx *c, const uint8_t *mask, double *U, void *stream)
{
    wdr_status e = pre(c, mask, U);
    if (e != WDR_OK) return e;
    launch_overrelax(c, mask, reinterpret_cast<double2 *>(U), S(stream));
    return finish(S(stream));
}

wdr_status wdr_filter_step(wdr_ctx *c, double beta, double kappa, const uint8_t *mask, int32_t n_block_steps,
                           const wdr_est_params *p, uint64_t seed, double *U, uint8_t *accepts,
                           wdr_filter_info *info, void *stream)
{
    wdr_status e = pre(c, mask, U);
    if (e != WDR_OK) return e;
    if ((e = check_kappa(kappa)) != WDR_OK) return e;
    if (!(beta > 0) || !std::isfinite(beta) || n_block_steps < 0 || !info) {
        set_error("need beta > 0, n_block_steps >= 0 and an info pointer");
        return WDR_EINVAL;
    }
    if (p && p->op != WDR_OP_SCHUR) {
        set_error("the global step needs op WDR_OP_SCHUR");
        return WDR_EINVAL;
    }
    if (p && (e = check_est(c, p)) != WDR_OK) return e;
    if ((e = check_blocks_usable(c, true)) != WDR_OK) return e;
    // every masked link must have both ends in one block
    const Geo &g = c->g;
    std::vector<uint8_t> hm((size_t)g.V * 4);
    WDR_HIP(hipMemcpyAsync(hm.data(), mask, hm.size(), hipMemcpyDeviceToHost, S(stream)));
    WDR_HIP(hipStreamSynchronize(S(stream)));
    for (long s = 0; s < g.V; ++s) {
        long r = s;
        for (int mu = 0; mu < 4; ++mu) {
            const int x = (int)(r % g.L[mu]);
            r /= g.L[mu];
            if (hm[s * 4 + mu] && x % g.B[mu] == g.B[mu] - 1) {
                set_error("the mask holds a link that leaves its block");
                return WDR_EINVAL;
            }
        }
    }
    e = filter_step(c, beta, kappa, mask, n_block_steps, p, seed, reinterpret_cast<double2 *>(U), accepts, *info,
                    S(stream));
    if (e == WDR_OK) e = finish(S(stream));
    return e;
}

}  // extern "C"
