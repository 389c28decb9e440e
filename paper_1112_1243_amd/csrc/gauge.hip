// Gauge update and the hierarchical filter (paper Sec. 2 hierarchical
// acceptance steps; Sec. 3 eq. 4step with one level; Sec. 5: heat-bath of
// the active links with the Wilson plaquette action, block acceptance with
// the exact block determinants, global acceptance with the stochastic
// Schur-complement estimate).
//
// The heat-bath works on the canonical field [site][mu][3][3]: one launch per
// direction mu and site parity (links of one such class share no plaquette),
// one thread per link.  Each link takes the Cabibbo-Marinari steps over the
// SU(2) subgroups (0,1), (0,2), (1,2) (Phys. Lett. B 119 (1982) 387): with
// W = U A (A the staple sum), the subgroup part of W is k v, v in SU(2);
// Y in SU(2) with density exp(2 beta k y0 / 3) is drawn by Kennedy and
// Pendleton's method (Phys. Lett. B 156 (1985) 393) for y0 and an isotropic
// direction, and U <- X U with X = Y v^+ on the subgroup's rows.
#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "philox.h"
#include "runtime.h"

namespace wdr {
namespace {

constexpr int HB_TAG = 5, ACC_TAG = 6, HB_TRIALS = 64;

struct Z {
    double re, im;
};
__device__ __forceinline__ Z zadd(Z a, Z b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ Z zmul(Z a, Z b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ Z zcj(Z a) { return {a.re, -a.im}; }

struct M {
    Z a[3][3];
};

__device__ __forceinline__ void load(const double2 *U, long site, int mu, M &m)
{
    const double2 *p = U + (site * 4 + mu) * 9;
    for (int e = 0; e < 9; ++e) m.a[e / 3][e % 3] = {p[e].x, p[e].y};
}
// C = A B, A B^+, A^+ B^+ ... by flags: da / db take the adjoint
__device__ __forceinline__ M mm(const M &A, bool da, const M &B, bool db)
{
    M C;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            Z s = {0.0, 0.0};
            for (int k = 0; k < 3; ++k) {
                const Z x = da ? zcj(A.a[k][i]) : A.a[i][k];
                const Z y = db ? zcj(B.a[j][k]) : B.a[k][j];
                s = zadd(s, zmul(x, y));
            }
            C.a[i][j] = s;
        }
    return C;
}

__device__ __forceinline__ long site_of(int4 L, const int x[4])
{
    return x[0] + (long)L.x * (x[1] + (long)L.y * (x[2] + (long)L.z * x[3]));
}

// canonical site s of the class (mu, par) and the staple sum A of its link,
// Re tr(U_mu(x) A) = the six plaquettes through the link; false when the
// link is not masked or has the other parity
__device__ __forceinline__ bool link_and_staple(int4 L, long V, const uint8_t *__restrict__ mask, int mu, int par,
                                                const double2 *U, long &s, M &A)
{
    s = (long)blockIdx.x * 256 + threadIdx.x;
    if (s >= V || !mask[s * 4 + mu]) return false;
    const int Ls[4] = {L.x, L.y, L.z, L.w};
    int x[4];
    long r = s;
    for (int d = 0; d < 4; ++d) {
        x[d] = (int)(r % Ls[d]);
        r /= Ls[d];
    }
    if (((x[0] + x[1] + x[2] + x[3]) & 1) != par) return false;
    auto nb = [&](const int *y, int d, int step) {
        int z[4] = {y[0], y[1], y[2], y[3]};
        z[d] = (z[d] + step + Ls[d]) % Ls[d];
        return site_of(L, z);
    };
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A.a[i][j] = {0.0, 0.0};
    const long xm = nb(x, mu, 1);
    int xmu[4] = {x[0], x[1], x[2], x[3]};
    xmu[mu] = (xmu[mu] + 1) % Ls[mu];
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        const long xn = nb(x, nu, 1), xd = nb(x, nu, -1), xmd = nb(xmu, nu, -1);
        M a, b, c;
        load(U, xm, nu, a);
        load(U, xn, mu, b);
        load(U, s, nu, c);
        const M up = mm(mm(a, false, b, true), false, c, true);
        load(U, xmd, nu, a);
        load(U, xd, mu, b);
        load(U, xd, nu, c);
        const M dn = mm(mm(a, true, b, true), false, c, false);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) A.a[i][j] = zadd(A.a[i][j], zadd(up.a[i][j], dn.a[i][j]));
    }
    return true;
}

// SU(2) subgroup (i, j) of W = u A: its part k v, v = [[a, b], [-b*, a*]] / k
__device__ __forceinline__ double subgroup_part(const M &u, const M &A, int i, int j, Z &a, Z &b)
{
    Z w[2][2];
    const int ij[2] = {i, j};
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q) {
            Z t = {0.0, 0.0};
            for (int k = 0; k < 3; ++k) t = zadd(t, zmul(u.a[ij[p]][k], A.a[k][ij[q]]));
            w[p][q] = t;
        }
    a = {0.5 * (w[0][0].re + w[1][1].re), 0.5 * (w[0][0].im - w[1][1].im)};
    b = {0.5 * (w[0][1].re - w[1][0].re), 0.5 * (w[0][1].im + w[1][0].im)};
    return sqrt(a.re * a.re + a.im * a.im + b.re * b.re + b.im * b.im);
}

// u <- X u on rows i, j
__device__ __forceinline__ void left_mul(M &u, const Z X[2][2], int i, int j)
{
    for (int col = 0; col < 3; ++col) {
        const Z ri = u.a[i][col], rj = u.a[j][col];
        u.a[i][col] = zadd(zmul(X[0][0], ri), zmul(X[0][1], rj));
        u.a[j][col] = zadd(zmul(X[1][0], ri), zmul(X[1][1], rj));
    }
}

__device__ __forceinline__ void store(double2 *U, long site, int mu, const M &u)
{
    double2 *p = U + (site * 4 + mu) * 9;
    for (int e = 0; e < 9; ++e) p[e] = make_double2(u.a[e / 3][e % 3].re, u.a[e / 3][e % 3].im);
}

// one heat-bath step of every masked link (x, mu) with x of parity par
__global__ __launch_bounds__(256) void k_heatbath(int4 L, long V, const uint8_t *__restrict__ mask, double beta,
                                                  uint64_t seed, uint64_t sweep, int mu, int par, double2 *U)
{
    long s;
    M A;
    if (!link_and_staple(L, V, mask, mu, par, U, s, A)) return;
    M u;
    load(U, s, mu, u);
    const int sub[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int g = 0; g < 3; ++g) {
        const int i = sub[g][0], j = sub[g][1];
        Z a, b;
        const double k = subgroup_part(u, A, i, j, a, b);
        const double alpha = 2.0 * beta * k / 3.0;
        const uint64_t c1 = (sweep << 32) | ((uint64_t)mu << 8) | (uint64_t)g;
        double a0 = 0.0;
        int t = 0;
        bool ok = false;
        for (; t < HB_TRIALS; ++t) {
            uint64_t c[4] = {(uint64_t)s, c1, (uint64_t)t, 0};
            philox4x64_10(c, seed, HB_TAG);
            const double u0 = uniform53(c[0]), u1 = uniform53(c[1]), u2 = uniform53(c[2]), u3 = uniform53(c[3]);
            const double cs = cos(2.0 * M_PI * u1);
            const double X = -(log(u0) + cs * cs * log(u2)) / alpha;
            if (u3 * u3 <= 1.0 - 0.5 * X) {
                a0 = 1.0 - X;
                ok = true;
                break;
            }
        }
        if (!ok) continue;
        uint64_t c[4] = {(uint64_t)s, c1, (uint64_t)t, 1};
        philox4x64_10(c, seed, HB_TAG);
        const double ct = 2.0 * uniform53(c[0]) - 1.0, phi = 2.0 * M_PI * uniform53(c[1]);
        const double rr = sqrt(fmax(0.0, 1.0 - a0 * a0)), st = sqrt(fmax(0.0, 1.0 - ct * ct));
        const double y1 = rr * st * cos(phi), y2 = rr * st * sin(phi), y3 = rr * ct;
        // Y = [[a0 + i y3, y2 + i y1], [-y2 + i y1, a0 - i y3]], v = [[a, b], [-b*, a*]] / k
        const Z Y[2][2] = {{{a0, y3}, {y2, y1}}, {{-y2, y1}, {a0, -y3}}};
        const double ik = 1.0 / k;
        const Z v[2][2] = {{{a.re * ik, a.im * ik}, {b.re * ik, b.im * ik}},
                           {{-b.re * ik, b.im * ik}, {a.re * ik, -a.im * ik}}};
        Z X[2][2];
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) X[p][q] = zadd(zmul(Y[p][0], zcj(v[q][0])), zmul(Y[p][1], zcj(v[q][1])));
        left_mul(u, X, i, j);
    }
    store(U, s, mu, u);
}

// over-relaxation of every masked link (x, mu) with x of parity par: per
// subgroup u <- (v^+)^2 u, the reflection through the maximum of Re tr(X W),
// which keeps the action
__global__ __launch_bounds__(256) void k_overrelax(int4 L, long V, const uint8_t *__restrict__ mask, int mu, int par,
                                                   double2 *U)
{
    long s;
    M A;
    if (!link_and_staple(L, V, mask, mu, par, U, s, A)) return;
    M u;
    load(U, s, mu, u);
    const int sub[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int g = 0; g < 3; ++g) {
        const int i = sub[g][0], j = sub[g][1];
        Z a, b;
        const double k = subgroup_part(u, A, i, j, a, b);
        if (!(k > 0.0)) continue;
        const double ik = 1.0 / k;
        // v^+ = [[a*, -b], [b*, a]] / k
        const Z vd[2][2] = {{{a.re * ik, -a.im * ik}, {-b.re * ik, -b.im * ik}},
                            {{b.re * ik, -b.im * ik}, {a.re * ik, a.im * ik}}};
        Z X[2][2];
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) X[p][q] = zadd(zmul(vd[p][0], vd[0][q]), zmul(vd[p][1], vd[1][q]));
        left_mul(u, X, i, j);
    }
    store(U, s, mu, u);
}

// one relaxation step of the relative gauge fixing of Up to U at every site
// of parity par: h maximises Re tr(h K), K = sum_mu [Up_mu(x) U_mu(x)^+ +
// Up_mu(x-mu)^+ U_mu(x-mu)], by one pass over the SU(2) subgroups from the
// identity; then Up_mu(x) <- h Up_mu(x), Up_mu(x-mu) <- Up_mu(x-mu) h^+
// (links into x have their other end on the other parity, so no two
// threads touch one link)
__global__ __launch_bounds__(256) void k_relgauge(int4 L, long V, int par, const double2 *__restrict__ U, double2 *Up)
{
    const long s = (long)blockIdx.x * 256 + threadIdx.x;
    if (s >= V) return;
    const int Ls[4] = {L.x, L.y, L.z, L.w};
    int x[4];
    long r = s;
    for (int d = 0; d < 4; ++d) {
        x[d] = (int)(r % Ls[d]);
        r /= Ls[d];
    }
    if (((x[0] + x[1] + x[2] + x[3]) & 1) != par) return;
    long back[4];
    for (int mu = 0; mu < 4; ++mu) {
        int z[4] = {x[0], x[1], x[2], x[3]};
        z[mu] = (z[mu] - 1 + Ls[mu]) % Ls[mu];
        back[mu] = site_of(L, z);
    }
    M K;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) K.a[i][j] = {0.0, 0.0};
    for (int mu = 0; mu < 4; ++mu) {
        M a, b;
        load(Up, s, mu, a);
        load(U, s, mu, b);
        const M f = mm(a, false, b, true);
        load(Up, back[mu], mu, a);
        load(U, back[mu], mu, b);
        const M g = mm(a, true, b, false);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) K.a[i][j] = zadd(K.a[i][j], zadd(f.a[i][j], g.a[i][j]));
    }
    M h;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) h.a[i][j] = {i == j ? 1.0 : 0.0, 0.0};
    const int sub[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int g = 0; g < 3; ++g) {
        const int i = sub[g][0], j = sub[g][1];
        Z a, b;
        const double k = subgroup_part(h, K, i, j, a, b);
        if (!(k > 0.0)) continue;
        const double ik = 1.0 / k;
        const Z vd[2][2] = {{{a.re * ik, -a.im * ik}, {-b.re * ik, -b.im * ik}},
                            {{b.re * ik, -b.im * ik}, {a.re * ik, a.im * ik}}};
        left_mul(h, vd, i, j);
    }
    for (int mu = 0; mu < 4; ++mu) {
        M a;
        load(Up, s, mu, a);
        store(Up, s, mu, mm(h, false, a, false));
        load(Up, back[mu], mu, a);
        store(Up, back[mu], mu, mm(a, false, h, true));
    }
}

// cur <- prop at every site whose block was accepted
__global__ __launch_bounds__(256) void k_merge_blocks(int4 L, int4 B, long V, const int32_t *__restrict__ acc,
                                                      const double2 *__restrict__ prop, double2 *__restrict__ cur)
{
    const long s = (long)blockIdx.x * 256 + threadIdx.x;
    if (s >= V) return;
    const int Ls[4] = {L.x, L.y, L.z, L.w}, Bs[4] = {B.x, B.y, B.z, B.w};
    long r = s, b = 0, stride = 1;
    for (int d = 0; d < 4; ++d) {
        const int x = (int)(r % Ls[d]);
        r /= Ls[d];
        b += (x / Bs[d]) * stride;
        stride *= Ls[d] / Bs[d];
    }
    if (!acc[b]) return;
    for (int e = 0; e < 36; ++e) cur[s * 36 + e] = prop[s * 36 + e];
}

// the links of every block as a canonical field of the block's extents:
// out[b][site][mu][9], site lexicographic in the block, boundary phases
// taken out again (an open boundary leaves the wrapping links zero)
__global__ __launch_bounds__(256) void k_block_fields(Geo g, int4 bc, const double2 *__restrict__ in,
                                                      double2 *__restrict__ out)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const int slot = blockIdx.y, blk = g.slot_blk[slot];
    const uint32_t lc = g.loc_coord[l];
    const int loc[4] = {(int)(lc & 255), (int)((lc >> 8) & 255), (int)((lc >> 16) & 255), (int)(lc >> 24)};
    int x[4], r = blk;
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (r % g.NB[mu]) * g.B[mu] + loc[mu];
        r /= g.NB[mu];
    }
    const long site = loc[0] + (long)g.B[0] * (loc[1] + (long)g.B[1] * (loc[2] + (long)g.B[2] * loc[3]));
    double2 *o = out + ((long)blk * g.Vb + site) * 36;
    const int bcv[4] = {bc.x, bc.y, bc.z, bc.w};
    for (int mu = 0; mu < 4; ++mu) {
        const double f = (x[mu] == g.L[mu] - 1) ? (double)bcv[mu] : 1.0;
        const long base = ((long)slot * 4 + mu) * 9 * g.Vb + l;
        for (int e = 0; e < 9; ++e) {
            const double2 v = in[base + (long)e * g.Vb];
            o[mu * 9 + e] = make_double2(f * v.x, f * v.y);
        }
    }
}

int4 i4(const int v[4]) { return make_int4(v[0], v[1], v[2], v[3]); }

}  // namespace

void launch_block_fields(const Geo &g, const int bc[4], const double2 *in, double2 *out, hipStream_t s)
{
    k_block_fields<<<dim3((g.Vb + 255) / 256, g.nblk), 256, 0, s>>>(g, make_int4(bc[0], bc[1], bc[2], bc[3]), in,
                                                                    out);
}

void launch_heatbath(const wdr_ctx *c, double beta, const uint8_t *mask, uint64_t seed, int sweep, double2 *U,
                     hipStream_t s)
{
    const long V = c->g.V;
    for (int mu = 0; mu < 4; ++mu)
        for (int par = 0; par < 2; ++par)
            k_heatbath<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(i4(c->geom.L), V, mask, beta, seed,
                                                                    (uint64_t)(uint32_t)sweep, mu, par, U);
}

void launch_relgauge(const wdr_ctx *c, const double2 *U, double2 *Up, int sweeps, hipStream_t s)
{
    const long V = c->g.V;
    for (int sw = 0; sw < sweeps; ++sw)
        for (int par = 0; par < 2; ++par)
            k_relgauge<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(i4(c->geom.L), V, par, U, Up);
}

void launch_overrelax(const wdr_ctx *c, const uint8_t *mask, double2 *U, hipStream_t s)
{
    const long V = c->g.V;
    for (int mu = 0; mu < 4; ++mu)
        for (int par = 0; par < 2; ++par)
            k_overrelax<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(i4(c->geom.L), V, mask, mu, par, U);
}

bool accept_metropolis(double r, uint64_t seed, uint64_t c0, uint64_t c1, uint64_t c2)
{
    uint64_t c[4] = {c0, c1, c2, 0};
    philox4x64_10(c, seed, ACC_TAG);
    return r >= 0.0 || uniform53(c[0]) < std::exp(r);
}

wdr_status filter_step(wdr_ctx *c, double beta, double kappa, const uint8_t *mask, int n_block_steps,
                       const wdr_est_params *p, uint64_t seed, double2 *U, uint8_t *accepts, wdr_filter_info &info,
                       hipStream_t s)
{
    const Geo &g = c->g;
    const long V = g.V;
    const int nb = g.nblk;
    Work u0w(c, V * 36 * sizeof(double2)), pw(c, V * 36 * sizeof(double2)), aw(c, nb * sizeof(int32_t));
    if (!u0w.ok() || !pw.ok() || !aw.ok()) return WDR_ENOMEM;
    double2 *u0 = u0w.as<double2>(), *prop = pw.as<double2>();
    WDR_HIP(hipMemcpyAsync(u0, U, V * 36 * sizeof(double2), hipMemcpyDeviceToDevice, s));
    auto gauge = [&](const double2 *f, std::unique_ptr<wdr_gauge, wdr_status (*)(wdr_gauge *)> &h) {
        wdr_gauge *raw = nullptr;
        const wdr_status e = wdr_gauge_create(c, reinterpret_cast<const double *>(f), &raw, s);
        h.reset(raw);
        return e;
    };
    std::unique_ptr<wdr_gauge, wdr_status (*)(wdr_gauge *)> hc(nullptr, wdr_gauge_destroy), hp(nullptr, wdr_gauge_destroy);
    std::vector<double> ld_cur(nb), ld_prop(nb);
    std::vector<int32_t> acc(nb);
    wdr_status e = WDR_OK;
    info = wdr_filter_info{};
    if (n_block_steps > 0) {
        if ((e = gauge(U, hc)) != WDR_OK) return e;
        if ((e = block_logdet(c, hc.get(), nullptr, kappa, 0, ld_cur.data(), s)) != WDR_OK) return e;
        hc.reset();
    }
    for (int st = 0; st < n_block_steps; ++st) {
        // step 0: heat-bath proposal; step 1: block-wise exact acceptance
        WDR_HIP(hipMemcpyAsync(prop, U, V * 36 * sizeof(double2), hipMemcpyDeviceToDevice, s));
        launch_heatbath(c, beta, mask, seed, st, prop, s);
        if ((e = gauge(prop, hp)) != WDR_OK) return e;
        if ((e = block_logdet(c, hp.get(), nullptr, kappa, 0, ld_prop.data(), s)) != WDR_OK) return e;
        hp.reset();
        for (int b = 0; b < nb; ++b) {
            const bool a = accept_metropolis(ld_prop[b] - ld_cur[b], seed, (uint64_t)b, (uint64_t)st, 0);
            acc[b] = a;
            if (a) ld_cur[b] = ld_prop[b];
            if (accepts) accepts[(size_t)st * nb + b] = a;
            info.block_accepts += a;
        }
        info.block_trials += nb;
        WDR_HIP(hipMemcpyAsync(aw.as<void>(), acc.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice, s));
        k_merge_blocks<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(i4(c->geom.L), i4(c->geom.B), V, aw.as<int32_t>(),
                                                                    prop, U);
        WDR_HIP(hipStreamSynchronize(s));  // acc is host memory reused next step
    }
    if (!p) {  // block steps only: keep their result
        info.accepted = 1;
        WDR_HIP(hipStreamSynchronize(s));
        return WDR_OK;
    }
    // global step with the stochastic Schur-complement ratio
    if ((e = gauge(u0, hc)) != WDR_OK) return e;
    if ((e = gauge(U, hp)) != WDR_OK) return e;
    Stats est;
    double lr = 0.0;
    e = logdet_ratio(c, {Proposal{hc.get(), hp.get(), kappa, p->seed}}, *p, nullptr, &lr, est, s);
    if (e != WDR_OK) return e;
    info.log_ratio = lr;
    info.accepted = accept_metropolis(lr, seed, 0, 0, 1);
    if (!info.accepted) WDR_HIP(hipMemcpyAsync(U, u0, V * 36 * sizeof(double2), hipMemcpyDeviceToDevice, s));
    WDR_HIP(hipStreamSynchronize(s));
    return WDR_OK;
}

}  // namespace wdr
