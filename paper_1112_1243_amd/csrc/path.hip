// Path U_0 = U ... U_N = U' of eq. param (paper Sec. 4): the geodesic
//     U_t = exp(t log W) U,   W = U' U^+,   t = i / N,
// link by link in FP64.  The paper only asks ||U_i - U_{i+1}|| ~ 1/N; the
// geodesic with the traceless branch of log W keeps every U_t in SU(3).
//
// Eigen-decomposition of the unitary W: rotate it by a phase e^{-i phi}
// chosen so that -1 is far from its spectrum, map it to the Hermitian
// K = i (1 - W')(1 + W')^-1 (Cayley transform, eigenvalues tan(theta'/2)),
// diagonalise K by cyclic complex Jacobi rotations (orthonormal
// eigenvectors to rounding even for close eigenvalues), and read the
// angles back as theta = 2 atan(kappa) + phi, wrapped to (-pi, pi].
#include "stencil.h"

namespace wdr {
namespace {

using namespace dev;
typedef cx<double> zc;

struct M3 {
    zc a[3][3];
};

__device__ __forceinline__ zc cj(zc z) { return {z.re, -z.im}; }
__device__ __forceinline__ double abs2(zc z) { return z.re * z.re + z.im * z.im; }

__device__ M3 mmul(const M3 &A, const M3 &B)
{
    M3 C;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C.a[i][j] = A.a[i][0] * B.a[0][j] + A.a[i][1] * B.a[1][j] + A.a[i][2] * B.a[2][j];
    return C;
}

__device__ zc det3(const M3 &A)
{
    return A.a[0][0] * (A.a[1][1] * A.a[2][2] - A.a[1][2] * A.a[2][1]) -
           A.a[0][1] * (A.a[1][0] * A.a[2][2] - A.a[1][2] * A.a[2][0]) +
           A.a[0][2] * (A.a[1][0] * A.a[2][1] - A.a[1][1] * A.a[2][0]);
}

__device__ zc cdiv(zc a, zc b)
{
    const double d = abs2(b);
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

__device__ M3 inv3(const M3 &A)
{
    M3 C;  // adjugate / det
    C.a[0][0] = A.a[1][1] * A.a[2][2] - A.a[1][2] * A.a[2][1];
    C.a[0][1] = A.a[0][2] * A.a[2][1] - A.a[0][1] * A.a[2][2];
    C.a[0][2] = A.a[0][1] * A.a[1][2] - A.a[0][2] * A.a[1][1];
    C.a[1][0] = A.a[1][2] * A.a[2][0] - A.a[1][0] * A.a[2][2];
    C.a[1][1] = A.a[0][0] * A.a[2][2] - A.a[0][2] * A.a[2][0];
    C.a[1][2] = A.a[0][2] * A.a[1][0] - A.a[0][0] * A.a[1][2];
    C.a[2][0] = A.a[1][0] * A.a[2][1] - A.a[1][1] * A.a[2][0];
    C.a[2][1] = A.a[0][1] * A.a[2][0] - A.a[0][0] * A.a[2][1];
    C.a[2][2] = A.a[0][0] * A.a[1][1] - A.a[0][1] * A.a[1][0];
    const zc d = det3(A);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C.a[i][j] = cdiv(C.a[i][j], d);
    return C;
}

// cyclic Jacobi for a Hermitian 3x3 K; V collects the eigenvectors (columns)
__device__ void herm_jacobi(M3 &K, M3 &V, double ev[3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V.a[i][j] = mk<double>(i == j ? 1.0 : 0.0, 0.0);
    const int P[3] = {0, 0, 1}, Q[3] = {1, 2, 2};
    for (int sweep = 0; sweep < 12; ++sweep) {
        const double off = abs2(K.a[0][1]) + abs2(K.a[0][2]) + abs2(K.a[1][2]);
        const double dia = K.a[0][0].re * K.a[0][0].re + K.a[1][1].re * K.a[1][1].re + K.a[2][2].re * K.a[2][2].re;
        if (off <= 1e-34 * (dia + 1e-300)) break;
        for (int r = 0; r < 3; ++r) {
            const int p = P[r], q = Q[r];
            const double b = sqrt(abs2(K.a[p][q]));
            if (b == 0.0) continue;
            const zc ph = {K.a[p][q].re / b, K.a[p][q].im / b};  // e^{i phi}
            const zc phc = cj(ph);
            const double zeta = (K.a[q][q].re - K.a[p][p].re) / (2.0 * b);
            const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
            // J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] on (p, q)
            for (int i = 0; i < 3; ++i) {  // K <- K J, V <- V J
                zc kp = K.a[i][p], kq = K.a[i][q];
                K.a[i][p] = scale(c, kp) - scale(s, phc * kq);
                K.a[i][q] = scale(s, kp) + scale(c, phc * kq);
                zc vp = V.a[i][p], vq = V.a[i][q];
                V.a[i][p] = scale(c, vp) - scale(s, phc * vq);
                V.a[i][q] = scale(s, vp) + scale(c, phc * vq);
            }
            for (int j = 0; j < 3; ++j) {  // K <- J^+ K
                zc kp = K.a[p][j], kq = K.a[q][j];
                K.a[p][j] = scale(c, kp) - scale(s, ph * kq);
                K.a[q][j] = scale(s, kp) + scale(c, ph * kq);
            }
            K.a[p][q] = K.a[q][p] = mk<double>(0.0, 0.0);
            K.a[p][p].im = K.a[q][q].im = 0.0;
        }
    }
    for (int i = 0; i < 3; ++i) ev[i] = K.a[i][i].re;
}

// Up to PATH_OUTS points of one path per launch: the decomposition of W is
// done once per link and serves every t.
constexpr int PATH_OUTS = 32;
struct PathOuts {
    double t[PATH_OUTS];
    double2 *p[PATH_OUTS];
    int n;
};

__global__ __launch_bounds__(256) void k_interpolate(Geo g, const double2 *__restrict__ U,
                                                     const double2 *__restrict__ Up, PathOuts outs)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const long q = blockIdx.y;  // slot * 4 + mu
    const long base = q * 9 * g.Vb + l;
    M3 u, w;
    bool same = true;
    for (int e = 0; e < 9; ++e) {
        double2 a = U[base + (long)e * g.Vb], b = Up[base + (long)e * g.Vb];
        u.a[e / 3][e % 3] = mk<double>(a.x, a.y);
        w.a[e / 3][e % 3] = mk<double>(b.x, b.y);
        same = same && a.x == b.x && a.y == b.y;
    }
    if (same) {
        for (int k = 0; k < outs.n; ++k)
            for (int e = 0; e < 9; ++e) outs.p[k][base + (long)e * g.Vb] = make_double2(u.a[e / 3][e % 3].re, u.a[e / 3][e % 3].im);
        return;
    }
    // W = U' U^+
    M3 W;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            W.a[i][j] = conjmul(u.a[j][0], w.a[i][0]) + conjmul(u.a[j][1], w.a[i][1]) + conjmul(u.a[j][2], w.a[i][2]);
    // phase rotation keeping -1 away from the spectrum of e^{-i phi} W
    double best = -1.0, phi = 0.0;
    for (int c = 0; c < 12; ++c) {
        const double ph = c * (M_PI / 6.0);
        double sn, cs;
        sincos(ph, &sn, &cs);
        M3 A = W;
        for (int i = 0; i < 3; ++i) A.a[i][i] = A.a[i][i] + mk<double>(cs, sn);
        const double d = abs2(det3(A));
        if (d > best) {
            best = d;
            phi = ph;
        }
    }
    double sn, cs;
    sincos(phi, &sn, &cs);
    const zc rot = {cs, -sn};
    M3 Wr, Ip, Im;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            Wr.a[i][j] = rot * W.a[i][j];
            const double d = i == j ? 1.0 : 0.0;
            Ip.a[i][j] = mk<double>(d, 0.0) + Wr.a[i][j];
            Im.a[i][j] = mk<double>(d, 0.0) - Wr.a[i][j];
        }
    M3 K = mmul(Im, inv3(Ip));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) K.a[i][j] = mul_i(K.a[i][j]);
    M3 Kh;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Kh.a[i][j] = scale(0.5, K.a[i][j] + cj(K.a[j][i]));
    M3 V;
    double ev[3];
    herm_jacobi(Kh, V, ev);
    double th[3];
    for (int j = 0; j < 3; ++j) {
        double a = 2.0 * atan(ev[j]) + phi;
        while (a > M_PI) a -= 2.0 * M_PI;
        while (a <= -M_PI) a += 2.0 * M_PI;
        th[j] = a;
    }
    const double ssum = th[0] + th[1] + th[2];
    if (ssum > M_PI) {
        int j = th[0] >= th[1] ? (th[0] >= th[2] ? 0 : 2) : (th[1] >= th[2] ? 1 : 2);
        th[j] -= 2.0 * M_PI;
    } else if (ssum < -M_PI) {
        int j = th[0] <= th[1] ? (th[0] <= th[2] ? 0 : 2) : (th[1] <= th[2] ? 1 : 2);
        th[j] += 2.0 * M_PI;
    }
    // W^t = V diag(e^{i t theta}) V^+ ; out = W^t U, for every requested t
    for (int o = 0; o < outs.n; ++o) {
        const double t = outs.t[o];
        zc e[3];
        for (int j = 0; j < 3; ++j) {
            double s2, c2;
            sincos(t * th[j], &s2, &c2);
            e[j] = mk<double>(c2, s2);
        }
        M3 Wt;
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) {
                zc acc = mk<double>(0.0, 0.0);
                for (int j = 0; j < 3; ++j) acc = acc + e[j] * (V.a[i][j] * cj(V.a[k][j]));
                Wt.a[i][k] = acc;
            }
        const M3 R = mmul(Wt, u);
        for (int ee = 0; ee < 9; ++ee) {
            zc v = R.a[ee / 3][ee % 3];
            outs.p[o][base + (long)ee * g.Vb] = make_double2(v.re, v.im);
        }
    }
}

}  // namespace

void launch_interpolate_many(const Geo &g, const double2 *U, const double2 *Up, const double *t, double2 *const *out,
                             int n, hipStream_t s)
{
    for (int k0 = 0; k0 < n; k0 += PATH_OUTS) {
        PathOuts o;
        o.n = n - k0 < PATH_OUTS ? n - k0 : PATH_OUTS;
        for (int k = 0; k < o.n; ++k) {
            o.t[k] = t[k0 + k];
            o.p[k] = out[k0 + k];
        }
        k_interpolate<<<dim3((g.Vb + 255) / 256, g.nblk * 4), 256, 0, s>>>(g, U, Up, o);
    }
}

void launch_interpolate(const Geo &g, const double2 *U, const double2 *Up, double t, double2 *out, hipStream_t s)
{
    launch_interpolate_many(g, U, Up, &t, &out, 1, s);
}

}  // namespace wdr
