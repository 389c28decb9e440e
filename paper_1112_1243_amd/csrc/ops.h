// Kernel launchers shared between the translation units of the library.
//
// Every launcher works on a batch of M independent systems that share one
// geometry: a field argument points at M consecutive fields of n = 12 V
// complex numbers, gauge fields come from a device table of M pointers, and
// `active` (device, M ints, may be NULL) switches individual systems off so
// a batched solver can stop the converged ones.  M = 1 is a single system.
#pragma once

#include "wdr_internal.h"

namespace wdr {

// hop selection of the Wilson stencil (paper Sec. 3, eq. domdec)
enum Hops { HOPS_ALL = 0, HOPS_IN = 1, HOPS_CROSS = 2 };

struct Sys {
    int M = 1;
    const int32_t *active = nullptr;  // device [M]
    long n = 0;                       // complex numbers per field (12 V)
    // optional device list of the systems a launch covers (count entries);
    // every system left out must be inactive.  Launchers that support it
    // size their grids by count (the others launch over all M, still correct)
    const int32_t *list = nullptr;
    int count = 0;
    // hs = log2(Vh) > 0: the elementwise passes that support it (norms, dots,
    // the CG updates, add_to64, sub_norm) visit only the even sites of every
    // block (the first Vh entries of each run of Vb = 2 Vh; the even-odd
    // solvers keep the odd halves of their vectors at zero)
    int hs = 0;
    int launch_m() const { return list ? count : M; }
    long ne() const { return hs ? n >> 1 : n; }  // elements visited per system
};

// log2(Vh) when the half-block volume is a power of two, else 0
inline int even_shift(const Geo &g)
{
    int s = 0;
    while ((1 << s) < g.Vh) ++s;
    return (1 << s) == g.Vh ? s : 0;
}

// canonical site index (site = x0 + L0*(x1 + L1*(x2 + L2*x3))) of local
// site l of slot `slot`; x receives the global coordinates
__device__ __forceinline__ long canon_index(const Geo &g, int slot, int l, int x[4])
{
    int b = g.slot_blk[slot];
    const uint32_t c = g.loc_coord[l];
    int loc[4] = {(int)(c & 255u), (int)((c >> 8) & 255u), (int)((c >> 16) & 255u), (int)(c >> 24)};
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (b % g.NB[mu]) * g.B[mu] + loc[mu];
        b /= g.NB[mu];
    }
    return x[0] + (long)g.L[0] * (x[1] + (long)g.L[1] * (x[2] + (long)g.L[2] * x[3]));
}

template <typename T> using T2 = typename C2<T>::type;
template <typename T> using UTab = const T2<T> *const *;  // device [M] gauge pointers

// what a stencil launch does with the clover term when its links carry one
// (the term and its layout: clover.h)
//   CLOV_DIAG  out = A diag - kappa H in      (the diagonal input times A)
//   CLOV_INV   out = A^-1 (diag - kappa H in) (diag may be absent)
enum { CLOV_NONE = 0, CLOV_DIAG = 1, CLOV_INV = 2 };

// the links of a batch: the device table of per-system gauge pointers,
// whether every field in it is SU(3) to SU3_TOL (then kernels may read two
// rows per link and rebuild the third), and optionally a device table of
// per-system hopping parameters (NULL: every system uses the kappa argument
// of the launch)
template <typename T> struct Links {
    UTab<T> tab;
    int su3;
    const double *kap = nullptr;
    int kneg = 0;  // stencil launches use -kap[m] (the kappa argument is then -kappa too)
    // clover term: device table of per-system clover fields (A then A^-1,
    // layout in clover.h; NULL: no clover term) and what a stencil launch
    // does with it (CLOV_NONE / CLOV_DIAG / CLOV_INV of clover.h)
    const T *const *ctab = nullptr;
    int cmode = 0;
};

// FP16 fields: [M][slot][12][Vb] values v / s with one power-of-two scale
// s = 2^ceil(log2 max |component|) per system and block ([M][nblk] floats)
struct H16 {
    h2 *v;
    float *s;
};
struct H16c {
    const h2 *v;
    const float *s;
};
// FP16 links of a batch: the first two rows of every link ([slot][mu][6][Vb],
// SU(3) fields only), per-system table and optional kappa table
struct Links16 {
    const h2 *const *tab;
    const double *kap = nullptr;
};

// out = in - kappa H in on one FP16 field (per-block scales) with the FP16
// two-row links U16 of an SU(3) field; false (nothing launched) unless the
// blocks are 4^4
bool launch_dslash_h16(const Geo &g, const h2 *U16, H16c in, H16 out, float kappa, hipStream_t s);

// out(x) = diag(x) - kappa * sum_{selected hops} [...] in(y), per system
//   diag    NULL (no diagonal term) or a field supplying the diagonal term
//   slots   [slot0, slot0 + nslots) receive output; other slots untouched
//   par     -1 every site of those slots, 0 / 1 only the even / odd sites
//           (then in is read only at sites of the other parity, so out may
//           be the same field as in: the odd half of x from its even half)
//   dag     1: g5 (stencil) g5, the adjoint of D (gamma5-hermiticity)
// r = b - D_b x on the slots [slot0, slot0 + nslots) (FP64, in-block hops)
// in one block-staged launch; false (nothing launched) where that kernel is
// not the context's choice for this launch (the caller then applies D_b and
// subtracts)
bool launch_block_residual(const Geo &g, const Sys &sy, Links<double> U, const double2 *x, const double2 *b,
                           double2 *r, double kappa, int slot0, int nslots, hipStream_t s);
template <typename T>
void launch_dslash(const Geo &g, const Sys &sy, Links<T> U, int hops, int par, int dag, const T2<T> *in,
                   const T2<T> *diag, T2<T> *out, T kappa, int slot0, int nslots, hipStream_t s);
// End of a round of the FP16 block solves on the slots [slot0, slot0 +
// nslots), in one pass: x += d (FP16 with block scales), then r = b - D_b x
// (FP64, in-block hops), rn[m * nblk + slot] = |r|^2 over the block and r16
// = r in FP16 with block scales (as launch_to_h16 rounds it); the FP64 r is
// not stored.  false (nothing launched) unless the blocks are 4^4, the links
// SU(3) without a clover term and the slot range has a schedule.
bool launch_block_round16(const Geo &g, const Sys &sy, Links<double> U, H16c d, double2 *x, const double2 *b,
                          H16 r16, double *rn, double kappa, int slot0, int nslots, hipStream_t s);

// Persistent form of `steps` steps of the even-odd CGNE (the step loop of
// the CG in solvers.hip: w = Dhat^+ p, q = Dhat w, x / r update, new p, the
// per-step control of k_cgm_beta) as one cooperative launch; part holds
// 3 * nblk * launch_m doubles.  Fits 4^4 blocks with SU(3) links and no
// clover term (cg_steps_fit); returns the launch status (nothing ran unless
// hipSuccess).
bool cg_steps_fit(const Geo &g, bool su3, bool clover);

// Halo of a slab cut along t (halo.hip): lo / hi receive the half spinors of
// the first / last t slice that the slabs below / above need ([6][F]
// complex, F = L0 L1 L2); unpack adds the hops across both faces from what
// the neighbours sent, times slo / shi (the links' boundary sign).  U:
// canonical FP64 links.
template <typename T>
void launch_halo_pack(const Geo &g, const double2 *U, const T2<T> *in, T2<T> *lo, T2<T> *hi, hipStream_t s);
template <typename T>
void launch_halo_unpack(const Geo &g, const double2 *U, T kappa, const T2<T> *lo, const T2<T> *hi, T slo, T shi,
                        T2<T> *out, hipStream_t s);
template <typename T>
hipError_t launch_cg_steps(const Geo &g, const Sys &sy, Links<T> U, T kappa, int steps, T2<T> *p, T2<T> *t,
                           T2<T> *w, T2<T> *q, T2<T> *r, T2<T> *e, double2 *sc, double *part, double delta2,
                           int max_iter, double *rmax, int32_t *upd, int32_t *its, hipStream_t s);

// ---------------------------------------------------------------- clover term
// A = 1 + T and A^-1 of every site (clover.h layout) in FP64 into c64 (144 V
// doubles) and rounded to FP32 into c32 (144 V floats), from the internal
// FP64 links U (boundary phases folded in; they cancel around the closed
// loops).  work: clover_work_bytes(g); worst (device, one double): the
// largest 1 / |pivot| of the LDL^H factorisations of the blocks (a singular
// block gives inf or nan).
size_t clover_work_bytes(const Geo &g);
void launch_clover_build(const Geo &g, const double2 *U, double csw, double kappa, void *work, double *c64, float *c32,
                         double *worst, hipStream_t s);
// out = A in (inv 0) or A^-1 in (inv 1) on the sites of parity par (-1: all)
// of every system; other sites of out are untouched
template <typename T>
void launch_clover_mul(const Geo &g, const Sys &sy, const T *const *ctab, int inv, int par, const T2<T> *in,
                       T2<T> *out, hipStream_t s);
// A (inv 0) or A^-1 (inv 1) of one FP64 clover field as canonical [V][12][12]
// complex (row and column 3 * spin + colour)
void launch_clover_canon(const Geo &g, const double *c64, int inv, double2 *canon, hipStream_t s);

// canonical FP64 AoS spinor <-> internal layout in precision T (one field)
template <typename T> void launch_pack_spinor(const Geo &g, const double2 *canon, T2<T> *out, hipStream_t s);
template <typename T> void launch_unpack_spinor(const Geo &g, const T2<T> *in, double2 *canon, hipStream_t s);
// canonical FP64 gauge -> internal layout in precision T, bc folded in
template <typename T>
void launch_pack_gauge(const Geo &g, const int bc[4], const double2 *canon, T2<T> *out, hipStream_t s);
void launch_unpack_gauge(const Geo &g, const int bc[4], const double2 *in, double2 *canon, hipStream_t s);
void launch_block_fields(const Geo &g, const int bc[4], const double2 *in, double2 *out, hipStream_t s);
void launch_convert_gauge_f32(const Geo &g, const double2 *in, float2 *out, hipStream_t s);
// largest deviation from SU(3) over the links (max |U U^+ - 1|, |det U - 1|,
// boundary phases divided out); dev_out: one double
void launch_su3_deviation(const Geo &g, const double2 *U, double *partial, double *dev_out, hipStream_t s);

// ---------------------------------------------------------------- BLAS-1
// Elementwise kernels act on all M * n elements of the batch; per-system
// scalars live in device arrays indexed by the system.

template <typename TO, typename TI>
void launch_convert(const Sys &sy, const T2<TI> *a, T2<TO> *out, hipStream_t s);
// out = (float) a and z = 0 over all M fields
void launch_convert_zero_f32(const Sys &sy, const double2 *a, float2 *out, float2 *z, hipStream_t s);
template <typename T> void launch_zero(T2<T> *a, long n, hipStream_t s);
// block-solve residual: on the slots [slot0, slot0 + nslots) r = b - t (t NULL:
// r already holds it) and out[m * nblk + slot] = |r|^2 over the slot; the
// other slots of r are left as they are
void launch_block_resid_norm(const Geo &g, const Sys &sy, const double2 *b, const double2 *t, double2 *r,
                             double *out, int slot0, int nslots, hipStream_t s);
// zero every site outside the slot range [slot0, slot0 + nslots) of each system
void launch_keep_slots(const Geo &g, const Sys &sy, double2 *f, int slot0, int nslots, hipStream_t s);
// multiply spin components 2, 3 by -1 (gamma_5), in place allowed
template <typename T> void launch_g5(const Geo &g, const Sys &sy, const T2<T> *in, T2<T> *out, hipStream_t s);

// Deterministic FP64 reductions (fixed grid, fixed order); red: device
// scratch of red_scratch(M) doubles; results in device memory.
constexpr int RED_BLOCKS = 256;
inline long red_scratch(int M) { return 2L * RED_BLOCKS * 16 * M + 64; }
// out[m * ostride + j] = <v_j[m], y[m]> for j < nv (nv <= 16), v_j given by a
// device table of nv batch fields
template <typename T>
void launch_multidot(const Sys &sy, const T2<T> *const *v, int nv, const T2<T> *y, double *red, double2 *out,
                     int ostride, hipStream_t s);
// out[m * ostride] = <a[m], b[m]>
template <typename T>
void launch_dot(const Sys &sy, const T2<T> *a, const T2<T> *b, double *red, double2 *out, int ostride, hipStream_t s);
// out[m * ostride].x = ||a[m]||^2
template <typename T>
void launch_norm2(const Sys &sy, const T2<T> *a, double *red, double2 *out, int ostride, hipStream_t s);

// Fused solver passes (same deterministic reductions; out written like launch_norm2):
// CG step with alpha = sc[m*sstride].x / sc[m*sstride+1].x (0 if the latter is
// not positive): x += alpha w, r -= alpha q, out[m * ostride].x = ||r[m]||^2
template <typename T>
void launch_cg_xr_norm(const Sys &sy, const double2 *sc, int sstride, T2<T> *x, const T2<T> *w, T2<T> *r,
                       const T2<T> *q, double *red, double2 *out, int ostride, hipStream_t s);
// out_n[m * nstride] = (||a[m]||^2, 0), out_d[m * dstride] = <a[m], b[m]> / ||a[m]||
void launch_norm_dot(const Sys &sy, const double2 *a, const double2 *b, double *red, double2 *out_n, int nstride,
                     double2 *out_d, int dstride, hipStream_t s);
// a[m] *= 1 / sqrt(nrm[m * nstride].x), b[m] -= c[m * cstride] a[m], out[m * ostride].x = ||b[m]||^2
void launch_orth_norm(const Sys &sy, const double2 *nrm, int nstride, const double2 *c, int cstride, double2 *a,
                      double2 *b, double *red, double2 *out, int ostride, hipStream_t s);
// y[m] -= sum_{j < nv} c[m * cstride + j] v_j[m] (1 <= nv <= 16), then
// out[m * ostride + j] = <v_j[m], y[m]>
void launch_cgs_multidot(const Sys &sy, const double2 *c, int cstride, const double2 *const *v, int nv, double2 *y,
                         double *red, double2 *out, int ostride, hipStream_t s);
// the same update, then out_n[m * nstride] = (||y[m]||^2, 0), out_d[m * dstride] = <y[m], b[m]> / ||y[m]||
void launch_cgs_norm_dot(const Sys &sy, const double2 *c, int cstride, const double2 *const *v, int nv, double2 *y,
                         const double2 *b, double *red, double2 *out_n, int nstride, double2 *out_d, int dstride,
                         hipStream_t s);
// r = b - a, out[m * ostride].x = ||r[m]||^2
void launch_sub_norm(const Sys &sy, const double2 *b, const double2 *a, double2 *r, double *red, double2 *out,
                     int ostride, hipStream_t s);

// y[m] = (acc ? y[m] : 0) + f * sum_{j < cnt[m]} c[m * cstride + j] v_j[m]  (cnt NULL: all nv)
void launch_multi_axpy(const Sys &sy, const double2 *c, int cstride, double f, const double2 *const *v, int nv,
                       const int32_t *cnt, double2 *y, int acc, hipStream_t s);
// r = b - a
void launch_sub(const Sys &sy, const double2 *b, const double2 *a, double2 *r, hipStream_t s);
// y += x for FP64 y and x of precision T
template <typename T> void launch_add_to64(const Sys &sy, const T2<T> *x, double2 *y, hipStream_t s);

// ---------------------------------------------------------------- SAP, MR
// Schwarz half-sweep on the blocks of one colour (slots [slot0, slot0 +
// nslots)): r = eta - D x (neighbours from x), nmr even-odd MR steps on
// D_b d = r, x += d.
template <typename T>
void launch_sap_colour(const Geo &g, const Sys &sy, Links<T> U, const T2<T> *eta, T2<T> *x, T kappa, int nmr,
                       int slot0, int nslots, hipStream_t s);
// Block MR: d = nmr even-odd MR steps on D_b d = r for the blocks in range.
template <typename T>
void launch_block_mr(const Geo &g, const Sys &sy, Links<T> U, const T2<T> *r, T2<T> *d, T kappa, int nmr, int slot0,
                     int nslots, hipStream_t s);
// out[m * g.nblk + slot] = sum over the slot of |a|^2, slots in range
void launch_slot_norm2(const Geo &g, const Sys &sy, const double2 *a, double *out, int slot0, int nslots,
                       hipStream_t s);

// ---------------------------------------------------------------- FP16 storage
// out = FP16 copy of in on the slots [slot0, slot0 + nslots) with fresh block scales
template <typename T>
void launch_to_h16(const Geo &g, const Sys &sy, const T2<T> *in, H16 out, int slot0, int nslots, hipStream_t s);
// y (+)= in on the slots [slot0, slot0 + nslots) (add = 1: y += in); other slots untouched
void launch_from_h16(const Geo &g, const Sys &sy, H16c in, double2 *y, int add, int slot0, int nslots,
                     hipStream_t s);
// values 0, scales 1
void launch_zero_h16(const Geo &g, const Sys &sy, H16 f, hipStream_t s);
// FP16 copy of the first two rows of the internal FP64 links
void launch_pack_links_h16(const Geo &g, const double2 *u64, h2 *u16, hipStream_t s);
// block MR with FP16 storage (4^4 blocks, SU(3) links): mode 0 is the Schwarz
// sweep of launch_sap_colour, mode 1 the block MR of launch_block_mr (ctab:
// the FP32 clover fields per system for the clover operator, mode 1 only);
// false if the geometry or the links do not allow it
bool launch_mr_h16(int mode, const Geo &g, const Sys &sy, Links16 U, H16c src, H16 dst, float kappa, int nmr,
                   int slot0, int nslots, hipStream_t s, const float *const *ctab = nullptr);

// ---------------------------------------------------------------- FP16 even-odd CG
// One parity of every block in FP16, site-major ([M][slot][Vh][12] complex,
// 48 bytes per site) with one power-of-two scale per (system, slot); the CG
// vectors of the FP16 inner level of the even-odd CGNE (4^4 blocks).
struct E16 {
    uint4 *v;
    float *s;
};
struct E16c {
    const uint4 *v;
    const float *s;
};
inline E16c cref(const E16 &f) { return E16c{f.v, f.s}; }
// 4^4 blocks in a 2-colourable checkerboard
bool e16_geometry(const Geo &g);
size_t e16_field_bytes(const Geo &g, int M);
E16 e16_field(const Geo &g, int M, void *p);
// E16 links (first two rows, [slot][parity][mu] chunks) of internal FP64 links
void launch_pack_links_e16(const Geo &g, const double2 *u64, h2 *e16, hipStream_t s);
// out = diag + f H_{par, 1-par} in (gamma_5 on both sides for dag), f = fs
// kappa_m with a kappa table in U, else fk; partial (may be NULL): |out|^2
// per (system, slot) for the deterministic reduction (2 doubles each); ctab
// (FP32 clover terms per system) with cmode CLOV_DIAG: A times the diagonal,
// CLOV_INV: A^-1 times the whole output
void launch_eo16(const Geo &g, const Sys &sy, Links16 U, float fs, float fk, int par, int dag, E16c in, E16c diag,
                 E16 out, double *partial, hipStream_t s, const float *const *ctab = nullptr,
                 int cmode = CLOV_NONE);
// x += alpha w (x FP32 internal layout, even sites), r -= alpha q, |r|^2 partials;
// alpha = sc[8m].x / sc[8m + 1].x; x NULL: no x update, alpha stored in alpha[m]
void launch_xr16(const Geo &g, const Sys &sy, const double2 *sc, float2 *x, float *alpha, E16c w, E16c q, E16 r,
                 double *partial, hipStream_t s);
// x += alpha_j w_j, j = 0 .. nk - 1 (nk <= 4) in step order: the x updates
// that launch_xr16 with x = NULL deferred (alpha_j of system m at alpha[j M + m])
void launch_x16_flush(const Geo &g, const Sys &sy, const float *alpha, int M, const E16c *w, int nk, float2 *x,
                      hipStream_t s);
// p = r + sc[8m + 4].x p, or p = r (copy)
void launch_p16(const Geo &g, const Sys &sy, const double2 *sc, int copy, E16c r, E16 p, hipStream_t s);
// r = bh - d (FP32 internal layout, even sites) into FP16, |r|^2 partials
void launch_r16_from32(const Geo &g, const Sys &sy, const float2 *bh, const float2 *d, E16 r, double *partial,
                       hipStream_t s);
// r = r64 into FP16, bh = (float) r64, x = 0 (even sites)
void launch_r16_from64(const Geo &g, const Sys &sy, const double2 *r64, float2 *bh, float2 *x, E16 r, hipStream_t s);
// the sites of parity par of M internal FP64 fields into E16 (fresh scales),
// and back (the other parity set to zero)
void launch_e16_from64(const Geo &g, int M, int par, const double2 *in, E16 out, hipStream_t s);
void launch_e16_to64(const Geo &g, int M, int par, E16c in, double2 *out, hipStream_t s);
// out[m * ostride].x = sum of the G partial pairs of system m (fixed order)
void launch_final(const Sys &sy, const double *partial, int G, double2 *out, int ostride, hipStream_t s);

// ---------------------------------------------------------------- noise, path
// system m gets the noise of path step steps[m], sample ks[m] (device
// arrays) under key (seeds[m], 3), or (seed, 3) when seeds is NULL
void launch_noise(const Geo &g, const Sys &sy, int kind, uint64_t seed, const uint64_t *seeds, const int32_t *steps,
                  const int32_t *ks, int black_only, double2 *out, hipStream_t s);
// out = U_t = exp(t log(U' U^+)) U on internal FP64 links
void launch_interpolate(const Geo &g, const double2 *U, const double2 *Up, double t, double2 *out, hipStream_t s);
// several points t[k] of the same path into out[k] (one decomposition of
// U' U^+ per link for all of them)
void launch_interpolate_many(const Geo &g, const double2 *U, const double2 *Up, const double *t, double2 *const *out,
                             int n, hipStream_t s);
void launch_site_maps(const Geo &g, int32_t *bid, int32_t *col, int32_t *par, int32_t *pos, hipStream_t s);
void launch_active_links(const Geo &g, int lo, int hi, uint8_t *mask, hipStream_t s);

// per-slot sums of |eta|^2 - |z|^2 - 2 Re(conj(w) r) into per_slot[m * nblk + slot]
void launch_sample_terms(const Geo &g, const Sys &sy, const double2 *eta, const double2 *z, const double2 *w,
                         const double2 *r, double *per_slot, hipStream_t s);

}  // namespace wdr
