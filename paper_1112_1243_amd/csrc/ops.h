// Kernel launchers shared between the translation units of the library.
#pragma once

#include "wdr_internal.h"

namespace wdr {

// hop selection of the Wilson stencil (paper Sec. 3, eq. domdec)
enum Hops { HOPS_ALL = 0, HOPS_IN = 1, HOPS_CROSS = 2 };

// out(x) = diag(x) - kappa * sum_{selected hops} [...] in(y)
//   diag    NULL (no diagonal term) or a field supplying the diagonal term
//   slots   [slot0, slot0 + nslots) receive output; other slots untouched
//   par     -1 every site of those slots, 0 / 1 only the even / odd sites
//   dag     1: compute g5 (stencil) g5, i.e. the adjoint of D (gamma5-hermiticity)
template <typename T>
void launch_dslash(const Geo &g, int hops, int par, int dag, const typename C2<T>::type *U,
                   const typename C2<T>::type *in, const typename C2<T>::type *diag, typename C2<T>::type *out,
                   T kappa, int slot0, int nslots, hipStream_t s);

// canonical FP64 AoS spinor <-> internal layout in precision T
template <typename T> void launch_pack_spinor(const Geo &g, const double2 *canon, typename C2<T>::type *out, hipStream_t s);
template <typename T> void launch_unpack_spinor(const Geo &g, const typename C2<T>::type *in, double2 *canon, hipStream_t s);
// canonical FP64 gauge -> internal layout in precision T, bc folded in
template <typename T>
void launch_pack_gauge(const Geo &g, const int bc[4], const double2 *canon, typename C2<T>::type *out, hipStream_t s);
void launch_unpack_gauge(const Geo &g, const int bc[4], const double2 *in, double2 *canon, hipStream_t s);
void launch_convert_gauge_f32(const Geo &g, const double2 *in, float2 *out, hipStream_t s);

// ---------------------------------------------------------------- BLAS-1
// fields are arrays of n complex numbers

// out = a (copy with precision change)
template <typename TO, typename TI>
void launch_convert(const typename C2<TI>::type *a, typename C2<TO>::type *out, long n, hipStream_t s);
template <typename T> void launch_zero(typename C2<T>::type *a, long n, hipStream_t s);
// multiply spin components 2, 3 by -1 (gamma_5), in place allowed
template <typename T> void launch_g5(const Geo &g, const typename C2<T>::type *in, typename C2<T>::type *out, int slot0,
                                     int nslots, hipStream_t s);

// Deterministic FP64 reductions.  red: device scratch of at least
// RED_SCRATCH doubles.  Results land in device memory.
constexpr int RED_BLOCKS = 512;
constexpr int RED_SCRATCH = 2 * RED_BLOCKS * 16 + 64;
// out[j] = <v_j, y> for j < m  (m <= 16), complex
template <typename T>
void launch_multidot(const typename C2<T>::type *const *v_dev, int m, const typename C2<T>::type *y, long n,
                     double *red, double2 *out, hipStream_t s);
// out = <a, b>, complex
template <typename T>
void launch_dot(const typename C2<T>::type *a, const typename C2<T>::type *b, long n, double *red, double2 *out,
                hipStream_t s);
// out = ||a||^2 (in out->x)
template <typename T> void launch_norm2(const typename C2<T>::type *a, long n, double *red, double2 *out, hipStream_t s);

// y = y + f * c * x, c a device complex scalar, f a host real factor
void launch_axpy_dev(const double2 *c, double f, const double2 *x, double2 *y, long n, hipStream_t s);
// y = sum_j c[j] * v_j with v_j device pointers (m <= 16), accumulate into y if acc
void launch_multi_axpy(const double2 *c, double f, const double2 *const *v_dev, int m, double2 *y, long n, int acc,
                       hipStream_t s);
// y = y * (1 / sqrt(nrm->x))
void launch_scale_invsqrt(const double2 *nrm, double2 *y, long n, hipStream_t s);
// r = b - a  (FP64)
void launch_sub(const double2 *b, const double2 *a, double2 *r, long n, hipStream_t s);
// y = a * x + b * y (host real scalars)
void launch_axpby(double a, const double2 *x, double b, double2 *y, long n, hipStream_t s);
// y += x for FP64 y and x of precision T
template <typename T> void launch_add_to64(const typename C2<T>::type *x, double2 *y, long n, hipStream_t s);

// ---------------------------------------------------------------- SAP, MR
// For every block of one colour (slots [slot0, slot0+nslots)): residual
// r = eta - D x (full stencil, neighbours from x), nmr even-odd MR steps on
// D_b d = r, x += d.  Fields in precision T.
template <typename T>
void launch_sap_colour(const Geo &g, const typename C2<T>::type *U, const typename C2<T>::type *eta,
                       typename C2<T>::type *x, T kappa, int nmr, int slot0, int nslots, hipStream_t s);
// Block MR solve: for blocks in the slot range, d = nmr even-odd MR steps on
// D_b d = r (r given), written to d (overwritten).  Also returns per-slot
// squared residual norms of r in rn (double per slot) when rn != NULL.
template <typename T>
void launch_block_mr(const Geo &g, const typename C2<T>::type *U, const typename C2<T>::type *r,
                     typename C2<T>::type *d, T kappa, int nmr, int slot0, int nslots, hipStream_t s);
// per-slot squared norms: out[slot - slot0] = sum over the slot of |a|^2
void launch_slot_norm2(const Geo &g, const double2 *a, double *out, int slot0, int nslots, hipStream_t s);

// ---------------------------------------------------------------- noise, path
void launch_noise(const Geo &g, int kind, uint64_t seed, int step, int k, int black_only, double2 *out,
                  hipStream_t s);
// out = U_t = exp(t log(U' U^+)) U on internal FP64 links
void launch_interpolate(const Geo &g, const double2 *U, const double2 *Up, double t, double2 *out, hipStream_t s);
void launch_site_maps(const Geo &g, int32_t *bid, int32_t *col, int32_t *par, int32_t *pos, hipStream_t s);
void launch_active_links(const Geo &g, int lo, int hi, uint8_t *mask, hipStream_t s);

// per-site quadratic form of the sample: for slots in range, per-slot sums of
//   |eta|^2 - |z|^2 - 2 Re(conj(w) r)   (z, w, r may be NULL: term dropped)
void launch_sample_terms(const Geo &g, const double2 *eta, const double2 *z, const double2 *w, const double2 *r,
                         double *per_slot, int slot0, int nslots, hipStream_t s);

}  // namespace wdr
