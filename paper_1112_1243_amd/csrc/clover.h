// Clover (Sheikholeslami-Wohlert) term on the device: its storage and the
// site-local products the stencils fuse into their diagonal term.
//
//   D = A - kappa H,  A(x) = 1 + T(x),
//   T(x) = c_sw kappa (i/2) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}(x)
//
// (paper Sec. 3: the active links are defined for Wilson fermions with this
// term; Sec. 7: the clover action).  T commutes with gamma_5, so in the
// chiral basis A is two hermitian 6 x 6 blocks per site, one per chirality
// (spins 0, 1 and spins 2, 3), with block index 3 * (spin mod 2) + colour,
// i.e. spinor component c = 3 * spin + colour sits in block c / 6 at c % 6.
// A block is stored as 36 reals: the six real diagonal entries, then Re and
// Im of the 15 entries above the diagonal, row by row.  A clover field in
// precision T holds [slot][chirality][36][Vb] reals for A and then the same
// for A^-1 (offset 72 V reals), so a wavefront reads each entry of 64
// consecutive sites as one contiguous run.
#pragma once

#include "ops.h"

namespace wdr {
namespace dev {

// packed position of entry (i, j), i < j, among the 15 above the diagonal
constexpr int herm_k(int i, int j) { return i * 6 - i * (i + 1) / 2 + (j - i - 1); }

// entry pointer of block chi of site (slot, l): A, or A^-1 with inv
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *clov_at(const T *base, long V, int inv, int slot,
                                                                               int chi, int Vb, int l)
{
    return as_global(base) + (inv ? 72 * V : 0) + ((long)slot * 2 + chi) * 36 * Vb + l;
}

// y = M x for one packed hermitian block (entries Vb apart)
template <typename T>
__device__ __forceinline__ void clov_mul6(const __attribute__((address_space(1))) T *p, int Vb, const cx<T> x[6],
                                          cx<T> y[6])
{
#pragma unroll
    for (int i = 0; i < 6; ++i) y[i] = scale(p[(long)i * Vb], x[i]);
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i + 1; j < 6; ++j) {
            const int k = herm_k(i, j);
            const cx<T> a = mk<T>(p[(long)(6 + 2 * k) * Vb], p[(long)(7 + 2 * k) * Vb]);
            y[i] = y[i] + a * x[j];
            y[j] = y[j] + conjmul(a, x[i]);
        }
}

// v <- A v (inv = 0) or A^-1 v (inv = 1) at site (slot, l), in place
template <typename T>
__device__ __forceinline__ void clov_spinor(const T *base, long V, int inv, int slot, int Vb, int l, spinor<T> &v)
{
#pragma unroll
    for (int chi = 0; chi < 2; ++chi) {
        cx<T> x[6], y[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) x[i] = v.s[(6 * chi + i) / 3].c[(6 * chi + i) % 3];
        clov_mul6<T>(clov_at<T>(base, V, inv, slot, chi, Vb, l), Vb, x, y);
#pragma unroll
        for (int i = 0; i < 6; ++i) v.s[(6 * chi + i) / 3].c[(6 * chi + i) % 3] = y[i];
    }
}

// The clover part of a one-lane-per-site epilogue.  v holds the hop part
// (-kappa H in, gamma_5-conjugated already for the adjoint), dg the diagonal
// input (zeros where the launch has none); on return v holds the output:
// A dg + v (CLOV_DIAG) or A^-1 (dg + v) (CLOV_INV).  A commutes with gamma_5,
// so the adjoint needs nothing more.
template <typename T, int CL>
__device__ __forceinline__ void clov_site(const T *base, long V, int slot, int Vb, int l, const cx<T> dg[12],
                                          cx<T> v[12])
{
#pragma unroll
    for (int chi = 0; chi < 2; ++chi) {
        cx<T> x[6], y[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) x[i] = CL == CLOV_DIAG ? dg[6 * chi + i] : dg[6 * chi + i] + v[6 * chi + i];
        clov_mul6<T>(clov_at<T>(base, V, CL == CLOV_INV, slot, chi, Vb, l), Vb, x, y);
#pragma unroll
        for (int i = 0; i < 6; ++i) v[6 * chi + i] = CL == CLOV_DIAG ? y[i] + v[6 * chi + i] : y[i];
    }
}

}  // namespace dev
}  // namespace wdr
