// Block minimal-residual solver and Schwarz sweep for gfx950.
//
// Domain decomposition (paper Sec. 3) with the Schwarz alternating
// procedure of Luscher (hep-lat/0310048, cited in Secs. 1 and 3).  One
// workgroup owns one block of Vb <= 256 sites, one lane per site (even
// sites in the first half of the workgroup, odd sites in the second, so the
// two halves are separate wavefronts).  The even-odd reduced block system
//     (1 - kappa^2 H_eo H_oe) d_e = r_e + kappa H_eo r_o,
//     d_o = r_o + kappa H_oe d_e,                    (D_b = 1 - kappa H_b)
// is solved by MR steps with both half fields resident in LDS; only the
// links are read from global memory (they stay in L2 across the steps).
// Per-block inner products are wavefront shuffles plus an LDS tree.
#include "clover.h"
#include "half2.h"
#include "lds_stencil.h"

namespace wdr {
namespace {

using namespace dev;

constexpr int MAXVB = 256;

// sum over the first `width` lanes (width = 16, 32 or 64: blocks smaller
// than a wavefront have a partial wavefront of a power-of-two size)
template <typename T> __device__ __forceinline__ T wave_sum(T v, int width)
{
    for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_down(v, off, width);
    return v;
}

// x moved across lanes by the DPP control CTRL into the rows of ROWS (zero
// where the source lane lies outside the row, and in the other rows)
template <int CTRL, int ROWS> __device__ __forceinline__ float dpp_in(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xf, true));
}
// the sum over a full wavefront by DPP row shifts and row broadcasts (vector
// ALU only, no LDS permutes), valid in lane 63.  The broadcasts write every
// row (so each step is one DPP add): lane 31 then holds rows 0 + 1 and lane
// 63 rows 2 + 3, then all four; the other lanes end with partial sums that
// nothing reads.
__device__ __forceinline__ float wave_total63(float v)
{
    v += dpp_in<0x111, 0xf>(v);  // row_shr:1
    v += dpp_in<0x112, 0xf>(v);  // row_shr:2
    v += dpp_in<0x114, 0xf>(v);  // row_shr:4
    v += dpp_in<0x118, 0xf>(v);  // row_shr:8: lane 15 of a row holds the row's sum
    v += dpp_in<0x142, 0xf>(v);  // row_bcast:15: lane 15 of each row into the next row
    v += dpp_in<0x143, 0xf>(v);  // row_bcast:31: lane 31 into rows 2 and 3
    return v;
}
// the lane of a wavefront that wave_total returns the full sum in
template <typename T> constexpr int TOTAL_LANE = sizeof(T) == 4 ? 63 : 0;
template <typename T> __device__ __forceinline__ T wave_total(T v)
{
    if constexpr (sizeof(T) == 4)
        return wave_total63(v);
    else
        return wave_sum(v, 64);
}

// MODE 0: Schwarz sweep on one colour: r = eta - D x (global stencil on x),
//         MR on the block, x += d.
// MODE 1: block MR for a given right-hand side: d = MR(D_b, rhs).
// CL: with the clover term (ctab, A and A^-1 per site, clover.h): D_b = A -
// kappa H_b, the reduced system (A_ee - kappa^2 H_eo A_oo^-1 H_oe) d_e =
// r_e + kappa H_eo A_oo^-1 r_o and d_o = A_oo^-1 (r_o + kappa H_oe d_e); the
// site blocks are read from memory where they are applied.
template <typename T, int MODE, int CL>
__global__ __launch_bounds__(MAXVB) void k_block_mr(Geo g, const int32_t *__restrict__ active, UTab<T> Utab,
                                                    const T *const *__restrict__ ctab, const double *__restrict__ kap,
                                                    long n, const typename C2<T>::type *__restrict__ src,
                                                    typename C2<T>::type *__restrict__ dst, T kappa, int nmr,
                                                    int slot0)
{
    typedef typename C2<T>::type T2;
    __shared__ T2 she[12 * MAXVB / 2];
    __shared__ T2 sho[12 * MAXVB / 2];
    __shared__ T red[3][MAXVB / 64];
    __shared__ T alpha_sh[2];

    const int m = blockIdx.y;
    if (active && !active[m]) return;
    if (kap) kappa = (T)kap[m];
    const typename C2<T>::type *__restrict__ U = Utab[m];
    const T *C = CL ? ctab[m] : nullptr;
    const long V = g.V;
    src += m * n;
    dst += m * n;
    const int Vb = g.Vb, Vh = g.Vh;
    const int slot = slot0 + blockIdx.x;
    const int l = threadIdx.x;
    const bool even = l < Vh;
    const int hi = even ? l : l - Vh;
    const int nw = (Vb + 63) / 64;
    const int ww = Vb < 64 ? Vb : 64;
    int x[4];
    local_coords(g, l, x);

    // ---- residual of the block system at this site
    spinor<T> r, acc;
    if (MODE == 0) {
        hop_sum<T, HOPS_ALL>(g, U, slot, l, x, GlobalLoader<T>{dst, Vb}, acc);
        spinor<T> e, xs;
        load_site<T>(src, slot, Vb, l, e);
        load_site<T>(dst, slot, Vb, l, xs);
        if (CL) clov_spinor<T>(C, V, 0, slot, Vb, l, xs);  // the diagonal term A x
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                r.s[sp].c[a] = e.s[sp].c[a] - xs.s[sp].c[a] + scale(kappa, acc.s[sp].c[a]);
    } else {
        load_site<T>(src, slot, Vb, l, r);
    }

    // ---- rhs_e = r_e + kappa H_eo r_o (A_oo^-1 r_o with the clover term)
    if (!even) {
        spinor<T> ro = r;
        if (CL) clov_spinor<T>(C, V, 1, slot, Vb, l, ro);
        lds_store<T>(sho, Vh, hi, ro);
    }
    __syncthreads();
    spinor<T> rho, del;
    if (even) {
        hop_sum<T, HOPS_IN>(g, U, slot, l, x, LdsLoader<T>{sho, Vh, Vh}, acc);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                rho.s[sp].c[a] = r.s[sp].c[a] + scale(kappa, acc.s[sp].c[a]);
                del.s[sp].c[a] = mk<T>(0, 0);
            }
        lds_store<T>(she, Vh, hi, rho);
    }

    // ---- MR steps on (1 - kappa^2 H_eo H_oe)
    const T k2 = kappa * kappa;
    for (int it = 0; it < nmr; ++it) {
        __syncthreads();
        if (!even) {  // t_o = H_oe rho (A_oo^-1 H_oe rho)
            hop_sum<T, HOPS_IN>(g, U, slot, l, x, LdsLoader<T>{she, Vh, 0}, acc);
            if (CL) clov_spinor<T>(C, V, 1, slot, Vb, l, acc);
            lds_store<T>(sho, Vh, hi, acc);
        }
        __syncthreads();
        T pr = 0, pi = 0, pp = 0;
        spinor<T> p;
        if (even) {  // p = rho - kappa^2 H_eo t_o (A_ee rho - ...)
            hop_sum<T, HOPS_IN>(g, U, slot, l, x, LdsLoader<T>{sho, Vh, Vh}, acc);
            spinor<T> dg = rho;
            if (CL) clov_spinor<T>(C, V, 0, slot, Vb, l, dg);
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    p.s[sp].c[a] = dg.s[sp].c[a] - scale(k2, acc.s[sp].c[a]);
                    const cx<T> q = conjmul(p.s[sp].c[a], rho.s[sp].c[a]);
                    pr += q.re;
                    pi += q.im;
                    pp += p.s[sp].c[a].re * p.s[sp].c[a].re + p.s[sp].c[a].im * p.s[sp].c[a].im;
                }
        }
        pr = wave_sum(pr, ww);
        pi = wave_sum(pi, ww);
        pp = wave_sum(pp, ww);
        if ((l & 63) == 0) {
            red[0][l >> 6] = pr;
            red[1][l >> 6] = pi;
            red[2][l >> 6] = pp;
        }
        __syncthreads();
        if (l == 0) {
            T sr = 0, si = 0, sp2 = 0;
            for (int w = 0; w < nw; ++w) {
                sr += red[0][w];
                si += red[1][w];
                sp2 += red[2][w];
            }
            alpha_sh[0] = sp2 > 0 ? sr / sp2 : T(0);
            alpha_sh[1] = sp2 > 0 ? si / sp2 : T(0);
        }
        __syncthreads();
        const cx<T> al = mk<T>(alpha_sh[0], alpha_sh[1]);
        if (even) {
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    del.s[sp].c[a] = del.s[sp].c[a] + al * rho.s[sp].c[a];
                    rho.s[sp].c[a] = rho.s[sp].c[a] - al * p.s[sp].c[a];
                }
            lds_store<T>(she, Vh, hi, rho);
        }
    }

    // ---- d_o = r_o + kappa H_oe d_e
    __syncthreads();
    if (even) lds_store<T>(she, Vh, hi, del);
    __syncthreads();
    if (!even) {
        hop_sum<T, HOPS_IN>(g, U, slot, l, x, LdsLoader<T>{she, Vh, 0}, acc);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) del.s[sp].c[a] = r.s[sp].c[a] + scale(kappa, acc.s[sp].c[a]);
        if (CL) clov_spinor<T>(C, V, 1, slot, Vb, l, del);  // d_o = A_oo^-1 (...)
    }

    if (MODE == 0) {
        spinor<T> xs;
        load_site<T>(dst, slot, Vb, l, xs);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) xs.s[sp].c[a] = xs.s[sp].c[a] + del.s[sp].c[a];
        // every lane of the block has read x (neighbour reads of this block
        // only come from this workgroup) before any lane writes it
        __syncthreads();
        store_site<T>(dst, slot, Vb, l, xs);
    } else {
        store_site<T>(dst, slot, Vb, l, del);
    }
}

// Same algorithm for B^4 blocks with the block (links included) in LDS:
// every MR step then runs from LDS only.
template <typename T, int MODE, int B>
__global__ __launch_bounds__(Cube<B>::Vb) void k_block_mr_cube(Geo g, const int32_t *__restrict__ active,
                                                               UTab<T> Utab, const double *__restrict__ kap, long n,
                                                               const int32_t *__restrict__ sched,
                                                               const typename C2<T>::type *__restrict__ src,
                                                               typename C2<T>::type *__restrict__ dst, T kappa,
                                                               int nmr)
{
    typedef Cube<B> CB;
    __shared__ CubeLds<T, B> S;
    constexpr int Vb = CB::Vb, Vh = CB::Vh;
    const int m = blockIdx.y;
    if (active && !active[m]) return;
    if (kap) kappa = (T)kap[m];
    const typename C2<T>::type *__restrict__ U = Utab[m];
    src += m * n;
    dst += m * n;
    const int slot = sched[blockIdx.x];
    const int l = threadIdx.x;
    const bool even = l < Vh;
    const int hi = even ? l : l - Vh;
    int x[4];
    CB::coords(l, x);

    // stage the block's links (two rows) in LDS
    {
        const long base = (long)slot * 4 * 9 * Vb + l;
        const auto *Ug = as_global(U);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int e = 0; e < 6; ++e) st<T>(S.lk, (mu * 6 + e) * Vb + l, ldg<T>(Ug, base + (long)(mu * 9 + e) * Vb));
    }

    spinor<T> r, acc;
    if (MODE == 0) {
        int nbr[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) nbr[k] = g.slot_nbr[slot * 8 + k];
        hop_sum_cube<T, HOPS_ALL, B, 0>(U, dst, slot, nbr, l, x, acc);
        spinor<T> e, xs;
        load_site<T>(src, slot, Vb, l, e);
        load_site<T>(dst, slot, Vb, l, xs);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                r.s[sp].c[a] = e.s[sp].c[a] - xs.s[sp].c[a] + scale(kappa, acc.s[sp].c[a]);
    } else {
        load_site<T>(src, slot, Vb, l, r);
    }

    if (!even) lds_store<T>(S.sho, Vh, hi, r);
    __syncthreads();
    spinor<T> rho, del;
    if (even) {
        hop_in_lds<T, B>(S.sho, Vh, S.lk, l, x, acc);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                rho.s[sp].c[a] = r.s[sp].c[a] + scale(kappa, acc.s[sp].c[a]);
                del.s[sp].c[a] = mk<T>(0, 0);
            }
        lds_store<T>(S.she, Vh, hi, rho);
    }
    const T k2 = kappa * kappa;
    for (int it = 0; it < nmr; ++it) {
        __syncthreads();
        if (!even) {
            hop_in_lds<T, B>(S.she, 0, S.lk, l, x, acc);
            lds_store<T>(S.sho, Vh, hi, acc);
        }
        __syncthreads();
        T pr = 0, pi = 0, pp = 0;
        spinor<T> p;
        if (even) {
            hop_in_lds<T, B>(S.sho, Vh, S.lk, l, x, acc);
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    p.s[sp].c[a] = rho.s[sp].c[a] - scale(k2, acc.s[sp].c[a]);
                    const cx<T> q = conjmul(p.s[sp].c[a], rho.s[sp].c[a]);
                    pr += q.re;
                    pi += q.im;
                    pp += p.s[sp].c[a].re * p.s[sp].c[a].re + p.s[sp].c[a].im * p.s[sp].c[a].im;
                }
        }
        pr = wave_sum(pr, 64);
        pi = wave_sum(pi, 64);
        pp = wave_sum(pp, 64);
        if ((l & 63) == 0) {
            S.red[0][l >> 6] = pr;
            S.red[1][l >> 6] = pi;
            S.red[2][l >> 6] = pp;
        }
        __syncthreads();
        if (l == 0) {
            T sr = 0, si = 0, sq = 0;
#pragma unroll
            for (int w = 0; w < Vb / 64; ++w) {
                sr += S.red[0][w];
                si += S.red[1][w];
                sq += S.red[2][w];
            }
            S.alpha[0] = sq > 0 ? sr / sq : T(0);
            S.alpha[1] = sq > 0 ? si / sq : T(0);
        }
        __syncthreads();
        const cx<T> al = mk<T>(S.alpha[0], S.alpha[1]);
        if (even) {
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    del.s[sp].c[a] = del.s[sp].c[a] + al * rho.s[sp].c[a];
                    rho.s[sp].c[a] = rho.s[sp].c[a] - al * p.s[sp].c[a];
                }
            lds_store<T>(S.she, Vh, hi, rho);
        }
    }
    __syncthreads();
    if (even) lds_store<T>(S.she, Vh, hi, del);
    __syncthreads();
    if (!even) {
        hop_in_lds<T, B>(S.she, 0, S.lk, l, x, acc);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) del.s[sp].c[a] = r.s[sp].c[a] + scale(kappa, acc.s[sp].c[a]);
    }
    if (MODE == 0) {
        spinor<T> xs;
        load_site<T>(dst, slot, Vb, l, xs);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) xs.s[sp].c[a] = xs.s[sp].c[a] + del.s[sp].c[a];
        __syncthreads();
        store_site<T>(dst, slot, Vb, l, xs);
    } else {
        store_site<T>(dst, slot, Vb, l, del);
    }
}

// ---------------------------------------------------------------- 4^4 blocks, direction-parallel
// The same algorithm with 4 Vh threads per block.  In a hop phase over the
// sites of one parity, thread (mu, h) computes the two in-block hops of
// direction mu at site h of that parity and leaves its partial sum in LDS;
// in the vector phases thread (q, h) owns spin q of site h, so the MR updates
// and inner products are spread over all threads.  mu and q are uniform per
// wavefront (Vh is a multiple of 64).  Thread (mu, h) keeps the four links
// of its hops in registers (forward and backward, at site h of either
// parity, third rows rebuilt once), so the hop phases read only spinors from
// LDS.  LDS: both half fields and the four partial sums (FP32: 74 KB for
// 4^4).
template <typename T, int B> struct DirLds {
    typedef typename C2<T>::type T2;
    static constexpr int Vb = Cube<B>::Vb, Vh = Cube<B>::Vh, NT = 4 * Vh;
    T2 she[12 * Vh];
    T2 sho[12 * Vh];
    T2 part[4 * 12 * Vh];
    T red[3][NT / 64];
    T alpha[2];
};

// The links and LDS neighbour indices of thread (MU, h) of k_block_mr_dir:
// entry p is for the output site h of parity p (even xe / odd xo): forward
// link U_mu(x), backward link U_mu(x - mu), and the indices of x + mu and
// x - mu in the LDS half field of the other parity (a hop that leaves the
// block: index 0 and a zero link).
template <typename T> struct HopRegs {
    su3<T> f[2], b[2];
    int nf[2], nb[2];
};

template <typename T> __device__ __forceinline__ void zero_link(su3<T> &u)
{
#pragma unroll
    for (int e = 0; e < 9; ++e) u.m[e / 3][e % 3] = mk<T>(0, 0);
}

// reads the first two rows of the link at site l, direction MU, and rebuilds
// the third (in-block links never carry the boundary sign)
template <typename T, int B, int MU, int ST>
__device__ __forceinline__ void load_link_rows(const void *Utab_m, int slot, int l, su3<T> &u)
{
    constexpr int Vb = Cube<B>::Vb;
    if constexpr (ST) {
        const auto *Ug = as_global(static_cast<const h2 *>(Utab_m));
        const long base = (long)slot * 4 * 6 * Vb + (long)MU * 6 * Vb + l;
#pragma unroll
        for (int e = 0; e < 6; ++e) u.m[e / 3][e % 3] = ldh(Ug, base + (long)e * Vb, 1.f);
    } else {
        const auto *Ug = as_global(static_cast<const typename C2<T>::type *>(Utab_m));
        const long base = (long)slot * 4 * 9 * Vb + (long)MU * 9 * Vb + l;
#pragma unroll
        for (int e = 0; e < 6; ++e) u.m[e / 3][e % 3] = ldg<T>(Ug, base + (long)e * Vb);
    }
    reconstruct(u);
}

template <typename T, int B, int MU, int ST>
__device__ __forceinline__ void load_hop_regs(const void *Utab_m, int slot, int h, const int xe[4], const int xo[4],
                                              HopRegs<T> &R)
{
    typedef Cube<B> CB;
#pragma unroll
    for (int par = 0; par < 2; ++par) {
        const int *x = par ? xo : xe;
        const int l = par * CB::Vh + h;
        const int off = par ? 0 : CB::Vh;  // the neighbours have the other parity
        int y[4] = {x[0], x[1], x[2], x[3]};
        // a hop that leaves the block keeps LDS index 0 and a zero link: it
        // adds exact zeros, so every lane takes both hops without a branch
        R.nf[par] = R.nb[par] = 0;
        if (x[MU] + 1 < B) {
            y[MU] = x[MU] + 1;
            R.nf[par] = CB::index(y) - off;
            load_link_rows<T, B, MU, ST>(Utab_m, slot, l, R.f[par]);
        } else {
            zero_link(R.f[par]);
        }
        if (x[MU] > 0) {
            y[MU] = x[MU] - 1;
            const int nl = CB::index(y);
            R.nb[par] = nl - off;
            load_link_rows<T, B, MU, ST>(Utab_m, slot, nl, R.b[par]);
        } else {
            zero_link(R.b[par]);
        }
    }
}

// hop phase of thread (mu, h): the in-block hops of direction mu at site h of
// parity par, neighbours from the LDS half field sh of the other parity,
// written to acc
template <typename T, int B>
__device__ __forceinline__ void hop_reg_rt(int mu, int par, const typename C2<T>::type *sh, const HopRegs<T> &R,
                                           spinor<T> &acc)
{
    constexpr int Vh = Cube<B>::Vh;
    switch (mu) {
    case 0: hop_dir_reg<T, 0>(sh, Vh, R.f[par], R.b[par], R.nf[par], R.nb[par], acc); break;
    case 1: hop_dir_reg<T, 1>(sh, Vh, R.f[par], R.b[par], R.nf[par], R.nb[par], acc); break;
    case 2: hop_dir_reg<T, 2>(sh, Vh, R.f[par], R.b[par], R.nf[par], R.nb[par], acc); break;
    default: hop_dir_reg<T, 3>(sh, Vh, R.f[par], R.b[par], R.nf[par], R.nb[par], acc); break;
    }
}

// partial sum of thread (mu, h) into LDS
template <typename T, int Vh>
__device__ __forceinline__ void put_part(typename C2<T>::type *part, int mu, int h, const spinor<T> &acc)
{
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) st<T>(part, (mu * 12 + 3 * sp + a) * Vh + h, acc.s[sp].c[a]);
}

// spin q of site h summed over the four partial sums
template <typename T, int Vh>
__device__ __forceinline__ void sum_part(const typename C2<T>::type *part, int q, int h, cx<T> v[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int c = 3 * q + a;
        v[a] = (ld<T>(part, c * Vh + h) + ld<T>(part, (12 + c) * Vh + h)) +
               (ld<T>(part, (24 + c) * Vh + h) + ld<T>(part, (36 + c) * Vh + h));
    }
}

//
// ST = 1: FP16 storage (SAP / block solves with FP16 inner): links are the
// FP16 two-row copy ([slot][mu][6][Vb]), src and dst are FP16 fields with a
// power-of-two scale per system and block; the output's scale is the block
// maximum of the new values (an LDS reduction: the workgroup owns the block).
//
// OCC: minimum waves per SIMD the compiler must allow (1: no constraint).
// Block solves of large lattices (thousands of blocks per launch) run faster
// at 4 (two blocks per CU) despite a few spilled registers.
template <typename T, int MODE, int B, int ST, int OCC = 1>
__global__ __launch_bounds__(4 * Cube<B>::Vh) __attribute__((amdgpu_waves_per_eu(OCC))) void k_block_mr_dir(Geo g, const int32_t *__restrict__ active,
                                                                  const void *const *__restrict__ Utab,
                                                                  const double *__restrict__ kap, long n,
                                                                  const int32_t *__restrict__ sched,
                                                                  const void *__restrict__ src_v,
                                                                  const float *__restrict__ src_s,
                                                                  void *__restrict__ dst_v, float *__restrict__ dst_s,
                                                                  T kappa, int nmr)
{
    typedef Cube<B> CB;
    typedef typename C2<T>::type T2;
    constexpr int Vb = CB::Vb, Vh = CB::Vh, NT = 4 * Vh;
    static_assert(Vh % 64 == 0, "a wavefront covers sites of one direction / spin only");
    static_assert(ST == 0 || sizeof(T) == 4, "FP16 storage is computed in FP32");
    __shared__ DirLds<T, B> S;
    const int m = blockIdx.y;
    if (active && !active[m]) return;
    if (kap) kappa = (T)kap[m];
    const T2 *__restrict__ src = static_cast<const T2 *>(src_v) + m * n;
    T2 *__restrict__ dst = static_cast<T2 *>(dst_v) + m * n;
    const h2 *__restrict__ src16 = static_cast<const h2 *>(src_v) + m * n;
    h2 *__restrict__ dst16 = static_cast<h2 *>(dst_v) + m * n;
    const float *__restrict__ dsc = ST ? dst_s + (long)m * g.nblk : nullptr;
    const int slot = sched[blockIdx.x];
    const float s_src = ST ? src_s[(long)m * g.nblk + slot] : 1.f, s_dst = ST ? dsc[slot] : 1.f;
    // loads of the block's own src / dst values (element index i of the system)
    auto ld_src = [&](long i) -> cx<T> {
        if constexpr (ST) return ldh(as_global(src16), i, s_src);
        else return ld<T>(src, i);
    };
    auto ld_dst = [&](long i) -> cx<T> {
        if constexpr (ST) return ldh(as_global((const h2 *)dst16), i, s_dst);
        else return ld<T>(dst, i);
    };
    const int tid = threadIdx.x;
    const int w4 = __builtin_amdgcn_readfirstlane(tid / Vh);  // mu in hop phases, spin q in vector phases
    const int h = tid % Vh;
    int xe[4], xo[4];
    CB::coords(h, xe);
    CB::coords(Vh + h, xo);
    const long be = (long)slot * 12 * Vb + h, bo = be + Vh;

    // the links of this thread's hops, in registers
    HopRegs<T> R;
    switch (w4) {
    case 0: load_hop_regs<T, B, 0, ST>(Utab[m], slot, h, xe, xo, R); break;
    case 1: load_hop_regs<T, B, 1, ST>(Utab[m], slot, h, xe, xo, R); break;
    case 2: load_hop_regs<T, B, 2, ST>(Utab[m], slot, h, xe, xo, R); break;
    default: load_hop_regs<T, B, 3, ST>(Utab[m], slot, h, xe, xo, R); break;
    }

    // residual of the block system, spin q of even site h (re) and odd site h (ro)
    cx<T> re[3], ro[3], v[3];
    if (MODE == 0) {
        int nbr[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) nbr[k] = g.slot_nbr[slot * 8 + k];
        int nmu = g.slot_blk[slot];
        for (int d = 0; d < w4; ++d) nmu /= g.NB[d];
        nmu %= g.NB[w4];
#pragma unroll
        for (int par = 0; par < 2; ++par) {
            const int *x = par ? xo : xe;
            const int l = par * Vh + h;
            // boundary sign of wrapping links (the third row is rebuilt)
            T wf = 1, wb = 1;
            if (g.bc[w4] < 0) {
                if (nmu == g.NB[w4] - 1 && x[w4] == B - 1) wf = -1;
                if (nmu == 0 && x[w4] == 0) wb = -1;
            }
            spinor<T> acc;
            zero(acc);
            if constexpr (ST) {
                const SpinorLdH<Vb> xin{as_global((const h2 *)dst16), dsc};
                const LinkLdH<Vb> lk{as_global(static_cast<const h2 *>(Utab[m]))};
                switch (w4) {
                case 0: hop_dir_ld<T, HOPS_ALL, B, 0, 0, 1>(xin, lk, slot, nbr, l, x, acc, wf, wb); break;
                case 1: hop_dir_ld<T, HOPS_ALL, B, 0, 1, 1>(xin, lk, slot, nbr, l, x, acc, wf, wb); break;
                case 2: hop_dir_ld<T, HOPS_ALL, B, 0, 2, 1>(xin, lk, slot, nbr, l, x, acc, wf, wb); break;
                default: hop_dir_ld<T, HOPS_ALL, B, 0, 3, 1>(xin, lk, slot, nbr, l, x, acc, wf, wb); break;
                }
            } else {
                const auto *Ug = as_global(static_cast<const T2 *>(Utab[m]));
                const auto *xg = as_global((const T2 *)dst);
                switch (w4) {
                case 0: hop_dir_cube<T, HOPS_ALL, B, 0, 0, 1>(Ug, xg, slot, nbr, l, x, 0, acc, wf, wb); break;
                case 1: hop_dir_cube<T, HOPS_ALL, B, 0, 1, 1>(Ug, xg, slot, nbr, l, x, 0, acc, wf, wb); break;
                case 2: hop_dir_cube<T, HOPS_ALL, B, 0, 2, 1>(Ug, xg, slot, nbr, l, x, 0, acc, wf, wb); break;
                default: hop_dir_cube<T, HOPS_ALL, B, 0, 3, 1>(Ug, xg, slot, nbr, l, x, 0, acc, wf, wb); break;
                }
            }
            put_part<T, Vh>(S.part, w4, h, acc);
            __syncthreads();
            sum_part<T, Vh>(S.part, w4, h, v);
            const long b = par ? bo : be;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const long i = b + (long)(3 * w4 + a) * Vb;
                const cx<T> r = ld_src(i) - ld_dst(i) + scale(kappa, v[a]);
                if (par) ro[a] = r;
                else re[a] = r;
            }
            __syncthreads();
        }
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            re[a] = ld_src(be + (long)(3 * w4 + a) * Vb);
            ro[a] = ld_src(bo + (long)(3 * w4 + a) * Vb);
        }
    }

    // rhs_e = r_e + kappa H_eo r_o
#pragma unroll
    for (int a = 0; a < 3; ++a) st<T>(S.sho, (3 * w4 + a) * Vh + h, ro[a]);
    __syncthreads();
    {
        spinor<T> acc;
        hop_reg_rt<T, B>(w4, 0, S.sho, R, acc);
        put_part<T, Vh>(S.part, w4, h, acc);
    }
    __syncthreads();
    cx<T> rho[3], del[3];
    sum_part<T, Vh>(S.part, w4, h, v);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        rho[a] = re[a] + scale(kappa, v[a]);
        del[a] = mk<T>(0, 0);
        st<T>(S.she, (3 * w4 + a) * Vh + h, rho[a]);
    }

    // MR steps on (1 - kappa^2 H_eo H_oe)
    const T k2 = kappa * kappa;
    for (int it = 0; it < nmr; ++it) {
        __syncthreads();
        {  // t_o = H_oe rho
            spinor<T> acc;
            hop_reg_rt<T, B>(w4, 1, S.she, R, acc);
            put_part<T, Vh>(S.part, w4, h, acc);
        }
        __syncthreads();
        sum_part<T, Vh>(S.part, w4, h, v);
#pragma unroll
        for (int a = 0; a < 3; ++a) st<T>(S.sho, (3 * w4 + a) * Vh + h, v[a]);
        __syncthreads();
        {  // H_eo t_o
            spinor<T> acc;
            hop_reg_rt<T, B>(w4, 0, S.sho, R, acc);
            put_part<T, Vh>(S.part, w4, h, acc);
        }
        __syncthreads();
        sum_part<T, Vh>(S.part, w4, h, v);
        T pr = 0, pi = 0, pp = 0;
        cx<T> p[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p[a] = rho[a] - scale(k2, v[a]);
            const cx<T> q = conjmul(p[a], rho[a]);
            pr += q.re;
            pi += q.im;
            pp += p[a].re * p[a].re + p[a].im * p[a].im;
        }
        pr = wave_total(pr);
        pi = wave_total(pi);
        pp = wave_total(pp);
        if ((tid & 63) == TOTAL_LANE<T>) {
            S.red[0][tid >> 6] = pr;
            S.red[1][tid >> 6] = pi;
            S.red[2][tid >> 6] = pp;
        }
        __syncthreads();
        if (tid == 0) {
            T sr = 0, si = 0, sq = 0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) {
                sr += S.red[0][w];
                si += S.red[1][w];
                sq += S.red[2][w];
            }
            S.alpha[0] = sq > 0 ? sr / sq : T(0);
            S.alpha[1] = sq > 0 ? si / sq : T(0);
        }
        __syncthreads();
        const cx<T> al = mk<T>(S.alpha[0], S.alpha[1]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            del[a] = del[a] + al * rho[a];
            rho[a] = rho[a] - al * p[a];
            st<T>(S.she, (3 * w4 + a) * Vh + h, rho[a]);
        }
    }

    // d_o = r_o + kappa H_oe d_e
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 3; ++a) st<T>(S.she, (3 * w4 + a) * Vh + h, del[a]);
    __syncthreads();
    {
        spinor<T> acc;
        hop_reg_rt<T, B>(w4, 1, S.she, R, acc);
        put_part<T, Vh>(S.part, w4, h, acc);
    }
    __syncthreads();
    sum_part<T, Vh>(S.part, w4, h, v);
    // new values of spin q at even site h (ye) and odd site h (yo): x + d, or d
    cx<T> ye[3], yo[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cx<T> dodd = ro[a] + scale(kappa, v[a]);
        const long ie = be + (long)(3 * w4 + a) * Vb, io = bo + (long)(3 * w4 + a) * Vb;
        // (MODE 0: this workgroup alone reads x of this block after its residual)
        ye[a] = MODE == 0 ? ld_dst(ie) + del[a] : del[a];
        yo[a] = MODE == 0 ? ld_dst(io) + dodd : dodd;
    }
    float inv = 1.f;
    if constexpr (ST) {  // block maximum -> power-of-two scale of the output
        float mx = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            mx = fmaxf(mx, fmaxf(fmaxf(fabsf(ye[a].re), fabsf(ye[a].im)), fmaxf(fabsf(yo[a].re), fabsf(yo[a].im))));
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_down(mx, off, 64));
        __syncthreads();  // S.red is free again
        if ((tid & 63) == 0) S.red[0][tid >> 6] = mx;
        __syncthreads();
        mx = S.red[0][0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) mx = fmaxf(mx, S.red[0][w]);
        const float sc = pow2_at_least(mx);
        inv = 1.f / sc;
        if (tid == 0) dst_s[(long)m * g.nblk + slot] = sc;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long ie = be + (long)(3 * w4 + a) * Vb, io = bo + (long)(3 * w4 + a) * Vb;
        if constexpr (ST) {
            dst16[ie] = to_h2(ye[a], inv);
            dst16[io] = to_h2(yo[a], inv);
        } else {
            st<T>(dst, ie, ye[a]);
            st<T>(dst, io, yo[a]);
        }
    }
}

// ---------------------------------------------------------------- FP16 hops
// The block-solve form (MODE 1, FP16 storage) of k_block_mr_dir with its hop
// phases in packed FP16 arithmetic: the LDS half fields and the partial sums
// hold FP16, the links sit in registers as FP16 (third rows rebuilt once),
// and each hop's spin projection, link times half spinor and accumulation
// run on (re, im) pairs with v_pk_* instructions; the MR vectors, the
// inner products and the step coefficients stay FP32.  The FP32 kernel was
// bound by its vector instruction issue (about 585 per wavefront and MR
// step); this form halves the hop arithmetic and the LDS bytes.  The MR
// iterate goes to LDS times a power-of-two factor sigma that keeps its RMS
// near 1 (from |rho|^2 of the previous step, which MR never increases), so
// the FP16 values neither overflow nor lose their small components; the
// operator's output is divided by sigma again in FP32.

// the FP16 links and LDS neighbour indices of thread (MU, h), as HopRegs
struct HopRegs16 {
    h2 f[2][9], b[2][9];
    int nf[2], nb[2];
};

// rows 0, 1 of the FP16 two-row link at site l, direction MU, and the third
// row conj(row0 x row1) (in-block links never carry a boundary sign)
template <int MU>
__device__ __forceinline__ void load_link16(const h2 *U16, int slot, int l, h2 u[9])
{
    constexpr int Vb = Cube<4>::Vb;
    const auto *Ug = as_global(U16);
    const long base = (long)slot * 4 * 6 * Vb + (long)MU * 6 * Vb + l;
#pragma unroll
    for (int e = 0; e < 6; ++e) u[e] = Ug[base + (long)e * Vb];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int a = (c + 1) % 3, b = (c + 2) % 3;
        const h2 v = hcfma(u[b], -u[3 + a], hcfma(u[a], u[3 + b], (h2){0, 0}));
        u[6 + c] = (h2){v.x, -v.y};
    }
}

template <int MU>
__device__ __forceinline__ void load_hop_regs16(const h2 *U16, int slot, int h, const int xe[4], const int xo[4],
                                                HopRegs16 &R)
{
    typedef Cube<4> CB;
#pragma unroll
    for (int par = 0; par < 2; ++par) {
        const int *x = par ? xo : xe;
        const int l = par * CB::Vh + h;
        const int off = par ? 0 : CB::Vh;  // the neighbours have the other parity
        int y[4] = {x[0], x[1], x[2], x[3]};
        // a hop that leaves the block keeps LDS index 0 and a zero link: it
        // adds exact zeros, so every lane takes both hops without a branch
        R.nf[par] = R.nb[par] = 0;
        if (x[MU] + 1 < 4) {
            y[MU] = x[MU] + 1;
            R.nf[par] = CB::index(y) - off;
            load_link16<MU>(U16, slot, l, R.f[par]);
        } else {
#pragma unroll
            for (int e = 0; e < 9; ++e) R.f[par][e] = (h2){0, 0};
        }
        if (x[MU] > 0) {
            y[MU] = x[MU] - 1;
            const int nl = CB::index(y);
            R.nb[par] = nl - off;
            load_link16<MU>(U16, slot, nl, R.b[par]);
        } else {
#pragma unroll
            for (int e = 0; e < 9; ++e) R.b[par][e] = (h2){0, 0};
        }
    }
}

// the in-block hops of direction MU at one output site: neighbours from the
// FP16 LDS half field sh ([12][Vh]), links from registers; the sum of the two
// hops into acc (12 FP16 complex, component 3 spin + colour).  Both hops are
// always taken (one that leaves the block has a zero link), so acc starts
// from the forward hop's values and no lane branches.
template <int MU>
__device__ __forceinline__ void hop_dir16(const h2 *sh, const h2 *uf, const h2 *ub, int nf, int nb, h2 acc[12])
{
    constexpr int Vh = Cube<4>::Vh;
    constexpr int i0 = MU <= 1 ? 1 : 0, i1 = MU <= 1 ? 0 : 1;  // A psi_dn takes (d_i0, d_i1)
    constexpr int m0 = MU == 0 ? 3 : MU == 1 ? 1 : MU == 2 ? 3 : 0, m1 = MU == 0 ? 3 : MU == 1 ? 0 : MU == 2 ? 2 : 0;
    constexpr int r0 = MU == 0 ? 2 : MU == 1 ? 0 : MU == 2 ? 2 : 0, r1 = MU == 0 ? 2 : MU == 1 ? 1 : MU == 2 ? 3 : 0;
    constexpr int j0 = MU <= 1 ? 1 : 0, j1 = MU <= 1 ? 0 : 1;  // A^+ h takes (c_j0, c_j1)
    h2 lo[6];  // spins 2, 3 of the forward hop before their sign
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        const bool fwd = dir == 0;
        const int nl = fwd ? nf : nb;
        h2 p[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = sh[c * Vh + nl];
        h2 hh[2][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const h2 o0 = hmap(p[6 + 3 * i0 + a], m0), o1 = hmap(p[6 + 3 * i1 + a], m1);
            hh[0][a] = fwd ? p[a] - o0 : p[a] + o0;
            hh[1][a] = fwd ? p[3 + a] - o1 : p[3 + a] + o1;
        }
        const h2 *u = fwd ? uf : ub;
        h2 c[2][3];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                h2 r = (h2){0, 0};
#pragma unroll
                for (int b = 0; b < 3; ++b) r = fwd ? hcfma(u[3 * a + b], hh[s][b], r) : hcjfma(u[3 * b + a], hh[s][b], r);
                c[s][a] = r;
            }
        // spins 2, 3: -A^+ c of the forward hop, +A^+ c of the backward one
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const h2 d0 = hmap(c[j0][a], r0), d1 = hmap(c[j1][a], r1);
            if (fwd) {
                acc[a] = c[0][a];
                acc[3 + a] = c[1][a];
                lo[a] = d0;
                lo[3 + a] = d1;
            } else {
                acc[a] = acc[a] + c[0][a];
                acc[3 + a] = acc[3 + a] + c[1][a];
                acc[6 + a] = d0 - lo[a];
                acc[9 + a] = d1 - lo[3 + a];
            }
        }
    }
}

// hop phase of thread (w4, h) into the FP16 partial sums
__device__ __forceinline__ void hop_phase16(int w4, int par, int h, const h2 *sh, const HopRegs16 &R, h2 *part)
{
    constexpr int Vh = Cube<4>::Vh;
    h2 acc[12];
    switch (w4) {
    case 0: hop_dir16<0>(sh, R.f[par], R.b[par], R.nf[par], R.nb[par], acc); break;
    case 1: hop_dir16<1>(sh, R.f[par], R.b[par], R.nf[par], R.nb[par], acc); break;
    case 2: hop_dir16<2>(sh, R.f[par], R.b[par], R.nf[par], R.nb[par], acc); break;
    default: hop_dir16<3>(sh, R.f[par], R.b[par], R.nf[par], R.nb[par], acc); break;
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) part[(w4 * 12 + c) * Vh + h] = acc[c];
}
// spin q of site h summed over the four FP16 partial sums, in FP32: each
// term enters through a mixed-precision dot product with (1, 0) or (0, 1),
// the exact value of its FP16 part added to the FP32 sum (one instruction
// instead of a conversion and an add)
__device__ __forceinline__ void sum_part16(const h2 *part, int q, int h, cx<float> v[3])
{
    constexpr int Vh = Cube<4>::Vh;
    const h2 pick_re = {(_Float16)1, (_Float16)0}, pick_im = {(_Float16)0, (_Float16)1};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int c = 3 * q + a;
        const h2 t0 = part[c * Vh + h];
        float re = (float)t0.x, im = (float)t0.y;
#pragma unroll
        for (int d = 1; d < 4; ++d) {
            const h2 t = part[(d * 12 + c) * Vh + h];
            re = __builtin_amdgcn_fdot2(t, pick_re, re, false);
            im = __builtin_amdgcn_fdot2(t, pick_im, im, false);
        }
        v[a] = mk<float>(re, im);
    }
}
__device__ __forceinline__ h2 to16(cx<float> a, float f) { return (h2){(_Float16)(a.re * f), (_Float16)(a.im * f)}; }
// the power of two 2^-e that brings a block's RMS component, sqrt(st / 1536)
// over the 12 x 128 components of a block half, to about 1, and 2^e (both
// exact)
__device__ __forceinline__ void rms_scale16(float st, float *out)
{
    constexpr float LOG2_1536 = 10.5849625007f;
    const int e = st > 0.f ? (int)rintf(0.5f * (log2f(st) - LOG2_1536)) : 0;
    out[0] = ldexpf(1.f, -e);
    out[1] = ldexpf(1.f, e);
}

// rows 3P, 3P + 1, 3P + 2 (spin 2 chi + P, colours 0-2) of one packed
// hermitian 6 x 6 clover block held in LDS as FP16 (the layout of clover.h,
// entries Vh apart) times the chirality's 6-vector x, in FP32
template <int P>
__device__ __forceinline__ void clov_rows16(const _Float16 *M, const cx<float> x[6], cx<float> y[3])
{
    constexpr int Vh = Cube<4>::Vh;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int i = 3 * P + r;
        cx<float> acc = scale((float)M[i * Vh], x[i]);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            if (j == i) continue;
            const int k = j > i ? herm_k(i, j) : herm_k(j, i);
            const float re = (float)M[(6 + 2 * k) * Vh], im = (float)M[(7 + 2 * k) * Vh];
            acc = acc + mk<float>(re, j > i ? im : -im) * x[j];  // M_ij, or conj(M_ji) below the diagonal
        }
        y[r] = acc;
    }
}
__device__ __forceinline__ void clov_rows16(int p, const _Float16 *M, const cx<float> x[6], cx<float> y[3])
{
    if (p)
        clov_rows16<1>(M, x, y);
    else
        clov_rows16<0>(M, x, y);
}

// CL = 1: with the clover term (ctab: FP32 clover fields per system, A then
// A^-1, clover.h).  The block system is then D_b = A - kappa H_in and the MR
// runs on A_ee - kappa^2 H_eo A_oo^-1 H_oe with rhs_e = r_e + kappa H_eo
// A_oo^-1 r_o and d_o = A_oo^-1 (r_o + kappa H_oe d_e).  The blocks that
// enter, A_ee - 1 of the even sites and A_oo^-1 of the odd ones, are read
// once per launch into LDS as FP16 (36 KB beside the 37 KB of the fields
// and partial sums: still two blocks per CU).  A thread owns one spin, so
// where a 6 x 6 block acts it sums the partial sums of both spins of its
// chirality (after a hop phase) or reads them from the LDS copy of the
// iterate (A_ee - 1 acting on it, in FP16 like the hops).
template <int OCC, int CL>
__global__ __launch_bounds__(4 * Cube<4>::Vh) __attribute__((amdgpu_waves_per_eu(OCC))) void k_block_mr_h16(
    Geo g, const int32_t *__restrict__ active, const void *const *__restrict__ Utab, const double *__restrict__ kap,
    const float *const *__restrict__ ctab, long n, const int32_t *__restrict__ sched,
    const void *__restrict__ src_v, const float *__restrict__ src_s, void *__restrict__ dst_v,
    float *__restrict__ dst_s, float kappa, int nmr)
{
    typedef Cube<4> CB;
    constexpr int Vb = CB::Vb, Vh = CB::Vh, NT = 4 * Vh;
    __shared__ h2 she[12 * Vh];
    __shared__ h2 sho[12 * Vh];
    __shared__ h2 part[4 * 12 * Vh];
    __shared__ float red[4][NT / 64];
    __shared__ float coef[4];
    // [parity][chirality][36][Vh]: A_ee - 1 (even sites), A_oo^-1 (odd)
    __shared__ _Float16 clv[CL ? 2 * 72 * Vh : 1];
    const int m = blockIdx.y;
    if (active && !active[m]) return;
    if (kap) kappa = (float)kap[m];
    const h2 *__restrict__ src16 = static_cast<const h2 *>(src_v) + m * n;
    h2 *__restrict__ dst16 = static_cast<h2 *>(dst_v) + m * n;
    const int slot = sched[blockIdx.x];
    // every vector below is in units of the right-hand side's block scale
    const float s_src = src_s[(long)m * g.nblk + slot];
    const int tid = threadIdx.x;
    const int w4 = __builtin_amdgcn_readfirstlane(tid / Vh);  // mu in hop phases, spin q in vector phases
    const int h = tid % Vh;
    int xe[4], xo[4];
    CB::coords(h, xe);
    CB::coords(Vh + h, xo);
    const long be = (long)slot * 12 * Vb + h, bo = be + Vh;

    HopRegs16 R;
    const h2 *U16 = static_cast<const h2 *>(Utab[m]);
    switch (w4) {
    case 0: load_hop_regs16<0>(U16, slot, h, xe, xo, R); break;
    case 1: load_hop_regs16<1>(U16, slot, h, xe, xo, R); break;
    case 2: load_hop_regs16<2>(U16, slot, h, xe, xo, R); break;
    default: load_hop_regs16<3>(U16, slot, h, xe, xo, R); break;
    }
    // the spin's chirality and its place in the chirality (clover term)
    const int chi = w4 >> 1, pq = w4 & 1;
    const int tee = chi * 36 * Vh + h, aoi = (72 + chi * 36) * Vh + h;  // clv offsets of site h
    if constexpr (CL) {
        // flat index f = (chirality * 36 + entry) * Vb + site of the block,
        // even sites from A (diagonal minus 1), odd ones from A^-1
        const auto *cb = as_global(ctab[m]);
        const long base = (long)slot * 72 * Vb, inv = 72L * g.V;
        for (int f = tid; f < 72 * Vb; f += NT) {
            const int l = f % Vb, ck = f / Vb, par = l >= Vh ? 1 : 0;
            float val = cb[base + f + (par ? inv : 0)];
            if (!par && ck % 36 < 6) val -= 1.f;
            clv[(par * 72 + ck) * Vh + l - par * Vh] = (_Float16)val;
        }
    }
    // the right-hand side as stored (|value| <= 1): spin q of site h
    cx<float> re[3], ro[3], v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const h2 x = src16[be + (long)(3 * w4 + a) * Vb], y = src16[bo + (long)(3 * w4 + a) * Vb];
        re[a] = mk<float>((float)x.x, (float)x.y);
        ro[a] = mk<float>((float)y.x, (float)y.y);
        sho[(3 * w4 + a) * Vh + h] = y;
    }
    __syncthreads();
    if constexpr (CL) {  // sho <- A_oo^-1 r_o
        cx<float> x6[6], y[3];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const h2 t = sho[(6 * chi + c) * Vh + h];
            x6[c] = mk<float>((float)t.x, (float)t.y);
        }
        clov_rows16(pq, clv + aoi, x6, y);
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 3; ++a) sho[(3 * w4 + a) * Vh + h] = to16(y[a], 1.f);
        __syncthreads();
    }
    // rhs_e = r_e + kappa H_eo r_o (H_eo A_oo^-1 r_o with the clover term)
    hop_phase16(w4, 0, h, sho, R, part);
    __syncthreads();
    cx<float> rho[3], del[3];
    sum_part16(part, w4, h, v);
    float rr = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        rho[a] = re[a] + scale(kappa, v[a]);
        del[a] = mk<float>(0, 0);
        rr += rho[a].re * rho[a].re + rho[a].im * rho[a].im;
    }
    // the first scale from |rho|^2 (coef[2]: a power of two, coef[3] its
    // inverse)
    rr = wave_total63(rr);
    if ((tid & 63) == 63) red[3][tid >> 6] = rr;
    __syncthreads();
    if (tid == 0) {
        float t = red[3][0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) t += red[3][w];
        rms_scale16(t, coef + 2);
    }
    __syncthreads();
    float sig = coef[2], isig = coef[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) she[(3 * w4 + a) * Vh + h] = to16(rho[a], sig);

    const float k2 = kappa * kappa;
    for (int it = 0; it < nmr; ++it) {
        __syncthreads();
        hop_phase16(w4, 1, h, she, R, part);  // t_o = sigma H_oe rho
        __syncthreads();
        if constexpr (CL) {  // t_o <- A_oo^-1 t_o
            cx<float> x6[6];
            sum_part16(part, 2 * chi, h, x6);
            sum_part16(part, 2 * chi + 1, h, x6 + 3);
            clov_rows16(pq, clv + aoi, x6, v);
        } else {
            sum_part16(part, w4, h, v);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) sho[(3 * w4 + a) * Vh + h] = to16(v[a], 1.f);
        __syncthreads();
        hop_phase16(w4, 0, h, sho, R, part);  // sigma H_eo H_oe rho
        __syncthreads();
        sum_part16(part, w4, h, v);
        cx<float> td[3];  // (A_ee - 1) rho, from the stored iterate
        if constexpr (CL) {
            cx<float> x6[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const h2 t = she[(6 * chi + c) * Vh + h];
                x6[c] = mk<float>((float)t.x * isig, (float)t.y * isig);
            }
            clov_rows16(pq, clv + tee, x6, td);
        }
        float pr = 0, pi = 0, pp = 0, r2 = 0;
        cx<float> p[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p[a] = rho[a] - scale(k2 * isig, v[a]);
            if constexpr (CL) p[a] = p[a] + td[a];
            const cx<float> q = conjmul(p[a], rho[a]);
            pr += q.re;
            pi += q.im;
            pp += p[a].re * p[a].re + p[a].im * p[a].im;
            r2 += rho[a].re * rho[a].re + rho[a].im * rho[a].im;
        }
        pr = wave_total63(pr);
        pi = wave_total63(pi);
        pp = wave_total63(pp);
        r2 = wave_total63(r2);
        if ((tid & 63) == 63) {
            red[0][tid >> 6] = pr;
            red[1][tid >> 6] = pi;
            red[2][tid >> 6] = pp;
            red[3][tid >> 6] = r2;
        }
        __syncthreads();
        if (tid == 0) {  // one lane: the step's coefficient and the next scale
            float sr = red[0][0], si = red[1][0], sq = red[2][0], st = red[3][0];
#pragma unroll
            for (int w = 1; w < NT / 64; ++w) {
                sr += red[0][w];
                si += red[1][w];
                sq += red[2][w];
                st += red[3][w];
            }
            coef[0] = sq > 0 ? __fdividef(sr, sq) : 0.f;
            coef[1] = sq > 0 ? __fdividef(si, sq) : 0.f;
            // |rho_new|^2 <= |rho|^2: the scale of the next stored iterate
            rms_scale16(st, coef + 2);
        }
        __syncthreads();
        const cx<float> al = mk<float>(coef[0], coef[1]);
        sig = coef[2];
        isig = coef[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            del[a] = del[a] + al * rho[a];
            rho[a] = rho[a] - al * p[a];
            she[(3 * w4 + a) * Vh + h] = to16(rho[a], sig);
        }
    }

    // d_o = r_o + kappa H_oe d_e, with d_e scaled to at most 1 in LDS
    float mx = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) mx = fmaxf(mx, fmaxf(fabsf(del[a].re), fabsf(del[a].im)));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_down(mx, off, 64));
    __syncthreads();  // the last step's LDS reads are done; red is free
    if ((tid & 63) == 0) red[0][tid >> 6] = mx;
    __syncthreads();
    mx = red[0][0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) mx = fmaxf(mx, red[0][w]);
    const float sd = pow2_at_least(mx), isd = 1.f / sd;
#pragma unroll
    for (int a = 0; a < 3; ++a) she[(3 * w4 + a) * Vh + h] = to16(del[a], isd);
    __syncthreads();
    hop_phase16(w4, 1, h, she, R, part);
    __syncthreads();
    sum_part16(part, w4, h, v);
    // the new values of spin q at even site h (ye) and odd site h (yo)
    cx<float> ye[3], yo[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) yo[a] = ro[a] + scale(kappa * sd, v[a]);
    if constexpr (CL) {  // yo <- A_oo^-1 yo, the chirality's other spin through LDS (FP32)
        float *wb = reinterpret_cast<float *>(part);
        __syncthreads();  // every lane has read the partial sums
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            wb[2 * ((3 * w4 + a) * Vh + h)] = yo[a].re;
            wb[2 * ((3 * w4 + a) * Vh + h) + 1] = yo[a].im;
        }
        __syncthreads();
        cx<float> x6[6];
#pragma unroll
        for (int c = 0; c < 6; ++c)
            x6[c] = mk<float>(wb[2 * ((6 * chi + c) * Vh + h)], wb[2 * ((6 * chi + c) * Vh + h) + 1]);
        clov_rows16(pq, clv + aoi, x6, yo);
    }
    float mo = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ye[a] = scale(s_src, del[a]);
        yo[a] = scale(s_src, yo[a]);
        mo = fmaxf(mo, fmaxf(fmaxf(fabsf(ye[a].re), fabsf(ye[a].im)), fmaxf(fabsf(yo[a].re), fabsf(yo[a].im))));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mo = fmaxf(mo, __shfl_down(mo, off, 64));
    __syncthreads();
    if ((tid & 63) == 0) red[0][tid >> 6] = mo;
    __syncthreads();
    mo = red[0][0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) mo = fmaxf(mo, red[0][w]);
    const float sc = pow2_at_least(mo), inv = 1.f / sc;
    if (tid == 0) dst_s[(long)m * g.nblk + slot] = sc;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dst16[be + (long)(3 * w4 + a) * Vb] = to_h2(ye[a], inv);
        dst16[bo + (long)(3 * w4 + a) * Vb] = to_h2(yo[a], inv);
    }
}

// block solves with at least this many workgroups (blocks x systems) use the
// four-waves-per-SIMD form: two blocks per CU, at the price of a few spills
constexpr long MR_OCC4_WORKGROUPS = 2048;
// the block-MR form of a block-solve launch of `wgs` workgroups (the
// context's wdr_mr_form choice, or the workgroup threshold)
inline bool two_per_cu(const Geo &g, long wgs)
{
    if (g.mr_form == WDR_MR_TWO_PER_CU) return true;
    if (g.mr_form == WDR_MR_ONE_PER_CU) return false;
    return wgs >= MR_OCC4_WORKGROUPS;
}

template <typename T, int MODE>
bool launch_mr_cube4(const Geo &g, const Sys &sy, Links<T> U, const T2<T> *src, T2<T> *dst, T kappa, int nmr,
                     int slot0, int nslots, hipStream_t s)
{
    // the LDS copy of the links holds two rows: SU(3) links only
    if (!U.su3 || g.B[0] != 4 || g.B[1] != 4 || g.B[2] != 4 || g.B[3] != 4) return false;
    const int si = sched_index(g, slot0, nslots);
    if (si < 0) return false;
    if constexpr (sizeof(T) == 4) {  // the FP64 partial sums would not fit in LDS next to the links
        const auto *tab = reinterpret_cast<const void *const *>(U.tab);
        if constexpr (MODE == 1) {
            if (two_per_cu(g, (long)nslots * sy.M)) {
                k_block_mr_dir<T, MODE, 4, 0, 4><<<dim3(nslots, sy.M), 4 * Cube<4>::Vh, 0, s>>>(
                    g, sy.active, tab, U.kap, sy.n, g.sched[si], src, nullptr, dst, nullptr, kappa, nmr);
                return true;
            }
        }
        k_block_mr_dir<T, MODE, 4, 0><<<dim3(nslots, sy.M), 4 * Cube<4>::Vh, 0, s>>>(
            g, sy.active, tab, U.kap, sy.n, g.sched[si], src, nullptr, dst, nullptr, kappa, nmr);
    } else
        k_block_mr_cube<T, MODE, 4><<<dim3(nslots, sy.M), 256, 0, s>>>(g, sy.active, U.tab, U.kap, sy.n, g.sched[si], src,
                                                                       dst, kappa, nmr);
    return true;
}

}  // namespace

template <typename T>
void launch_sap_colour(const Geo &g, const Sys &sy, Links<T> U, const T2<T> *eta, T2<T> *x, T kappa, int nmr,
                       int slot0, int nslots, hipStream_t s)
{
    if (nslots <= 0 || sy.M <= 0) return;
    if (U.ctab) {  // the clover term: the one-lane-per-site form
        k_block_mr<T, 0, 1><<<dim3(nslots, sy.M), g.Vb, 0, s>>>(g, sy.active, U.tab, U.ctab, U.kap, sy.n, eta, x,
                                                                kappa, nmr, slot0);
        return;
    }
    if (launch_mr_cube4<T, 0>(g, sy, U, eta, x, kappa, nmr, slot0, nslots, s)) return;
    k_block_mr<T, 0, 0><<<dim3(nslots, sy.M), g.Vb, 0, s>>>(g, sy.active, U.tab, nullptr, U.kap, sy.n, eta, x, kappa,
                                                            nmr, slot0);
}

template <typename T>
void launch_block_mr(const Geo &g, const Sys &sy, Links<T> U, const T2<T> *r, T2<T> *d, T kappa, int nmr, int slot0,
                     int nslots, hipStream_t s)
{
    if (nslots <= 0 || sy.M <= 0) return;
    if (U.ctab) {
        k_block_mr<T, 1, 1><<<dim3(nslots, sy.M), g.Vb, 0, s>>>(g, sy.active, U.tab, U.ctab, U.kap, sy.n, r, d, kappa,
                                                                nmr, slot0);
        return;
    }
    if (launch_mr_cube4<T, 1>(g, sy, U, r, d, kappa, nmr, slot0, nslots, s)) return;
    k_block_mr<T, 1, 0><<<dim3(nslots, sy.M), g.Vb, 0, s>>>(g, sy.active, U.tab, nullptr, U.kap, sy.n, r, d, kappa,
                                                            nmr, slot0);
}

bool launch_mr_h16(int mode, const Geo &g, const Sys &sy, Links16 U, H16c src, H16 dst, float kappa, int nmr,
                   int slot0, int nslots, hipStream_t s, const float *const *ctab)
{
    if (nslots <= 0 || sy.M <= 0) return true;
    if (!U.tab || g.B[0] != 4 || g.B[1] != 4 || g.B[2] != 4 || g.B[3] != 4) return false;
    if (mode == 0 && ctab) return false;  // the FP16 Schwarz sweep has no clover form
    const int si = sched_index(g, slot0, nslots);
    if (si < 0) return false;
    const dim3 grid(nslots, sy.M);
    const auto *tab = reinterpret_cast<const void *const *>(U.tab);
    const bool two = two_per_cu(g, (long)nslots * sy.M);
#define WDR_MR16(OCC, CL)                                                                                    \
    k_block_mr_h16<OCC, CL><<<grid, 4 * Cube<4>::Vh, 0, s>>>(g, sy.active, tab, U.kap, ctab, sy.n, g.sched[si], \
                                                             src.v, src.s, dst.v, dst.s, kappa, nmr)
    if (mode == 0)
        k_block_mr_dir<float, 0, 4, 1><<<grid, 4 * Cube<4>::Vh, 0, s>>>(g, sy.active, tab, U.kap, sy.n, g.sched[si],
                                                                       src.v, src.s, dst.v, dst.s, kappa, nmr);
    else if (ctab && two)
        WDR_MR16(4, 1);
    else if (ctab)
        WDR_MR16(1, 1);
    else if (two)
        WDR_MR16(4, 0);
    else
        WDR_MR16(1, 0);
#undef WDR_MR16
    return true;
}

#define INST(T)                                                                                                  \
    template void launch_sap_colour<T>(const Geo &, const Sys &, Links<T>, const T2<T> *, T2<T> *, T, int, int,   \
                                       int, hipStream_t);                                                        \
    template void launch_block_mr<T>(const Geo &, const Sys &, Links<T>, const T2<T> *, T2<T> *, T, int, int, int, \
                                     hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace wdr
