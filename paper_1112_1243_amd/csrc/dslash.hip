// Wilson-Dirac stencil for gfx950 (paper Sec. 5: plain Wilson-Dirac
// operator; Sec. 3: Dirichlet block operators and block-interaction hops).
//
// Hops are spin-projected: only the 2-spin half spinor is multiplied by the
// link, and the lower two spins are reconstructed from it.
//
// 4^4 blocks (every workload here): k_dslash_blk for D and D_b on SU(3)
// fields (block input staged in LDS, one lane per site); k_dslash_dir for
// the rest (even-odd halves, cross-boundary hops, gamma_5-conjugated forms,
// general links), one wavefront per direction over 64 sites of a block,
// partial sums combined in LDS.  Both read two rows per SU(3) link and
// rebuild the third.  With a clover term the diagonal term is A times the
// diagonal input, or the whole result is multiplied by A^-1 (clover.h), in
// the same launch.  Other block
// shapes: k_dslash, one lane per site and 256 consecutive sites of one block
// per workgroup.  In both, a wavefront reads each spinor / link component of
// 64 consecutive sites as one contiguous 512 B (FP32) or 1 KiB (FP64) run.
#include "blk_stencil.h"

namespace wdr {
namespace {

using namespace dev;

// loader that applies gamma_5 (flip the sign of spins 2, 3) when dag is set
template <typename T> struct G5Loader {
    const typename C2<T>::type *f;
    int Vb, dag;
    __device__ __forceinline__ void operator()(int ns, int nl, spinor<T> &p) const
    {
        GlobalLoader<T>{f, Vb}(ns, nl, p);
        if (dag) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                p.s[2].c[a] = neg(p.s[2].c[a]);
                p.s[3].c[a] = neg(p.s[3].c[a]);
            }
        }
    }
};

template <typename T, int HOPS, int CL>
__global__ __launch_bounds__(256) void k_dslash(Geo g, const int32_t *__restrict__ active,
                                                const int32_t *__restrict__ list, UTab<T> Utab,
                                                const double *__restrict__ kap, int kneg,
                                                const T *const *__restrict__ ctab, long n,
                                                int par, int dag, const typename C2<T>::type *__restrict__ in,
                                                const typename C2<T>::type *__restrict__ diag,
                                                typename C2<T>::type *__restrict__ out, T kappa, int slot0)
{
    const int m = sys_at(list, blockIdx.z);
    if (active && !active[m]) return;
    if (kap) kappa = kneg ? -(T)kap[m] : (T)kap[m];
    const int Vb = g.Vb;
    const int nloc = par < 0 ? Vb : g.Vh;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nloc) return;
    const int l = (par > 0 ? g.Vh : 0) + i;
    const int slot = slot0 + blockIdx.y;
    const typename C2<T>::type *__restrict__ U = Utab[m];
    in += m * n;
    out += m * n;
    if (diag) diag += m * n;
    int x[4];
    local_coords(g, l, x);
    spinor<T> acc;
    hop_sum<T, HOPS>(g, U, slot, l, x, G5Loader<T>{in, Vb, dag}, acc);

    const long base = (long)slot * 12 * Vb + l;
    if (CL) {
        cx<T> v[12], dg[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            v[c] = scale(-kappa, acc.s[c / 3].c[c % 3]);
            if (dag && c >= 6) v[c] = neg(v[c]);
            dg[c] = diag ? ld<T>(diag, base + (long)c * Vb) : mk<T>(0, 0);
        }
        clov_site<T, CL>(ctab[m], (long)g.V, slot, Vb, l, dg, v);
#pragma unroll
        for (int c = 0; c < 12; ++c) st<T>(out, base + (long)c * Vb, v[c]);
        return;
    }
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<T> v = scale(-kappa, acc.s[sp].c[a]);
            if (dag && sp >= 2) v = neg(v);
            if (diag) v = v + ld<T>(diag, base + (long)(3 * sp + a) * Vb);
            st<T>(out, base + (long)(3 * sp + a) * Vb, v);
        }
}

// ---------------------------------------------------------------- B^4 blocks
// Direction-parallel stencil for B^4 blocks.  A workgroup takes 64 sites of
// one block (grid.x = blocks x chunks of 64 sites) with four wavefronts:
// wavefront w computes the two hops of direction mu = w for all 64 sites
// (mu is uniform per wavefront, so its spin projection is specialised at
// compile time) and issues the loads of both hops in one round trip.  The
// four partial sums meet in LDS; wavefront w then adds spin w of the diagonal
// term and writes spin w of the result (contiguous over the 64 sites).  With
// the clover term wavefront w forms both spins of its chirality and keeps
// the rows of spin w of the block product.
template <typename T, int HOPS, int B, int DAG, int R2, int CL>
__global__ __launch_bounds__(256) void k_dslash_dir(Geo g, const int32_t *__restrict__ active,
                                                    const int32_t *__restrict__ list, UTab<T> Utab,
                                                    const double *__restrict__ kap, int kneg,
                                                    const T *const *__restrict__ ctab, long n,
                                                    const int32_t *__restrict__ sched, int par, int chunks,
                                                    int xcd8, const T2<T> *__restrict__ in,
                                                    const T2<T> *__restrict__ diag, T2<T> *__restrict__ out, T kappa)
{
    typedef Cube<B> CB;
    constexpr int Vb = CB::Vb;
    __shared__ T2<T> part[4][12][64];  // [mu][colour-spin component][site]
    const int m = sys_at(list, blockIdx.y);
    if (active && !active[m]) return;
    if (kap) kappa = kneg ? -(T)kap[m] : (T)kap[m];
    // workgroup i runs on XCD i % 8; with a slot count divisible by 8 all
    // chunks of a block go to the XCD the schedule gives that block
    int bi, chunk;
    if (xcd8) {
        const int t = blockIdx.x >> 3;
        bi = (t / chunks) * 8 + (blockIdx.x & 7);
        chunk = t % chunks;
    } else {
        bi = blockIdx.x / chunks;
        chunk = blockIdx.x % chunks;
    }
    const int slot = sched[bi];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int mu = __builtin_amdgcn_readfirstlane(w);
    const int l = (par > 0 ? CB::Vh : 0) + chunk * 64 + lane;
    const auto *Ug = as_global(Utab[m]);
    const auto *ing = as_global(in + m * n);
    int x[4];
    CB::coords(l, x);
    int nbr[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) nbr[k] = g.slot_nbr[slot * 8 + k];
    // spin mu of the diagonal term (with the clover term both spins of its
    // chirality), issued early
    constexpr int ND = CL ? 6 : 3;
    const int chi = mu >> 1;
    cx<T> dg[ND];
#pragma unroll
    for (int a = 0; a < ND; ++a) dg[a] = mk<T>(0, 0);
    const long obase = m * n + (long)slot * 12 * Vb + l;
    if (diag) {
#pragma unroll
        for (int a = 0; a < ND; ++a) dg[a] = ld<T>(diag, obase + (long)((CL ? 6 * chi : 3 * mu) + a) * Vb);
    }
    // boundary sign of the forward and backward links of this site when they
    // wrap around the lattice (only needed to rebuild a third row)
    T wf = 1, wb = 1;
    if (R2 && g.bc[mu] < 0) {
        int bl = g.slot_blk[slot];
        for (int d = 0; d < mu; ++d) bl /= g.NB[d];
        const int nmu = bl % g.NB[mu];
        if (nmu == g.NB[mu] - 1 && x[mu] == B - 1) wf = -1;
        if (nmu == 0 && x[mu] == 0) wb = -1;
    }
    spinor<T> acc;
    zero(acc);
    switch (mu) {
    case 0: hop_dir_cube<T, HOPS, B, DAG, 0, R2>(Ug, ing, slot, nbr, l, x, 0, acc, wf, wb); break;
    case 1: hop_dir_cube<T, HOPS, B, DAG, 1, R2>(Ug, ing, slot, nbr, l, x, 0, acc, wf, wb); break;
    case 2: hop_dir_cube<T, HOPS, B, DAG, 2, R2>(Ug, ing, slot, nbr, l, x, 0, acc, wf, wb); break;
    default: hop_dir_cube<T, HOPS, B, DAG, 3, R2>(Ug, ing, slot, nbr, l, x, 0, acc, wf, wb); break;
    }
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) st<T>(&part[w][0][0], (3 * sp + a) * 64 + lane, acc.s[sp].c[a]);
    __syncthreads();
    if (CL) {
        // both spins of chirality chi over the four directions, the block
        // product, and the three rows of spin mu
        cx<T> v[6], x[6], y[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const int c = 6 * chi + i;
            cx<T> t = ld<T>(&part[0][0][0], c * 64 + lane);
#pragma unroll
            for (int d = 1; d < 4; ++d) t = t + ld<T>(&part[d][0][0], c * 64 + lane);
            t = scale(-kappa, t);
            v[i] = DAG && chi ? neg(t) : t;
            x[i] = CL == CLOV_DIAG ? dg[i % ND] : dg[i % ND] + v[i];
        }
        clov_mul6<T>(clov_at<T>(ctab[m], (long)g.V, CL == CLOV_INV, slot, chi, Vb, l), Vb, x, y);
        const bool upper = mu & 1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const cx<T> yo = upper ? y[3 + a] : y[a], vo = upper ? v[3 + a] : v[a];
            st_nt<T>(out, obase + (long)(3 * mu + a) * Vb, CL == CLOV_DIAG ? yo + vo : yo);
        }
        return;
    }
    // wavefront w sums spin w over the four directions
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int c = 3 * mu + a;
        cx<T> v = ld<T>(&part[0][0][0], c * 64 + lane);
#pragma unroll
        for (int d = 1; d < 4; ++d) v = v + ld<T>(&part[d][0][0], c * 64 + lane);
        v = scale(-kappa, v);
        if (DAG && mu >= 2) v = neg(v);
        st_nt<T>(out, obase + (long)c * Vb, v + dg[a % ND]);
    }
}

// Block-staged stencil for B^4 blocks (full-lattice operator D or the
// Dirichlet block operator D_b, diagonal term = the input): one workgroup per
// block and one lane per site.  The block's input spinor is read once into
// LDS; in-block neighbours come from there, only the neighbours across the
// block faces from global memory; links (two rows, third rebuilt) from
// global memory.  Against k_dslash_dir this cuts the vector-memory
// instructions per site (each in-block spinor is read once instead of once
// per neighbour), which bound that kernel.
//
// RES: write the residual b - out instead of out (the residual of a block
// solve, r = b - D_b x, in one pass).  CL = CLOV_DIAG: the diagonal term is
// A times the staged input.
template <typename T, int B, int HOPS, int RES = 0, int CL = CLOV_NONE>
__global__ __launch_bounds__(Cube<B>::Vb) void k_dslash_blk(Geo g, const int32_t *__restrict__ active,
                                                           const int32_t *__restrict__ list, UTab<T> Utab,
                                                           const double *__restrict__ kap, int kneg,
                                                           const T *const *__restrict__ ctab, long n,
                                                           const int32_t *__restrict__ sched,
                                                           const T2<T> *__restrict__ in, const T2<T> *__restrict__ b,
                                                           T2<T> *__restrict__ out, T kappa)
{
    typedef Cube<B> CB;
    constexpr int Vb = CB::Vb;
    __shared__ T2<T> sh[12][Vb];  // the block's input, component-major
    const int m = sys_at(list, blockIdx.y);
    if (active && !active[m]) return;
    if (kap) kappa = kneg ? -(T)kap[m] : (T)kap[m];
    const int slot = sched[blockIdx.x];
    const int l = threadIdx.x;
    const auto *Ug = as_global(Utab[m]);
    const auto *ing = as_global(in + m * n);
    const long base = (long)slot * 12 * Vb + l;
#pragma unroll
    for (int c = 0; c < 12; ++c) st<T>(&sh[c][0], l, ldg<T>(ing, base + c * Vb));
    int x[4];
    CB::coords(l, x);
    int nbr[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) nbr[k] = g.slot_nbr[slot * 8 + k];
    const int bl = g.slot_blk[slot];
    __syncthreads();
    spinor<T> acc;
    zero(acc);
    // directions one at a time (the loop stays rolled; `pin`, a zero the
    // compiler cannot see through, keeps each direction's loads inside it)
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        int pin = 0;
        asm volatile("" : "+s"(pin));
        // boundary sign of this site's links that wrap around the lattice
        T wf = 1, wb = 1;
        if (HOPS == HOPS_ALL && g.bc[mu] < 0) {
            int b2 = bl;
            for (int d = 0; d < mu; ++d) b2 /= g.NB[d];
            const int nmu = b2 % g.NB[mu];
            if (nmu == g.NB[mu] - 1 && x[mu] == B - 1) wf = -1;
            if (nmu == 0 && x[mu] == 0) wb = -1;
        }
        switch (mu) {
        case 0: hop_blk<T, B, 0, HOPS, 0, Vb>(&sh[0][0], 0, ing, Ug, slot, nbr, l, x, pin, acc, wf, wb); break;
        case 1: hop_blk<T, B, 1, HOPS, 0, Vb>(&sh[0][0], 0, ing, Ug, slot, nbr, l, x, pin, acc, wf, wb); break;
        case 2: hop_blk<T, B, 2, HOPS, 0, Vb>(&sh[0][0], 0, ing, Ug, slot, nbr, l, x, pin, acc, wf, wb); break;
        default: hop_blk<T, B, 3, HOPS, 0, Vb>(&sh[0][0], 0, ing, Ug, slot, nbr, l, x, pin, acc, wf, wb); break;
        }
    }
    if (CL) {
        cx<T> v[12], dg[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            v[c] = scale(-kappa, acc.s[c / 3].c[c % 3]);
            dg[c] = ld<T>(&sh[c][0], l);
        }
        clov_site<T, CLOV_DIAG>(ctab[m], (long)g.V, slot, Vb, l, dg, v);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const long i = m * n + base + (long)c * Vb;
            st_nt<T>(out, i, RES ? ld<T>(b, i) - v[c] : v[c]);
        }
        return;
    }
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int c = 3 * sp + a;
            const long i = m * n + base + (long)c * Vb;
            const cx<T> v = ld<T>(&sh[c][0], l) - scale(kappa, acc.s[sp].c[a]);
            st_nt<T>(out, i, RES ? ld<T>(b, i) - v : v);
        }
}

// The even-odd halves of the same operator (the stencil of the even-odd
// reduced solvers): out = diag - kappa H_{par, 1-par} in on the sites of
// parity par, gamma_5 on both sides for DAG; one workgroup per block, the
// body blk_eo_block (blk_stencil.h).
template <typename T, int B, int DAG, int CL>
__global__ __launch_bounds__(Cube<B>::Vh) void k_dslash_blk_eo(Geo g, const int32_t *__restrict__ active,
                                                              const int32_t *__restrict__ list, UTab<T> Utab,
                                                              const double *__restrict__ kap, int kneg,
                                                              const T *const *__restrict__ ctab, long n,
                                                              const int32_t *__restrict__ sched, int par,
                                                              const T2<T> *__restrict__ in,
                                                              const T2<T> *__restrict__ diag, T2<T> *__restrict__ out,
                                                              T kappa)
{
    __shared__ T2<T> sh[12][Cube<B>::Vh];  // the block's input on the other parity, component-major
    const int m = sys_at(list, blockIdx.y);
    if (active && !active[m]) return;
    blk_eo_block<T, B, DAG, CL, 0>(g, m, sched[blockIdx.x], threadIdx.x, Utab, kap, kneg, ctab, n, par, in, diag, out,
                                   kappa, sh);
}

// below this many workgroups (blocks x systems) the 4-workgroups-per-block
// k_dslash_dir keeps more of the GPU busy
constexpr long BLK_MIN_WORKGROUPS = 2048;

// the direction-parallel kernel for one (hops, clover mode); dag and the
// two-row link reads are chosen at run time
template <typename T, int B, int H, int CL>
void launch_dir(const Geo &g, const Sys &sy, Links<T> U, int par, int dag, const T2<T> *in, const T2<T> *diag,
                T2<T> *out, T kappa, int nslots, const int32_t *sc, hipStream_t s)
{
    const int chunks = (par < 0 ? Cube<B>::Vb : Cube<B>::Vh) / 64;
    const dim3 grid(nslots * chunks, sy.launch_m());
    const int xcd8 = nslots % 8 == 0;
#define WDR_DIR(D, R)                                                                                          \
    k_dslash_dir<T, H, B, D, R, CL><<<grid, 256, 0, s>>>(g, sy.active, sy.list, U.tab, U.kap, U.kneg, U.ctab, sy.n, \
                                                         sc, par, chunks, xcd8, in, diag, out, kappa)
    if (dag) {
        if (U.su3) WDR_DIR(1, 1);
        else WDR_DIR(1, 0);
    } else {
        if (U.su3) WDR_DIR(0, 1);
        else WDR_DIR(0, 0);
    }
#undef WDR_DIR
}

template <typename T, int B, int CL>
void launch_blk_eo(const Geo &g, const Sys &sy, Links<T> U, int par, int dag, const T2<T> *in, const T2<T> *diag,
                   T2<T> *out, T kappa, int nslots, const int32_t *sc, hipStream_t s)
{
    const dim3 gb(nslots, sy.launch_m());
    if (dag)
        k_dslash_blk_eo<T, B, 1, CL><<<gb, Cube<B>::Vh, 0, s>>>(g, sy.active, sy.list, U.tab, U.kap, U.kneg, U.ctab,
                                                               sy.n, sc, par, in, diag, out, kappa);
    else
        k_dslash_blk_eo<T, B, 0, CL><<<gb, Cube<B>::Vh, 0, s>>>(g, sy.active, sy.list, U.tab, U.kap, U.kneg, U.ctab,
                                                               sy.n, sc, par, in, diag, out, kappa);
}

// clover mode of a launch: the links' mode when they carry a clover term and
// the launch has a diagonal term or multiplies by A^-1 (hops across block
// faces have neither)
template <typename T> int clover_mode(const Links<T> &U, int hops)
{
    return U.ctab && hops != HOPS_CROSS ? U.cmode : CLOV_NONE;
}

template <typename T, int B>
bool launch_cube(const Geo &g, const Sys &sy, Links<T> U, int hops, int par, int dag, const T2<T> *in,
                 const T2<T> *diag, T2<T> *out, T kappa, int slot0, int nslots, hipStream_t s)
{
    if (g.B[0] != B || g.B[1] != B || g.B[2] != B || g.B[3] != B) return false;
    const int si = sched_index(g, slot0, nslots);
    if (si < 0) return false;
    static_assert(Cube<B>::Vh % 64 == 0, "sites of one parity fill whole wavefronts");
    const int32_t *sc = g.sched[si];
    const int cl = clover_mode(U, hops);
    // D or D_b with the input as diagonal term, with enough blocks to fill
    // the GPU (one workgroup per block): the block-staged kernel
    const bool big = (long)nslots * sy.launch_m() >= BLK_MIN_WORKGROUPS;
    const bool blk = g.stencil == WDR_STENCIL_BLK || (g.stencil == WDR_STENCIL_AUTO && big);
    if (par < 0 && !dag && U.su3 && diag == in && (hops == HOPS_ALL || hops == HOPS_IN) && cl != CLOV_INV && blk) {
        const dim3 gb(nslots, sy.launch_m());
#define WDR_BLK(H, C)                                                                                          \
    k_dslash_blk<T, B, H, 0, C><<<gb, Cube<B>::Vb, 0, s>>>(g, sy.active, sy.list, U.tab, U.kap, U.kneg, U.ctab, sy.n, \
                                                           sc, in, nullptr, out, kappa)
        if (hops == HOPS_ALL) {
            if (cl) WDR_BLK(HOPS_ALL, CLOV_DIAG);
            else WDR_BLK(HOPS_ALL, CLOV_NONE);
        } else {
            if (cl) WDR_BLK(HOPS_IN, CLOV_DIAG);
            else WDR_BLK(HOPS_IN, CLOV_NONE);
        }
#undef WDR_BLK
        return true;
    }
    // the even-odd halves (all hops), same choice
    if (par >= 0 && hops == HOPS_ALL && U.su3 && blk) {
        if (cl == CLOV_DIAG) launch_blk_eo<T, B, CLOV_DIAG>(g, sy, U, par, dag, in, diag, out, kappa, nslots, sc, s);
        else if (cl == CLOV_INV) launch_blk_eo<T, B, CLOV_INV>(g, sy, U, par, dag, in, diag, out, kappa, nslots, sc, s);
        else launch_blk_eo<T, B, CLOV_NONE>(g, sy, U, par, dag, in, diag, out, kappa, nslots, sc, s);
        return true;
    }
    if (hops == HOPS_CROSS) {
        launch_dir<T, B, HOPS_CROSS, CLOV_NONE>(g, sy, U, par, dag, in, diag, out, kappa, nslots, sc, s);
    } else if (hops == HOPS_ALL) {
        if (cl == CLOV_DIAG) launch_dir<T, B, HOPS_ALL, CLOV_DIAG>(g, sy, U, par, dag, in, diag, out, kappa, nslots, sc, s);
        else if (cl == CLOV_INV) launch_dir<T, B, HOPS_ALL, CLOV_INV>(g, sy, U, par, dag, in, diag, out, kappa, nslots, sc, s);
        else launch_dir<T, B, HOPS_ALL, CLOV_NONE>(g, sy, U, par, dag, in, diag, out, kappa, nslots, sc, s);
    } else {
        if (cl == CLOV_DIAG) launch_dir<T, B, HOPS_IN, CLOV_DIAG>(g, sy, U, par, dag, in, diag, out, kappa, nslots, sc, s);
        else if (cl == CLOV_INV) launch_dir<T, B, HOPS_IN, CLOV_INV>(g, sy, U, par, dag, in, diag, out, kappa, nslots, sc, s);
        else launch_dir<T, B, HOPS_IN, CLOV_NONE>(g, sy, U, par, dag, in, diag, out, kappa, nslots, sc, s);
    }
    return true;
}

// SU(3) deviation of canonical FP64 links: per workgroup max into partial
__global__ __launch_bounds__(256) void k_su3_dev(long nlinks, const double2 *__restrict__ U, double *partial)
{
    __shared__ double sh[256];
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    double dev = 0;
    if (i < nlinks) {
        su3<double> u;
        for (int e = 0; e < 9; ++e) {
            const double2 v = U[i * 9 + e];
            u.m[e / 3][e % 3] = mk<double>(v.x, v.y);
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                cx<double> s = mk<double>(0, 0);
                for (int k = 0; k < 3; ++k) s = s + u.m[a][k] * mk<double>(u.m[b][k].re, -u.m[b][k].im);
                const double want = a == b ? 1.0 : 0.0;
                dev = fmax(dev, fabs(s.re - want) + fabs(s.im));
            }
        const cx<double> det = u.m[0][0] * (u.m[1][1] * u.m[2][2] - u.m[1][2] * u.m[2][1]) -
                               u.m[0][1] * (u.m[1][0] * u.m[2][2] - u.m[1][2] * u.m[2][0]) +
                               u.m[0][2] * (u.m[1][0] * u.m[2][1] - u.m[1][1] * u.m[2][0]);
        dev = fmax(dev, fabs(det.re - 1.0) + fabs(det.im));
        if (!(dev == dev)) dev = 1e300;  // NaN
    }
    sh[threadIdx.x] = dev;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_max_final(int n, const double *partial, double *out)
{
    __shared__ double sh[256];
    double v = 0;
    for (int i = threadIdx.x; i < n; i += 256) v = fmax(v, partial[i]);
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// ---------------------------------------------------------------- packing

template <typename T>
__global__ __launch_bounds__(256) void k_pack_spinor(Geo g, const double2 *__restrict__ canon,
                                                     typename C2<T>::type *__restrict__ out)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const int slot = blockIdx.y;
    int x[4];
    const long s = canon_index(g, slot, l, x);
    const long base = (long)slot * 12 * g.Vb + l;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double2 v = canon[s * 12 + c];
        typename C2<T>::type w;
        w.x = (T)v.x;
        w.y = (T)v.y;
        out[base + (long)c * g.Vb] = w;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_unpack_spinor(Geo g, const typename C2<T>::type *__restrict__ in,
                                                       double2 *__restrict__ canon)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const int slot = blockIdx.y;
    int x[4];
    const long s = canon_index(g, slot, l, x);
    const long base = (long)slot * 12 * g.Vb + l;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        typename C2<T>::type v = in[base + (long)c * g.Vb];
        canon[s * 12 + c] = make_double2((double)v.x, (double)v.y);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_pack_gauge(Geo g, int4 bc, const double2 *__restrict__ canon,
                                                    typename C2<T>::type *__restrict__ out)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const int slot = blockIdx.y;
    int x[4];
    const long s = canon_index(g, slot, l, x);
    const int bcv[4] = {bc.x, bc.y, bc.z, bc.w};
    for (int mu = 0; mu < 4; ++mu) {
        const double f = (x[mu] == g.L[mu] - 1) ? (double)bcv[mu] : 1.0;
        const long base = ((long)slot * 4 + mu) * 9 * g.Vb + l;
        for (int e = 0; e < 9; ++e) {
            double2 v = canon[(s * 4 + mu) * 9 + e];
            typename C2<T>::type w;
            w.x = (T)(f * v.x);
            w.y = (T)(f * v.y);
            out[base + (long)e * g.Vb] = w;
        }
    }
}

__global__ __launch_bounds__(256) void k_unpack_gauge(Geo g, int4 bc, const double2 *__restrict__ in,
                                                      double2 *__restrict__ canon)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= g.Vb) return;
    const int slot = blockIdx.y;
    int x[4];
    const long s = canon_index(g, slot, l, x);
    const int bcv[4] = {bc.x, bc.y, bc.z, bc.w};
    for (int mu = 0; mu < 4; ++mu) {
        const double f = (x[mu] == g.L[mu] - 1) ? (double)bcv[mu] : 1.0;
        const long base = ((long)slot * 4 + mu) * 9 * g.Vb + l;
        for (int e = 0; e < 9; ++e) {
            double2 v = in[base + (long)e * g.Vb];
            canon[(s * 4 + mu) * 9 + e] = make_double2(f * v.x, f * v.y);
        }
    }
}

__global__ __launch_bounds__(256) void k_convert_gauge_f32(long n, const double2 *__restrict__ in, float2 *__restrict__ out)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double2 v = in[i];
    out[i] = make_float2((float)v.x, (float)v.y);
}

// gamma_5 on every element of the batch: component c = (i / Vb) mod 12,
// spins 2 and 3 are the components c >= 6
template <typename T>
__global__ __launch_bounds__(256) void k_g5(long total, int Vb, const typename C2<T>::type *__restrict__ in,
                                            typename C2<T>::type *__restrict__ out)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= total) return;
    typename C2<T>::type v = in[i];
    if ((i / Vb) % 12 >= 6) {
        v.x = -v.x;
        v.y = -v.y;
    }
    out[i] = v;
}

}  // namespace

template <typename T>
void launch_dslash(const Geo &g, const Sys &sy, Links<T> U, int hops, int par, int dag, const T2<T> *in,
                   const T2<T> *diag, T2<T> *out, T kappa, int slot0, int nslots, hipStream_t s)
{
    if (nslots <= 0 || sy.M <= 0) return;
    if (launch_cube<T, 4>(g, sy, U, hops, par, dag, in, diag, out, kappa, slot0, nslots, s)) return;
    const int nloc = par < 0 ? g.Vb : g.Vh;
    dim3 grid((nloc + 255) / 256, nslots, sy.launch_m());
    const int cl = clover_mode(U, hops);
#define WDR_GEN(H, C)                                                                                        \
    k_dslash<T, H, C><<<grid, 256, 0, s>>>(g, sy.active, sy.list, U.tab, U.kap, U.kneg, U.ctab, sy.n, par, dag, in, \
                                           diag, out, kappa, slot0)
#define WDR_GEN2(H)                                                                                          \
    do {                                                                                                     \
        if (cl == CLOV_DIAG) WDR_GEN(H, CLOV_DIAG);                                                         \
        else if (cl == CLOV_INV) WDR_GEN(H, CLOV_INV);                                                      \
        else WDR_GEN(H, CLOV_NONE);                                                                          \
    } while (0)
    if (hops == HOPS_ALL) WDR_GEN2(HOPS_ALL);
    else if (hops == HOPS_IN) WDR_GEN2(HOPS_IN);
    else WDR_GEN(HOPS_CROSS, CLOV_NONE);
#undef WDR_GEN2
#undef WDR_GEN
}

bool launch_block_residual(const Geo &g, const Sys &sy, Links<double> U, const double2 *x, const double2 *b,
                           double2 *r, double kappa, int slot0, int nslots, hipStream_t s)
{
    if (nslots <= 0 || sy.M <= 0) return true;
    if (g.B[0] != 4 || g.B[1] != 4 || g.B[2] != 4 || g.B[3] != 4 || !U.su3 || U.ctab) return false;
    const bool big = (long)nslots * sy.launch_m() >= BLK_MIN_WORKGROUPS;
    if (!(g.stencil == WDR_STENCIL_BLK || (g.stencil == WDR_STENCIL_AUTO && big))) return false;
    const int si = sched_index(g, slot0, nslots);
    if (si < 0) return false;
    k_dslash_blk<double, 4, HOPS_IN, 1><<<dim3(nslots, sy.launch_m()), Cube<4>::Vb, 0, s>>>(
        g, sy.active, sy.list, U.tab, U.kap, U.kneg, nullptr, sy.n, g.sched[si], x, b, r, kappa);
    return true;
}

template <typename T> void launch_pack_spinor(const Geo &g, const double2 *canon, typename C2<T>::type *out, hipStream_t s)
{
    k_pack_spinor<T><<<dim3((g.Vb + 255) / 256, g.nblk), 256, 0, s>>>(g, canon, out);
}
template <typename T> void launch_unpack_spinor(const Geo &g, const typename C2<T>::type *in, double2 *canon, hipStream_t s)
{
    k_unpack_spinor<T><<<dim3((g.Vb + 255) / 256, g.nblk), 256, 0, s>>>(g, in, canon);
}
template <typename T>
void launch_pack_gauge(const Geo &g, const int bc[4], const double2 *canon, typename C2<T>::type *out, hipStream_t s)
{
    k_pack_gauge<T><<<dim3((g.Vb + 255) / 256, g.nblk), 256, 0, s>>>(g, make_int4(bc[0], bc[1], bc[2], bc[3]), canon,
                                                                     out);
}
void launch_unpack_gauge(const Geo &g, const int bc[4], const double2 *in, double2 *canon, hipStream_t s)
{
    k_unpack_gauge<<<dim3((g.Vb + 255) / 256, g.nblk), 256, 0, s>>>(g, make_int4(bc[0], bc[1], bc[2], bc[3]), in,
                                                                    canon);
}
void launch_su3_deviation(const Geo &g, const double2 *U, double *partial, double *dev_out, hipStream_t s)
{
    const long nl = (long)g.V * 4;
    const int nb = (int)((nl + 255) / 256);
    k_su3_dev<<<nb, 256, 0, s>>>(nl, U, partial);
    k_max_final<<<1, 256, 0, s>>>(nb, partial, dev_out);
}

void launch_convert_gauge_f32(const Geo &g, const double2 *in, float2 *out, hipStream_t s)
{
    long n = (long)g.V * 36;
    k_convert_gauge_f32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, in, out);
}
template <typename T> void launch_g5(const Geo &g, const Sys &sy, const T2<T> *in, T2<T> *out, hipStream_t s)
{
    const long total = sy.n * sy.M;
    k_g5<T><<<(unsigned)((total + 255) / 256), 256, 0, s>>>(total, g.Vb, in, out);
}

#define INST(T)                                                                                                  \
    template void launch_dslash<T>(const Geo &, const Sys &, Links<T>, int, int, int, const T2<T> *,              \
                                   const T2<T> *, T2<T> *, T, int, int, hipStream_t);                            \
    template void launch_pack_spinor<T>(const Geo &, const double2 *, C2<T>::type *, hipStream_t);               \
    template void launch_unpack_spinor<T>(const Geo &, const C2<T>::type *, double2 *, hipStream_t);             \
    template void launch_pack_gauge<T>(const Geo &, const int *, const double2 *, C2<T>::type *, hipStream_t);   \
    template void launch_g5<T>(const Geo &, const Sys &, const T2<T> *, T2<T> *, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace wdr
