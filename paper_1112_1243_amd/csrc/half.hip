// FP16 storage with per-block power-of-two scales for the inner solver
// (blocks of Sec. 3).  A block's values are stored as fp16(v / s) with
// s = 2^ceil(log2 max |component|) over the block, so every stored value lies
// in [-1, 1] with an 11-bit significand and the scaling itself is exact;
// arithmetic on FP16 data is done in FP32.  SU(3) links (entries of modulus
// at most 1) are stored unscaled, first two rows only.
#include "stencil.h"

namespace wdr {
namespace {

using namespace dev;

constexpr int NT = 256;

// one workgroup per (slot, system): block maximum, scale, rounded store
template <typename T>
__global__ __launch_bounds__(NT) void k_to_h16(Geo g, const int32_t *__restrict__ active, long n, int slot0,
                                              const T2<T> *__restrict__ in, h2 *__restrict__ out,
                                              float *__restrict__ scale)
{
    __shared__ float red[NT / 64];
    const int slot = slot0 + blockIdx.x, m = blockIdx.y;
    if (active && !active[m]) return;
    const long cnt = 12L * g.Vb, base = m * n + (long)slot * cnt;
    float mx = 0.f;
    for (long i = threadIdx.x; i < cnt; i += NT) {
        const T2<T> v = in[base + i];
        mx = fmaxf(mx, fmaxf(fabsf((float)v.x), fabsf((float)v.y)));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_down(mx, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    float bmax = red[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) bmax = fmaxf(bmax, red[w]);
    const float s = pow2_at_least(bmax), inv = 1.f / s;
    for (long i = threadIdx.x; i < cnt; i += NT) {
        const T2<T> v = in[base + i];
        out[base + i] = to_h2(mk<float>((float)v.x, (float)v.y), inv);
    }
    if (threadIdx.x == 0) scale[(long)m * g.nblk + slot] = s;
}

// elements of the slots [slot0, slot0 + cnt / (12 Vb)) of every system
__global__ __launch_bounds__(NT) void k_from_h16(Geo g, const int32_t *__restrict__ active, long n, long cnt,
                                                int slot0, long total, const h2 *__restrict__ in,
                                                const float *__restrict__ scale, double2 *__restrict__ y, int add)
{
    const long k = (long)blockIdx.x * NT + threadIdx.x;
    if (k >= total) return;
    const int m = (int)(k / cnt);
    if (active && !active[m]) return;
    const long i = (long)m * n + 12L * g.Vb * slot0 + (k - (long)m * cnt);
    const int slot = (int)((i - (long)m * n) / (12L * g.Vb));
    const float s = scale[(long)m * g.nblk + slot];
    const h2 v = in[i];
    const double re = (double)((float)v.x * s), im = (double)((float)v.y * s);
    if (add) {
        const double2 o = y[i];
        y[i] = make_double2(o.x + re, o.y + im);
    } else {
        y[i] = make_double2(re, im);
    }
}

__global__ __launch_bounds__(NT) void k_zero_h16(long total, long nscale, h2 *__restrict__ v, float *__restrict__ s)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i < total) v[i] = h2{(_Float16)0.f, (_Float16)0.f};
    if (i < nscale) s[i] = 1.f;
}

// [slot][mu][9][Vb] FP64 -> [slot][mu][6][Vb] FP16 (rows 0 and 1)
__global__ __launch_bounds__(NT) void k_pack_links_h16(long total, int Vb, const double2 *__restrict__ u64,
                                                      h2 *__restrict__ u16)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;  // over slots x 4 x 6 x Vb
    if (i >= total) return;
    const long l = i % Vb, e = (i / Vb) % 6, sm = i / (6L * Vb);  // sm = slot * 4 + mu
    const double2 v = u64[(sm * 9 + e) * Vb + l];
    h2 r;
    r.x = (_Float16)(float)v.x;
    r.y = (_Float16)(float)v.y;
    u16[i] = r;
}

// Wilson-Dirac operator out = in - kappa H in on FP16 fields (the storage
// of the inner solver, paper Sec. 5 operator on the blocks of Sec. 3): in and
// out FP16 with per-block power-of-two scales, the links the FP16 first two
// rows of an SU(3) field, arithmetic in FP32.  One workgroup per B^4 block;
// wavefront mu computes the two hops of direction mu (compile-time spin
// projection) for the 64 sites of each of the block's chunks in turn, the
// partial sums meet in LDS, and wavefront w keeps spin w of every site of the
// block in registers until the block maximum, and with it the output scale,
// is known.
template <int B>
__global__ __launch_bounds__(NT) void k_dslash_h16(Geo g, const h2 *__restrict__ Uh, const int32_t *__restrict__ sched,
                                                  const h2 *__restrict__ in, const float *__restrict__ in_s,
                                                  h2 *__restrict__ out, float *__restrict__ out_s, float kappa)
{
    typedef Cube<B> CB;
    constexpr int Vb = CB::Vb, NC = Vb / 64;
    static_assert(Vb % 64 == 0, "a block is a whole number of 64-site chunks");
    __shared__ float2 part[4][12][64];  // [mu][colour-spin component][site of the chunk]
    __shared__ float red[NT / 64];
    const int slot = sched[blockIdx.x];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int mu = __builtin_amdgcn_readfirstlane(w);
    int nbr[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) nbr[k] = g.slot_nbr[slot * 8 + k];
    int nmu = g.slot_blk[slot];  // block coordinate along mu
    for (int d = 0; d < mu; ++d) nmu /= g.NB[d];
    nmu %= g.NB[mu];
    const SpinorLdH<Vb> xin{as_global(in), in_s};
    const LinkLdH<Vb> lk{as_global(Uh)};
    cx<float> res[NC][3];
    float mx = 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int l = c * 64 + lane;
        int x[4];
        CB::coords(l, x);
        // boundary sign of the links of this site that wrap around the
        // lattice (needed to rebuild their third rows)
        float wf = 1.f, wb = 1.f;
        if (g.bc[mu] < 0) {
            if (nmu == g.NB[mu] - 1 && x[mu] == B - 1) wf = -1.f;
            if (nmu == 0 && x[mu] == 0) wb = -1.f;
        }
        spinor<float> acc;
        zero(acc);
        switch (mu) {
        case 0: hop_dir_ld<float, HOPS_ALL, B, 0, 0, 1>(xin, lk, slot, nbr, l, x, acc, wf, wb); break;
        case 1: hop_dir_ld<float, HOPS_ALL, B, 0, 1, 1>(xin, lk, slot, nbr, l, x, acc, wf, wb); break;
        case 2: hop_dir_ld<float, HOPS_ALL, B, 0, 2, 1>(xin, lk, slot, nbr, l, x, acc, wf, wb); break;
        default: hop_dir_ld<float, HOPS_ALL, B, 0, 3, 1>(xin, lk, slot, nbr, l, x, acc, wf, wb); break;
        }
        if (c) __syncthreads();  // the previous chunk's partial sums have been read
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) part[w][3 * sp + a][lane] = make_float2(acc.s[sp].c[a].re, acc.s[sp].c[a].im);
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int comp = 3 * mu + a;
            float2 v = part[0][comp][lane];
#pragma unroll
            for (int d = 1; d < 4; ++d) {
                const float2 q = part[d][comp][lane];
                v.x += q.x;
                v.y += q.y;
            }
            const cx<float> o = xin(slot, comp, l) - scale(kappa, mk<float>(v.x, v.y));
            res[c][a] = o;
            mx = fmaxf(mx, fmaxf(fabsf(o.re), fabsf(o.im)));
        }
    }
    // block maximum -> power-of-two scale of the output
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_down(mx, off, 64));
    if (lane == 0) red[w] = mx;
    __syncthreads();
    float bmax = red[0];
#pragma unroll
    for (int k = 1; k < NT / 64; ++k) bmax = fmaxf(bmax, red[k]);
    const float sc = pow2_at_least(bmax), inv = 1.f / sc;
    const long base = (long)slot * 12 * Vb;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) out[base + (long)(3 * mu + a) * Vb + c * 64 + lane] = to_h2(res[c][a], inv);
    if (threadIdx.x == 0) out_s[slot] = sc;
}

inline unsigned nblocks(long n) { return (unsigned)((n + NT - 1) / NT); }

}  // namespace

bool launch_dslash_h16(const Geo &g, const h2 *U16, H16c in, H16 out, float kappa, hipStream_t s)
{
    if (!U16 || g.B[0] != 4 || g.B[1] != 4 || g.B[2] != 4 || g.B[3] != 4) return false;
    const int si = sched_index(g, 0, g.nblk);
    if (si < 0) return false;
    k_dslash_h16<4><<<g.nblk, NT, 0, s>>>(g, U16, g.sched[si], in.v, in.s, out.v, out.s, kappa);
    return true;
}

template <typename T>
void launch_to_h16(const Geo &g, const Sys &sy, const T2<T> *in, H16 out, int slot0, int nslots, hipStream_t s)
{
    if (nslots <= 0 || sy.M <= 0) return;
    k_to_h16<T><<<dim3(nslots, sy.M), NT, 0, s>>>(g, sy.active, sy.n, slot0, in, out.v, out.s);
}
void launch_from_h16(const Geo &g, const Sys &sy, H16c in, double2 *y, int add, int slot0, int nslots, hipStream_t s)
{
    const long cnt = 12L * g.Vb * nslots, total = cnt * sy.M;
    if (total > 0)
        k_from_h16<<<nblocks(total), NT, 0, s>>>(g, sy.active, sy.n, cnt, slot0, total, in.v, in.s, y, add);
}
void launch_zero_h16(const Geo &g, const Sys &sy, H16 f, hipStream_t s)
{
    const long total = sy.n * sy.M, ns = (long)g.nblk * sy.M;
    const long m = total > ns ? total : ns;
    if (m > 0) k_zero_h16<<<nblocks(m), NT, 0, s>>>(total, ns, f.v, f.s);
}
void launch_pack_links_h16(const Geo &g, const double2 *u64, h2 *u16, hipStream_t s)
{
    const long total = (long)g.nblk * 4 * 6 * g.Vb;
    k_pack_links_h16<<<nblocks(total), NT, 0, s>>>(total, g.Vb, u64, u16);
}
template void launch_to_h16<double>(const Geo &, const Sys &, const double2 *, H16, int, int, hipStream_t);
template void launch_to_h16<float>(const Geo &, const Sys &, const float2 *, H16, int, int, hipStream_t);

}  // namespace wdr
