// Packed FP16 arithmetic on complex numbers stored as (re, im) pairs of
// IEEE binary16: one v_pk_* instruction acts on both halves, so a complex
// multiply-add is two packed FMAs.  Used by the hop arithmetic of the FP16
// solver levels, whose operands are stored values of magnitude at most a few
// units (block-scaled fields, SU(3) links).
#pragma once

#include "wdr_internal.h"

namespace wdr {
namespace dev {

__device__ __forceinline__ h2 hbr(_Float16 a) { return (h2){a, a}; }
// acc + u v
__device__ __forceinline__ h2 hcfma(h2 u, h2 v, h2 acc)
{
    const h2 t = hbr(u.x) * v + acc;
    return hbr(u.y) * (h2){-v.y, v.x} + t;
}
// acc + conj(u) v
__device__ __forceinline__ h2 hcjfma(h2 u, h2 v, h2 acc)
{
    const h2 t = hbr(u.x) * v + acc;
    return hbr(u.y) * (h2){v.y, -v.x} + t;
}
// the maps of the spin projections (A_dn, Adag_h): 0 identity, 1 negate,
// 2 times i, 3 times -i
__device__ __forceinline__ h2 hmap(h2 v, int op)
{
    return op == 0 ? v : op == 1 ? -v : op == 2 ? (h2){-v.y, v.x} : (h2){v.y, -v.x};
}

}  // namespace dev
}  // namespace wdr
