// Point-to-point exchange of interface copies between the tiles of a
// persistent launch (one workgroup per subdomain for the whole solve).
//
// Every copy travels in a 64-bit word that also holds its outer step + 1,
// written and polled with relaxed agent-scope atomics, so a word is valid
// exactly when its step number matches and no fence or grid-wide barrier is
// needed (an agent-scope fence writes back and invalidates a whole L2).  The
// words alternate between two slots by step parity; a tile overwrites slot
// n % 2 at step n + 2 only after it has read its neighbour's step n + 1 copy,
// which the neighbour publishes only after reading the step n word.  The
// cooperative launch keeps every tile resident, so every wait can end; a wait
// is also bounded and then reported.
#pragma once

#include "dtvdd_internal.h"

namespace dtv {
namespace xchg {

constexpr int kSides = 4;                // 0 top (t copies), 1 bottom (s), 2 left (t), 3 right (s)

// exchange word: the copy in the low half, its outer step + 1 in the high half
__device__ __forceinline__ void publish(unsigned long long *w, float q, int n)
{
    const unsigned long long v = ((unsigned long long)(unsigned)(n + 1) << 32) | __float_as_uint(q);
    __hip_atomic_store(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// waits for the step-n word; false after `limit` polls
__device__ __forceinline__ bool fetch(const unsigned long long *w, int n, float &q, unsigned limit)
{
    for (unsigned spins = 0; spins < limit; ++spins) {
        const unsigned long long v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((unsigned)(v >> 32) == (unsigned)(n + 1)) {
            q = __uint_as_float((unsigned)v);
            return true;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return false;
}

// lambda index of edge i of side `side` of tile (r, c) (interface edges only)
__device__ __forceinline__ long long side_edge(const ImgDev &im, const SubTile &tl, int side, int i)
{
    switch (side) {
    case 0: return (long long)(tl.r - 1) * im.W + tl.ca + i;
    case 1: return (long long)tl.r * im.W + tl.ca + i;
    case 2: return im.nlh + (long long)(tl.c - 1) * im.H + tl.ra + i;
    default: return im.nlh + (long long)tl.c * im.H + tl.ra + i;
    }
}

__device__ __forceinline__ bool side_exists(const ImgDev &im, const SubTile &tl, int side)
{
    switch (side) {
    case 0: return tl.r > 0;
    case 1: return tl.r < im.ny - 1;
    case 2: return tl.c > 0;
    default: return tl.c < im.nx - 1;
    }
}

}  // namespace xchg
}  // namespace dtv
