// The persistent reverse (fused_bwd.hip) and the transposed multiplier update it shares with the
// interface-transpose kernel (kernels_bwd.hip).
#pragma once

#include "dtvdd_internal.h"

namespace dtv {

// The reverse of every outer step of a range in one cooperative launch (fused_bwd.hip): outer
// steps q = n_steps - 1 .. 0, pbar kept on chip between them, the interface transpose done with
// point-to-point exchange words.  The result is bitwise that of the per-step launches (the fused
// reverse followed by the interface transpose, step by step).
struct PersistBwdArgs {
    FusedBwdArgs b;           // imgs, subs, f, gf, galpha, tau, inv_tau, n_inner, beta; pb1/pb2: in
                              // pbar after the range, out pbar before it (the other pointers unused)
    const float *st;          // state before outer step q (p~^q: P1 block, P2 block at p2_off; the
    long long st_stride;      // lambda state at lam_off) at st + q st_stride, q = 0 .. n_steps
    long long p2_off, lam_off;
    const float4 *rec;        // step records of outer step q at rec + q rec_outer
    long long rec_outer;
    int n_steps;
    float sigma;
    float *lamb;              // lambdabar state (3 values per multiplier), in and out
    unsigned long long *xch;  // exchange words: 2 slots of xch_stride, zero at launch
    long long xch_stride;     // >= length of the lambda state
    int *err;                 // set to 1 when a wait for a neighbour times out
    unsigned spin_limit;      // polls of one exchange word before a wait gives up
};
int persist_bwd_capacity(int device, int K);  // workgroups of the persistent reverse resident at once
hipError_t launch_persist_bwd(const PersistBwdArgs &a, int nsub, hipStream_t s);

// The transposed multiplier update of one interface edge (the adjoint of
// lambda^(n+1) = lambda^n + sigma (q_s - q_t), q = 2 p~^n - p~^(n-1), and of the
// anchors phat = p~^n -/+ tau lambda^(n+1) on the two copies): from phatbar on the
// s and t copies and the lambdabar state (l0, l1, l2), the increments of pbar on
// the two copies; l0 becomes the new first component (the others are -sigma l0
// and sigma l0).
__device__ __forceinline__ void iface_bwd(float hs, float ht, float tau, float sigma, float &l0, float l1, float l2,
                                          float &ds, float &dt)
{
    const float lt = fmaf(-tau, hs - ht, l0);
    const float s2 = 2.0f * sigma;
    ds = fmaf(s2, lt, l1);
    dt = fmaf(-s2, lt, l2);
    l0 = lt;
}

}  // namespace dtv
