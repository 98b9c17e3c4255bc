// Per-element arithmetic of the local accelerated primal-dual step (Chambolle
// and Pock, Alg. 2, on the local saddle problem eq. (local) of Sec. 5), shared
// by the streaming and the fused kernels so that both schedules round
// identically:
//   xbar_{k-1} = x_{k-1} + theta_{k-1} (x_{k-1} - x_{k-2})          (per edge)
//   u_k = prox_{sigma_k alpha F}(u_{k-1} + sigma_k div_s xbar_{k-1})  (per pixel)
//   x_k = proj_C(c_keep (x_{k-1} - tau_k div_s^* u_k) + c_anchor phat)  (per edge)
// with c_keep = tau/(tau + tau_k), c_anchor = tau_k/(tau + tau_k) (1 and 0
// without the proximal term).
#pragma once

#include <hip/hip_runtime.h>

namespace dtv {

// prox of a F at one pixel: L2 (z + a f)/(1 + a); L1 f + shr(z - f, a), eq.
// (shrinkage); convex Chan-Vese (Sec. 3, segmentation) the projection of z - a g
// onto [0, 1], with g = (f - c1)^2 - (f - c2)^2 evaluated as (c2 - c1)((f - c1) + (f - c2)),
// the same value without the cancellation of two squares.  Pixels in the
// inpainting set D (not observed) have no fidelity term.
__device__ __forceinline__ float prox_fid(int fidelity, float z, float fv, bool observed, float a, float c1,
                                          float c2)
{
    if (!observed) return z;
    if (fidelity == 0) return (z + a * fv) / (1.0f + a);
    if (fidelity == 2) {
        const float g = (c2 - c1) * ((fv - c1) + (fv - c2));
        return fminf(fmaxf(fmaf(-a, g, z), 0.0f), 1.0f);
    }
    const float d = z - fv;
    const float mag = fmaxf(fabsf(d) - a, 0.0f);
    return d > 0.0f ? fv + mag : (d < 0.0f ? fv - mag : fv);
}

// the primal update of one pixel from the divergence d of xbar
__device__ __forceinline__ float cp2_u(int fidelity, float u, float d, float sk, float fv, bool observed, float sa,
                                       float c1, float c2)
{
    return prox_fid(fidelity, fmaf(sk, d, u), fv, observed, sa, c1, c2);
}

// the dual update of one edge before the projection: du = (div_s^* u) on the
// edge (u of the pixel before it minus u of the pixel after it)
__device__ __forceinline__ float cp2_pre(float x, float du, float anchor, float tk, float ck, float ca)
{
    return fmaf(ck, fmaf(-tk, du, x), ca * anchor);
}

}  // namespace dtv
