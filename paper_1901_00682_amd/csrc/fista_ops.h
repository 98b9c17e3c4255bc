// Per-edge arithmetic of the local FISTA step, shared by the streaming and
// the fused kernels so that both schedules round identically.
//
// Local dual problem of one subdomain (eq. DD_local_dual for ROF):
//   min_{|p| <= 1} (alpha/2)|f + div_s p / alpha|^2 + (1/(2 tau))|p - phat|^2,
// gradient div_s^*(f + div_s p / alpha) + (p - phat)/tau, Lipschitz bound
// L = 8/alpha + 1/tau.  On an edge e with pixel b before it and pixel a after
// it (value 0 outside the subdomain), the projected gradient step from y is
//   z = y - (1/L) [ (f_b - f_a) + (d_b - d_a)/alpha + (y - phat)/tau ],  d = div_s y,
//     = a_keep y + c' - kL (d_b - d_a),
//   a_keep = 1 - 1/(L tau),  kL = 1/(alpha L),  c' = (phat/tau - (f_b - f_a))/L,
// followed by the projection onto [-1, 1] (eq. proj_C).
#pragma once

#include <hip/hip_runtime.h>

namespace dtv {

// Workgroup ids are dealt to the 8 XCDs round-robin; remap them so that
// consecutive work items (which share halo rows in L2) run on one XCD.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int xcd = b & 7, idx = b >> 3;
    const int per = n >> 3, rem = n & 7;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

__device__ __forceinline__ float clamp1(float z) { return __builtin_amdgcn_fmed3f(z, -1.0f, 1.0f); }

// c' of one edge from its anchor phat and the image values on both sides
__device__ __forceinline__ float fista_cprime(float anchor, float f_b, float f_a, float inv_tau, float invL)
{
    return fmaf(anchor, inv_tau, -(f_b - f_a)) * invL;
}

// extrapolated point y = x + beta (x - x_prev)
__device__ __forceinline__ float fista_y(float x, float x_prev, float beta) { return fmaf(beta, x - x_prev, x); }

// gradient step on one edge before the projection
__device__ __forceinline__ float fista_z(float y, float d_b, float d_a, float c, float a_keep, float kL)
{
    return fmaf(-kL, d_b - d_a, fmaf(a_keep, y, c));
}

// projected step on one edge
__device__ __forceinline__ float fista_edge(float y, float d_b, float d_a, float c, float a_keep, float kL)
{
    return clamp1(fista_z(y, d_b, d_a, c, a_keep, kL));
}

// unscaled divergence of a pixel from its four edge values
__device__ __forceinline__ float div4(float top, float bottom, float left, float right)
{
    return (bottom - top) + (right - left);
}

}  // namespace dtv
