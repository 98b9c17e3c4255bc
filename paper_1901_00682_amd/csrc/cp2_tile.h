// One subdomain's local accelerated primal-dual solve (Lee & Park, arXiv
// 1901.00682, Sec. 5: Chambolle-Pock Alg. 2 on the local saddle problem eq.
// (local)) held on chip by one 1024-thread workgroup: the device code shared by
// the fused and the persistent primal-dual kernels.
//
// Layout (as in the fused FISTA kernels): wave s owns pixel rows 8 s .. 8 s + 7
// of the 128 x 128 tile, lane l owns columns 2l ("a") and 2l + 1 ("b"); each
// thread owns the top and left edges of its 16 pixels, strip 15 the tile's
// bottom boundary edges, lanes 0..7 of each strip the right boundary edges of
// the strip's rows (in LDS).
//   VGPRs: x_k on the owned edges, u, f (and the observed bits) of the pixels.
//   LDS:   the anchor phat of every edge (128 KB), u of each strip's last row,
//          xbar of each strip's first-row top edges, u of the last column.
// The step is reordered so that xbar never needs a register slot of its own:
// u_1 = prox(u_0 + sigma_1 div x_0) first; then step k updates x_k from u_k
// row by row, forms xbar_k on the row's edges and, one row behind, the
// divergence of xbar_k and u_(k+1).  Two barriers per step: (A) u of the
// strips' last rows, (B) xbar of their first rows.
//
// The per-element arithmetic is that of the streaming kernel (cp2_ops.h), so
// all schedules give bitwise identical results.
//
// Adaptive stopping (the inner rule of Sec. 5.1): after step k the tile sums
// |x_k - x_(k-1)|^2 and |x_k|^2 over its edges (FP32 per thread, then FP64
// over the workgroup in a fixed order) and stops when the first is below
// tol^2 times the second.  Step k has already formed u_(k+1) one row behind
// the x update, so u_k is written to the tile's own pixels of the u buffer at
// the start of the step (no other tile reads them) and read back on a stop.
#pragma once

#include "cp2_ops.h"
#include "fused_common.h"

namespace dtv {
namespace cp2tile {

using namespace fused;

struct Cp2Lds {
    // the small arrays first, so that their offsets fit the 16-bit immediate of LDS instructions
    float ab[kFusedMax];              // anchor of the bottom boundary edges (per column)
    float ar[kFusedMax];              // anchor of the right boundary edges (per row)
    float rx[kFusedMax];              // right boundary edges: x_k (per row)
    float rxb[kFusedMax];             // right boundary edges: xbar_k (per row)
    float uR[kFusedMax];              // u of the last column (per row)
    double red[2 * kWaves];           // adaptive stopping: per-wave sums of the relative-change test
    float ut[kWaves][kFusedMax];      // u of each strip's last row
    float xt[kWaves][kFusedMax];      // xbar of the top edges of each strip's first row
    float a1[kFusedMax][kFusedMax];   // anchor of the edge above pixel (il, jl)
    float a2[kFusedMax][kFusedMax];   // anchor of the edge left of pixel (il, jl)
};

__device__ __forceinline__ void ld2g(const float *p, float &x, float &y)
{
    float2 v;
    __builtin_memcpy(&v, p, 8);
    x = v.x;
    y = v.y;
}

__device__ __forceinline__ void st2g(float *p, float x, float y)
{
    const float2 v = make_float2(x, y);
    __builtin_memcpy(p, &v, 8);
}

// divergence of the two pixels of a row from xbar on their edges: top (ta, tb),
// bottom (ba, bb), left (la, lb); the right edge of column b is the next lane's
// left edge of column a, or the tile's right boundary edge rxb on lane 63
__device__ __forceinline__ void div_pair(float ta, float tb, float ba, float bb, float la, float lb, float rxb,
                                         float &da, float &db)
{
    const float rb = from_right_or(la, rxb);
    da = div4(ta, ba, la, lb);
    db = div4(tb, bb, lb, rb);
}

// the tile and thread constants of the solve
struct Cp2Ctx {
    int s, lane, ja, jb, il0;
    bool last, bot_bnd, right_bnd;
    float lo1, hi1, lo2a, hi2a;  // clamp bounds of the first row's top edges and of column a's left edge
    float alpha, cv1, cv2;
    // framed tiles only (smaller than 128 x 128, short sides on the image boundary, run in a
    // 128 x 128 frame): clamp bounds of column b's left edge, and the strip's rows whose top edges
    // are the tile's bottom boundary (bit r: row 8 s + r)
    float lo2b, hi2b;
    unsigned zrows;
    // adaptive stopping: the tile's pixels in the u buffer (row pitch W), its extent (h x w)
    float *u_tile;
    int W, h, w;
};

// u of the thread's pixels inside the tile to / from the u buffer (adaptive stopping)
template <bool FR>
__device__ __forceinline__ void save_u(const Cp2Ctx &c, const float (&ua)[kR], const float (&ub)[kR])
{
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int il = c.il0 + r;
        float *p = c.u_tile + (long long)il * c.W + c.ja;
        if (!FR || (il < c.h && c.jb < c.w)) st2g(p, ua[r], ub[r]);
        else if (il < c.h && c.ja < c.w) p[0] = ua[r];
    }
}

template <bool FR>
__device__ __forceinline__ void load_u(const Cp2Ctx &c, float (&ua)[kR], float (&ub)[kR])
{
    // volatile: past the vector L1, which may hold the values of an earlier outer step
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int il = c.il0 + r;
        volatile const float *p = c.u_tile + (long long)il * c.W + c.ja;
        if (!FR || (il < c.h && c.jb < c.w)) {
            ua[r] = p[0];
            ub[r] = p[1];
        } else if (il < c.h && c.ja < c.w) {
            ua[r] = p[0];
        }
    }
}

// The n_inner steps of one outer step from x_0 (X, and the right boundary
// column in S.rx) and u_0, with the anchors in S.a1, a2, ab, ar (written by
// every thread before the call; the first barrier here orders them).  On
// return X, S.rx and (ua, ub) hold x_K and u_K.  ADAPT: at most n_inner steps,
// the step scalars from a.tab, stopping by the relative-change rule; returns
// the steps taken (n_inner without ADAPT).
// FR: a framed tile, its h x w pixels at the top left of the frame and its short sides on the
// image boundary.  Outside the tile x, u, f and the anchors start at 0; the top edges of row h and
// the left edges of column w are clamped to 0 like other image-boundary edges, so no value
// outside reaches the tile's edges and pixels (the pixels outside may move, bounded, under the
// Chan-Vese prox, which is not zero at f = 0).
template <int FID, bool FR = false, bool ADAPT = false>
__device__ __forceinline__ int solve(const Cp2Ctx &c, Cp2Lds &S, Slot &X, float (&ua)[kR], float (&ub)[kR],
                                     const float (&fa)[kR], const float (&fb)[kR], unsigned obs,
                                     const FusedCp2Args &a)
{
    const int s = c.s, lane = c.lane, ja = c.ja, jb = c.jb, il0 = c.il0;
    const bool last = c.last, bot_bnd = c.bot_bnd, right_bnd = c.right_bnd;
    const float lo1 = c.lo1, hi1 = c.hi1, lo2a = c.lo2a, hi2a = c.hi2a;
    const float alpha = c.alpha, cv1 = c.cv1, cv2 = c.cv2;
    constexpr int fid = FID;
    const int K = a.n_inner;
    // xbar_0 = x_0 on the first row's top edges (for the strip above) and on the right column
    if (s > 0) lds_st2(&S.xt[s][ja], X.e1a[0], X.e1b[0]);
    if (lane < kR) S.rxb[il0 + lane] = S.rx[il0 + lane];
    __syncthreads();

    auto observed = [&](int bit) { return ((obs >> bit) & 1u) != 0; };

    // ---- u_1 = prox(u_0 + sigma_1 div x_0)
    {
        const float sk = ADAPT ? a.tab[1] : a.sk[0], sa = sk * alpha;
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            float ba_ = 0.0f, bb_ = 0.0f;
            if (r < kR - 1) {
                ba_ = X.e1a[r + 1];
                bb_ = X.e1b[r + 1];
            } else if (!last) {
                lds_ld2(&S.xt[s + 1][ja], ba_, bb_);
            } else {
                ba_ = X.ba;
                bb_ = X.bb;
            }
            float da, db;
            div_pair(X.e1a[r], X.e1b[r], ba_, bb_, X.e2a[r], X.e2b[r], S.rxb[il0 + r], da, db);
            ua[r] = cp2_u(fid, ua[r], da, sk, fa[r], observed(2 * r), sa, cv1, cv2);
            ub[r] = cp2_u(fid, ub[r], db, sk, fb[r], observed(2 * r + 1), sa, cv1, cv2);
        }
    }

    // ---- the K steps
    int taken = K;
    for (int k = 1; k <= K; ++k) {
        float tk, ck, ca, th;
        if constexpr (ADAPT) {
            const float *tb = a.tab + 5 * (k - 1);
            tk = tb[0];
            th = tb[2];
            ck = tb[3];
            ca = tb[4];
        } else {
            tk = a.tk[k - 1];
            ck = a.ck[k - 1];
            ca = a.ca[k - 1];
            th = a.th[k - 1];
        }
        const bool ext = k < K;  // u_(k+1) is needed
        const float skn = ext ? (ADAPT ? a.tab[5 * k + 1] : a.sk[k]) : 0.0f, san = skn * alpha;
        float dd = 0.0f, nn = 0.0f;  // adaptive: |x_k - x_(k-1)|^2, |x_k|^2 over the thread's edges
        if constexpr (ADAPT) {
            if (ext) save_u<FR>(c, ua, ub);  // u_k, in case the rule stops after this step
        }
        // (A) publish u_k of the strip's last row (for the strip below) and of the last column
        if (!last) lds_st2(&S.ut[s][ja], ua[kR - 1], ub[kR - 1]);
        if (lane == 63)
#pragma unroll
            for (int r = 0; r < kR; ++r) S.uR[il0 + r] = ub[r];
        __syncthreads();

        // (B) right boundary edges of the strip's rows (lanes 0..7), du = u of the last column
        if (lane < kR) {
            const int il = il0 + lane;
            const float xo = S.rx[il];
            const float xn = right_bnd ? xo : clamp1(cp2_pre(xo, S.uR[il], S.ar[il], tk, ck, ca));
            S.rx[il] = xn;
            S.rxb[il] = fmaf(th, xn - xo, xn);
            if constexpr (ADAPT) conv_acc(xn, xo, dd, nn);
        }
        // row sweep: x_k on the row's edges, xbar_k, and one row behind, u_(k+1)
        float uua = 0.0f, uub = 0.0f;  // u_k of the row above (0 above the tile: one-sided copy)
        if (s > 0) lds_ld2(&S.ut[s - 1][ja], uua, uub);
        float pta = 0.0f, ptb = 0.0f, pla = 0.0f, plb = 0.0f;  // xbar_k on the previous row's top / left edges
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            __builtin_amdgcn_sched_barrier(0);  // one row at a time: bounds the registers in flight
            const int il = il0 + r;
            const float ura = ua[r], urb = ub[r];
            const float ul = from_left(urb);  // u of column a - 1 (lane 0: left of the tile, 0)
            float A1a, A1b, A2a, A2b;
            lds_ld2(&S.a1[il][ja], A1a, A1b);
            lds_ld2(&S.a2[il][ja], A2a, A2b);
            const float o1a = X.e1a[r], o1b = X.e1b[r], o2a = X.e2a[r], o2b = X.e2b[r];
            float l1 = r == 0 ? lo1 : -1.0f, h1 = r == 0 ? hi1 : 1.0f;
            if constexpr (FR) {
                const bool zr = ((c.zrows >> r) & 1u) != 0;
                l1 = zr ? 0.0f : l1;
                h1 = zr ? 0.0f : h1;
            }
            const float n1a = __builtin_amdgcn_fmed3f(cp2_pre(o1a, uua - ura, A1a, tk, ck, ca), l1, h1);
            const float n1b = __builtin_amdgcn_fmed3f(cp2_pre(o1b, uub - urb, A1b, tk, ck, ca), l1, h1);
            const float n2a = __builtin_amdgcn_fmed3f(cp2_pre(o2a, ul - ura, A2a, tk, ck, ca), lo2a, hi2a);
            const float n2b = FR ? __builtin_amdgcn_fmed3f(cp2_pre(o2b, ura - urb, A2b, tk, ck, ca), c.lo2b, c.hi2b)
                                 : clamp1(cp2_pre(o2b, ura - urb, A2b, tk, ck, ca));
            X.e1a[r] = n1a;
            X.e1b[r] = n1b;
            X.e2a[r] = n2a;
            X.e2b[r] = n2b;
            if constexpr (ADAPT) {
                conv_acc(n1a, o1a, dd, nn);
                conv_acc(n1b, o1b, dd, nn);
                conv_acc(n2a, o2a, dd, nn);
                conv_acc(n2b, o2b, dd, nn);
                // the sums are formed here, row by row: left to the compiler they are deferred and
                // keep every row's old and new values alive (register spills)
                asm volatile("" : "+v"(dd), "+v"(nn));
            }
            if (ext) {
                const float b1a = fmaf(th, n1a - o1a, n1a), b1b = fmaf(th, n1b - o1b, n1b);
                const float b2a = fmaf(th, n2a - o2a, n2a), b2b = fmaf(th, n2b - o2b, n2b);
                if (r == 0 && s > 0) lds_st2(&S.xt[s][ja], b1a, b1b);
                if (r > 0) {
                    float da, db;
                    div_pair(pta, ptb, b1a, b1b, pla, plb, S.rxb[il - 1], da, db);
                    ua[r - 1] = cp2_u(fid, ua[r - 1], da, skn, fa[r - 1], observed(2 * r - 2), san, cv1, cv2);
                    ub[r - 1] = cp2_u(fid, ub[r - 1], db, skn, fb[r - 1], observed(2 * r - 1), san, cv1, cv2);
                }
                pta = b1a;
                ptb = b1b;
                pla = b2a;
                plb = b2b;
            }
            uua = ura;
            uub = urb;
            pin4(X.e1a[r], X.e1b[r], X.e2a[r], X.e2b[r]);
        }
        // bottom boundary edges of the tile (strip 15), du = u_k of the last row
        float bxa = 0.0f, bxb = 0.0f;  // their xbar_k
        if (last && !bot_bnd) {
            const float oba = X.ba, obb = X.bb;
            X.ba = clamp1(cp2_pre(oba, ua[kR - 1], S.ab[ja], tk, ck, ca));
            X.bb = clamp1(cp2_pre(obb, ub[kR - 1], S.ab[jb], tk, ck, ca));
            bxa = fmaf(th, X.ba - oba, X.ba);
            bxb = fmaf(th, X.bb - obb, X.bb);
            if constexpr (ADAPT) {
                conv_acc(X.ba, oba, dd, nn);
                conv_acc(X.bb, obb, dd, nn);
            }
        }
        if (ext) {
            __syncthreads();
            // (C) the last row: its bottom edges are the next strip's first-row top edges
            float ba_ = bxa, bb_ = bxb;
            if (!last) lds_ld2(&S.xt[s + 1][ja], ba_, bb_);
            float da, db;
            div_pair(pta, ptb, ba_, bb_, pla, plb, S.rxb[il0 + kR - 1], da, db);
            ua[kR - 1] = cp2_u(fid, ua[kR - 1], da, skn, fa[kR - 1], observed(2 * kR - 2), san, cv1, cv2);
            ub[kR - 1] = cp2_u(fid, ub[kR - 1], db, skn, fb[kR - 1], observed(2 * kR - 1), san, cv1, cv2);
            if constexpr (ADAPT) {
                // the decision is the same in every thread (one FP64 sum in a fixed order)
                if (block_converged(s, lane, dd, nn, a.tol2, S.red)) {
                    taken = k;
                    break;
                }
            }
        }
    }
    if constexpr (ADAPT) {
        if (taken < K) load_u<FR>(c, ua, ub);  // back to u_k: the state of the last step taken
    }
    return taken;
}

}  // namespace cp2tile
}  // namespace dtv
