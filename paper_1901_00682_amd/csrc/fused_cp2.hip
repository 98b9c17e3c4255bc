// Fused schedule of the local accelerated primal-dual solves (Lee & Park,
// arXiv 1901.00682, Sec. 5: Chambolle-Pock Alg. 2 on the local saddle problem
// eq. (local), any fidelity of Sec. 3) on 128 x 128 subdomains, or smaller
// ones whose short sides lie on the image boundary (framed: run in a 128 x 128
// frame): one 1024-thread workgroup owns one subdomain and runs all n_inner
// steps of an outer iteration on chip.
// The on-chip layout and the step are those of cp2_tile.h; this kernel loads
// the tile, updates the multipliers of its interfaces (Algorithm 1, first
// line), forms the anchors from p~^n and lambda^(n+1), solves and stores
// p~^(n+1) into the other edge buffer (a neighbouring tile may still read this
// tile's copies of p~^n for its own multiplier update).
#include "cp2_tile.h"

namespace dtv {

using namespace fused;
using namespace cp2tile;

// FID: the fidelity (0 L2, 1 L1, 2 convex Chan-Vese); MASK: an inpainting mask is given;
// FR: some subdomains are framed tiles (every tile then takes the framed path, which on a
// 128 x 128 tile does what the full-tile path does); ADAPT: adaptive stopping (cp2_tile.h)
template <int FID, bool MASK, bool FR, bool ADAPT = false>
__global__ __launch_bounds__(1024) void k_fused_cp2(FusedCp2Args a)
{
    __shared__ Cp2Lds S;
    __shared__ float LS[4][kFusedMax];  // lambda^(n+1) on the top, bottom, left and right sides
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const SubTile tl = a.subs[t];
    const ImgDev im = a.imgs[tl.img];
    const int s = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform strip index
    const int lane = threadIdx.x & 63;
    const int ja = 2 * lane, jb = ja + 1;
    const int il0 = kR * s;
    const int H = im.H, W = im.W;
    const int h = FR ? tl.h : kFusedMax, w = FR ? tl.w : kFusedMax;
    const bool top_bnd = tl.ra == 0, bot_bnd = tl.ra + h == H;
    const bool left_bnd = tl.ca == 0, right_bnd = tl.ca + w == W;
    const bool last = s == kWaves - 1;
    const long long P1 = im.pitch1, P2 = im.pitch2;
    const long long row1 = (long long)tl.ra + tl.r;  // P1 row of the tile's edge row 0
    const long long col2 = (long long)tl.ca + tl.c;  // P2 column of the tile's edge column 0
    const float *p1_tile = a.p1 + im.p1 + row1 * P1 + tl.ca;
    const float *p2_tile = a.p2 + im.p2 + (long long)tl.ra * P2 + col2;
    float *q1_tile = a.out1 + im.p1 + row1 * P1 + tl.ca;
    float *q2_tile = a.out2 + im.p2 + (long long)tl.ra * P2 + col2;
    const long long px0 = im.px + (long long)tl.ra * W + tl.ca;
    const float *f_tile = a.f + px0;
    float *u_tile = a.u + px0;
    const uint8_t *m_tile = MASK ? a.mask + px0 : nullptr;
    const float tau = a.tau, alpha = im.alpha, cv1 = a.cv_c1, cv2 = a.cv_c2;
    // clamp bounds, (-1, 1) or (0, 0) for edges on the image boundary (no dof)
    const float lo1 = (top_bnd && s == 0) ? 0.0f : -1.0f, hi1 = -lo1;
    const float lo2a = (left_bnd && lane == 0) ? 0.0f : -1.0f, hi2a = -lo2a;

    Slot X;  // x on the owned edges
    float ua[kR], ub[kR], fa[kR], fb[kR];
    float xr[kR];  // lane 63: the right boundary edges of the strip's rows
    unsigned obs = 0xFFFFu;  // observed pixels: bit 2r (column a), 2r + 1 (column b) of row r

    // ---- load p~^n, u, f (every load first, then the conditional ones).  A framed tile loads its
    // own h x w pixels and edges; the rest of the frame starts at 0 (the zeros are written in every
    // lane before the loads, so that no load waits for another lane's load into the same register)
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int il = il0 + r;
        xr[r] = 0.0f;
        if constexpr (FR) {
            X.e1a[r] = X.e1b[r] = X.e2a[r] = X.e2b[r] = 0.0f;
            fa[r] = fb[r] = ua[r] = ub[r] = 0.0f;
            pin4(X.e1a[r], X.e1b[r], X.e2a[r], X.e2b[r]);
            pin4(fa[r], fb[r], ua[r], ub[r]);
        }
        if (!FR || (il < h && ja + 1 < w)) {
            ld2g(p1_tile + (long long)il * P1 + ja, X.e1a[r], X.e1b[r]);
            ld2g(p2_tile + (long long)il * P2 + ja, X.e2a[r], X.e2b[r]);
            ld2g(f_tile + (long long)il * W + ja, fa[r], fb[r]);
            ld2g(u_tile + (long long)il * W + ja, ua[r], ub[r]);
        } else if (il < h && ja < w) {  // framed: the tile's last column alone
            X.e1a[r] = p1_tile[(long long)il * P1 + ja];
            X.e2a[r] = p2_tile[(long long)il * P2 + ja];
            fa[r] = f_tile[(long long)il * W + ja];
            ua[r] = u_tile[(long long)il * W + ja];
        }
    }
    X.ba = X.bb = 0.0f;
    if (last && (!FR || (h == kFusedMax && ja + 1 < w))) ld2g(p1_tile + (long long)kFusedMax * P1 + ja, X.ba, X.bb);
    else if (FR && last && h == kFusedMax && ja < w) X.ba = p1_tile[(long long)kFusedMax * P1 + ja];
    if (lane == 63 && (!FR || w == kFusedMax))
#pragma unroll
        for (int r = 0; r < kR; ++r)
            if (!FR || il0 + r < h) xr[r] = p2_tile[(long long)(il0 + r) * P2 + kFusedMax];
    if constexpr (MASK) {
        obs = 0;  // (a framed tile: the pixels outside it are unobserved)
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            if (FR && il0 + r >= h) continue;
            const uint8_t *mr = m_tile + (long long)(il0 + r) * W + ja;
            if (!FR || ja < w) obs |= (mr[0] != 0 ? 1u : 0u) << (2 * r);
            if (!FR || ja + 1 < w) obs |= (mr[1] != 0 ? 1u : 0u) << (2 * r + 1);
        }
    }

    // ---- (a1) lambda^(n+1) = lambda^n + sigma [(2 p_s^n - p_s^(n-1)) - (2 p_t^n - p_t^(n-1))] on the
    // tile's interface edges, with the operations of the multiplier kernel (the two tiles of an
    // interface compute the same value).  Waves 0..7 take the top, bottom, left and right sides
    // (two waves each, edge si = 64 (wave % 2) + lane).  The new lambda state goes to lam_out:
    // lambda^(n+1) and p_s^n by the s side (bottom, right), p_t^n by the t side (top, left).
    {
        const int side = s >> 1, si = (s & 1) * 64 + lane;
        bool has = false;
        long long e = 0, ips = 0, ipt = 0;  // lambda index; P1 or P2 offsets of the s and t copies
        if (s < 2 * 4 && (!FR || si < (side < 2 ? w : h))) {
            const long long rs = (long long)(tl.ra + si) * P2;  // P2 row of a left / right edge
            switch (side) {
            case 0:  // top: the tile above holds the s copy
                has = tl.r > 0;
                e = (long long)(tl.r - 1) * W + tl.ca + si;
                ips = (row1 - 1) * P1 + tl.ca + si;
                ipt = row1 * P1 + tl.ca + si;
                break;
            case 1:  // bottom: the tile below holds the t copy
                has = !bot_bnd;
                e = (long long)tl.r * W + tl.ca + si;
                ips = (row1 + kFusedMax) * P1 + tl.ca + si;
                ipt = (row1 + kFusedMax + 1) * P1 + tl.ca + si;
                break;
            case 2:  // left: the tile on the left holds the s copy
                has = tl.c > 0;
                e = im.nlh + (long long)(tl.c - 1) * H + tl.ra + si;
                ips = rs + col2 - 1;
                ipt = rs + col2;
                break;
            default:  // right: the tile on the right holds the t copy
                has = !right_bnd;
                e = im.nlh + (long long)tl.c * H + tl.ra + si;
                ips = rs + col2 + kFusedMax;
                ipt = rs + col2 + kFusedMax + 1;
                break;
            }
        }
        if (has) {
            const float *pp = side < 2 ? a.p1 + im.p1 : a.p2 + im.p2;
            const float ps = pp[ips], pt = pp[ipt];
            const float *Li = a.lam + im.lam;
            float *Lo = a.lam_out + im.lam;
            const long long nl = im.nlam;
            const float l1 = Li[e] + a.sigma * ((2.0f * ps - Li[nl + e]) - (2.0f * pt - Li[2 * nl + e]));
            LS[side][si] = l1;
            if (side == 1 || side == 3) {
                Lo[e] = l1;
                Lo[nl + e] = ps;
            } else {
                Lo[2 * nl + e] = pt;
            }
        }
    }
    __syncthreads();

    // ---- (a2) anchors phat = p~^n, with +tau lambda^(n+1) on the t copies (top edges below an
    // interface, left edges right of one) and -tau lambda^(n+1) on the s copies (bottom, right)
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int il = il0 + r;
        float a1a = X.e1a[r], a1b = X.e1b[r], a2a = X.e2a[r];
        if (il == 0 && tl.r > 0) {
            if (!FR || ja < w) a1a = fmaf(tau, LS[0][ja], a1a);
            if (!FR || jb < w) a1b = fmaf(tau, LS[0][jb], a1b);
        }
        if (ja == 0 && tl.c > 0 && (!FR || il < h)) a2a = fmaf(tau, LS[2][il], a2a);
        lds_st2(&S.a1[il][ja], a1a, a1b);
        lds_st2(&S.a2[il][ja], a2a, X.e2b[r]);
    }
    if (last) {
        float aba = X.ba, abb = X.bb;
        if (!bot_bnd) {  // (lambda exists on the tile's own columns only)
            if (!FR || ja < w) aba = fmaf(-tau, LS[1][ja], aba);
            if (!FR || jb < w) abb = fmaf(-tau, LS[1][jb], abb);
        }
        S.ab[ja] = aba;
        S.ab[jb] = abb;
    }
    if (lane == 63)
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int il = il0 + r;
            S.rx[il] = xr[r];
            float ar = xr[r];
            if (!right_bnd && (!FR || il < h)) ar = fmaf(-tau, LS[3][il], ar);
            S.ar[il] = ar;
        }
    // ---- (a3) the local solve
    Cp2Ctx cx;
    cx.s = s;
    cx.lane = lane;
    cx.ja = ja;
    cx.jb = jb;
    cx.il0 = il0;
    cx.last = last;
    cx.bot_bnd = bot_bnd;
    cx.right_bnd = right_bnd;
    cx.lo1 = lo1;
    cx.hi1 = hi1;
    cx.lo2a = lo2a;
    cx.hi2a = hi2a;
    cx.alpha = alpha;
    cx.cv1 = cv1;
    cx.cv2 = cv2;
    cx.lo2b = -1.0f;
    cx.hi2b = 1.0f;
    cx.zrows = 0u;
    if constexpr (FR) {
        // the boundary lines of a framed tile (the left edges of column w, the top edges of row h);
        // the frame's bottom row and right column lie outside a tile shorter or narrower than it
        const bool za = w < kFusedMax && ja == w, zb = w < kFusedMax && jb == w;
        cx.lo2a = za ? 0.0f : cx.lo2a;
        cx.hi2a = za ? 0.0f : cx.hi2a;
        cx.lo2b = zb ? 0.0f : -1.0f;
        cx.hi2b = zb ? 0.0f : 1.0f;
        const int zr = h - il0;
        cx.zrows = (h < kFusedMax && zr >= 0 && zr < kR) ? 1u << zr : 0u;
        cx.bot_bnd = bot_bnd || h < kFusedMax;
        cx.right_bnd = right_bnd || w < kFusedMax;
    }
    cx.u_tile = u_tile;
    cx.W = W;
    cx.h = h;
    cx.w = w;
    const int taken = solve<FID, FR, ADAPT>(cx, S, X, ua, ub, fa, fb, obs, a);
    if constexpr (ADAPT) {
        if (threadIdx.x == 0) {  // the subdomain's only workgroup of this launch
            int *cnt = a.counts + 2 * (long long)t;
            cnt[0] += taken;
            cnt[1] = max(cnt[1], taken);
        }
    }

    // ---- store x_K as p~^(n+1) and u_K
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int il = il0 + r;
        if (!FR || (il < h && ja + 1 < w)) {
            st2g(q1_tile + (long long)il * P1 + ja, X.e1a[r], X.e1b[r]);
            st2g(q2_tile + (long long)il * P2 + ja, X.e2a[r], X.e2b[r]);
            st2g(u_tile + (long long)il * W + ja, ua[r], ub[r]);
        } else if (il < h && ja < w) {  // framed: the tile's last column alone
            q1_tile[(long long)il * P1 + ja] = X.e1a[r];
            q2_tile[(long long)il * P2 + ja] = X.e2a[r];
            u_tile[(long long)il * W + ja] = ua[r];
        }
        // the frame's right column and bottom row: a framed tile's own only when it spans the frame
        if (lane == 63 && (!FR || (w == kFusedMax && il < h))) q2_tile[(long long)il * P2 + kFusedMax] = S.rx[il];
    }
    if (last && (!FR || (h == kFusedMax && ja + 1 < w))) st2g(q1_tile + (long long)kFusedMax * P1 + ja, X.ba, X.bb);
    else if (FR && last && h == kFusedMax && ja < w) q1_tile[(long long)kFusedMax * P1 + ja] = X.ba;
}

namespace {

template <int FID, bool MASK>
hipError_t launch_cp2_variant(const FusedCp2Args &a, int nsub, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    const bool adapt = a.tol2 > 0.0;
    auto k = a.frames ? (adapt ? k_fused_cp2<FID, MASK, true, true> : k_fused_cp2<FID, MASK, true, false>)
                      : (adapt ? k_fused_cp2<FID, MASK, false, true> : k_fused_cp2<FID, MASK, false, false>);
    if (e0)
        hipExtLaunchKernelGGL(k, dim3(nsub), dim3(1024), 0, s, e0, e1, 0, a);
    else
        hipLaunchKernelGGL(k, dim3(nsub), dim3(1024), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fused_cp2(const FusedCp2Args &a, int nsub, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (nsub <= 0) return hipSuccess;
    const bool adapt = a.tol2 > 0.0;
    if (a.n_inner < 1 || a.n_inner > (adapt ? kMaxAdaptiveInner : kMaxFusedInner)) return hipErrorInvalidValue;
    if (adapt && (!a.tab || !a.counts)) return hipErrorInvalidValue;
    // p~^(n+1) and the new lambda state go to buffers of their own: other tiles read p~^n and
    // lambda^n (without interfaces there is no lambda state)
    if (!a.out1 || !a.out2 || a.out1 == a.p1 || a.out2 == a.p2 || (a.lam && a.lam_out == a.lam))
        return hipErrorInvalidValue;
    const bool m = a.mask != nullptr;
    switch (a.fidelity) {
    case 0: return m ? launch_cp2_variant<0, true>(a, nsub, s, e0, e1) : launch_cp2_variant<0, false>(a, nsub, s, e0, e1);
    case 1: return m ? launch_cp2_variant<1, true>(a, nsub, s, e0, e1) : launch_cp2_variant<1, false>(a, nsub, s, e0, e1);
    case 2: return m ? hipErrorInvalidValue : launch_cp2_variant<2, false>(a, nsub, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace dtv
