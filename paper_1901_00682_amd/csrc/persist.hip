// Persistent schedule of Algorithm 1 (Lee & Park, arXiv 1901.00682) for ROF
// with FISTA local solves: one cooperative launch runs every outer step.
//
// Each workgroup owns one 128 x 128 subdomain (or a framed one: any smaller
// subdomain, held in a 128 x 128 frame) for the whole solve; its iterate stays in VGPRs (the slots of the fused kernel) from
// the first outer step to the last, so p~ crosses HBM twice per solve instead
// of twice per outer step.  The images of a plan whose subdomains do not all
// fit on the device at once run as groups of launches.  Per outer step n:
//   (1) each tile forms q = 2 p^n - p^(n-1) on its own interface copies (the
//       extrapolated copies of the multiplier update) and publishes them;
//   (4a) meanwhile it rebuilds c' of every edge but the interface copies from
//       the anchor p^n and f (fista_ops.h);
//   (2) it waits for the copies its neighbours publish on the same edges;
//   (3) both tiles of an interface edge compute lambda^(n+1) = lambda^n +
//       sigma (q_s - q_t) from the two copies, with the operations of the
//       multiplier-update kernel, so both hold the same value;
//   (4b) c' of the interface copies from phat = p^n -/+ tau lambda^(n+1);
//   (5) the n_inner FISTA steps of the fused kernel (full_step).
// Two workgroup barriers per outer step besides the steps' own: after the
// staging of the copies (1) and before the steps (5).
// lambda^n and the tile's own previous copies live in LDS.
//
// Synchronisation is point to point, between the two tiles of an interface:
// every copy travels in a 64-bit word that also holds n + 1, written and
// polled with relaxed agent-scope atomics, so a word is valid exactly when its
// step number matches and no fence or grid-wide barrier is needed (an
// agent-scope fence writes back and invalidates a whole L2).  The words
// alternate between two slots by step parity; a tile overwrites slot n % 2 at
// step n + 2 only after it has read its neighbour's step n + 1 copy, which
// the neighbour publishes only after reading the step n word.  The
// cooperative launch keeps every tile resident, so every wait can end.
//
// The arithmetic per edge and per multiplier is that of the fused and
// streaming schedules, so all three give bitwise identical results.
#include "exchange.h"
#include "fused_common.h"

namespace dtv {

using namespace fused;
using namespace xchg;

namespace {

struct PersistLds {
    FusedLds f;
    float lam[kSides][kFusedMax];  // lambda on the tile's interface edges
    float prv[kSides][kFusedMax];  // the tile's own copies on those edges at the previous outer step
    double red[2 * kWaves];        // adaptive stopping: the per-wave sums of the relative-change test
    int ok;                        // every wait of the current step completed
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

}  // namespace

// The whole solve of subdomain t.  KF > 0: n_inner = KF (steps unrolled); KF = 0: any n_inner.
// ADAPT (KF = 0): each local solve stops by the relative-change rule (fused_common.h,
// a.fa.tol2, cap n_inner), full or framed tiles; the steps taken are counted per subdomain.  FR: a framed tile, smaller
// than 128 x 128 (full_step<.., FR> in a 128 x 128 frame, with p~ and f zero outside the tile):
// FR = 1 with its short sides on the image boundary, FR = 2 for any tile, whose bottom edges then
// lie in frame row h and its right edges in frame column w, interface copies or not.
template <int KF, bool ADAPT, int FR>
__device__ __forceinline__ void persist_tile(const PersistArgs &a, PersistLds &L, int t)
{
    FusedLds &S = L.f;
    const SubTile tl = a.fa.subs[t];
    const ImgDev im = a.fa.imgs[tl.img];
    const int h = FR ? tl.h : kFusedMax, w = FR ? tl.w : kFusedMax;
    const int s = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // strip (wave) index
    const int lane = threadIdx.x & 63;
    const int ja = 2 * lane, il0 = kR * s;
    const int H = im.H, W = im.W;
    const bool top_bnd = tl.ra == 0, bot_bnd = tl.ra + h == H;
    const bool left_bnd = tl.ca == 0, right_bnd = tl.ca + w == W;
    const long long P1 = im.pitch1, P2 = im.pitch2;
    const long long row1 = (long long)tl.ra + tl.r;  // P1 row of the tile's edge row 0
    const long long col2 = (long long)tl.ca + tl.c;  // P2 column of the tile's edge column 0
    const float tau = a.fa.tau, itau = a.fa.inv_tau, invL = im.invL;
    const float *f_tile = a.fa.f + im.px + (long long)tl.ra * W + tl.ca;
    const long long nlam = im.nlam;

    FullCtx fc;
    fc.s = s;
    fc.lane = lane;
    fc.ja = ja;
    fc.il0 = il0;
    fc.oc = il0 * kFusedMax + ja;
    fc.oy = s * kFusedMax + ja;
    fc.olr = il0 + lane;
    fc.last = s == kWaves - 1;
    fc.right_bnd = right_bnd;
    {
        const bool tb = top_bnd && s == 0, lb = left_bnd && lane == 0;
        fc.lo1 = tb ? 0.0f : -1.0f;
        fc.hi1 = tb ? 0.0f : 1.0f;
        fc.lo2a = lb ? 0.0f : -1.0f;
        fc.hi2a = lb ? 0.0f : 1.0f;
        fc.lob = bot_bnd ? 0.0f : -1.0f;
        fc.hib = bot_bnd ? 0.0f : 1.0f;
    }
    fc.ak = im.a_keep;
    fc.kL = im.kL;
    fc.lo2b = -1.0f;
    fc.hi2b = 1.0f;
    fc.zrows = 0u;
    fc.mrows = 0xFFu;
    fc.lva = fc.lvb = true;
    if constexpr (FR) {
        // the boundary lines of a framed tile: the left edges of column w, the top edges of row h;
        // clamped when on the image boundary (always, without masks)
        const bool rz = FR == 1 || right_bnd, bz = FR == 1 || bot_bnd;
        const bool za = rz && w < kFusedMax && ja == w, zb = rz && w < kFusedMax && ja + 1 == w;
        fc.lo2a = za ? 0.0f : fc.lo2a;
        fc.hi2a = za ? 0.0f : fc.hi2a;
        fc.lo2b = zb ? 0.0f : -1.0f;
        fc.hi2b = zb ? 0.0f : 1.0f;
        const int zr = h - il0;
        fc.zrows = (bz && h < kFusedMax && zr >= 0 && zr < kR) ? 1u << zr : 0u;
        fc.right_bnd = right_bnd || w < kFusedMax;  // the frame's right column lies outside the tile
        // the pixels inside the tile: rows il0 .. h - 1 of the strip, columns below w
        fc.mrows = zr >= kR ? 0xFFu : zr <= 0 ? 0u : (1u << zr) - 1u;
        fc.lva = ja < w;
        fc.lvb = ja + 1 < w;
    }
    // with masks, the tile's bottom edges lie in frame row h and its right edges in frame column w
    // when the tile is shorter or narrower than the frame
    const bool in_row = FR == 2 && h < kFusedMax, in_col = FR == 2 && w < kFusedMax;

    // side work (multiplier update): waves 0..7, side = wave / 2 (wave-uniform), edge
    // si = 64 (wave % 2) + lane; the lambda index is side_base + si.  A framed tile's sides are
    // shorter than 128 (lanes beyond the side's length idle).
    const int side = s >> 1;
    const bool side_wave = s < 2 * kSides && side_exists(im, tl, side);
    const bool side_lane = side_wave && (s & 1) * 64 + lane < (side < 2 ? w : h);
    const bool side_s = side == 1 || side == 3;  // s copies: bottom and right sides
    const long long side_base = side_wave ? side_edge(im, tl, side, 0) : 0;

    // ---- load p~^0 (slot A, right boundary column in LDS) and the lambda state
    Slot A, B;
    A.ba = A.bb = 0.0f;
    {
        const float *p1_tile = a.fa.base1 + im.p1 + row1 * P1 + tl.ca;
        const float *p2_tile = a.fa.base2 + im.p2 + (long long)tl.ra * P2 + col2;
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int il = il0 + r;
            A.e1a[r] = A.e1b[r] = A.e2a[r] = A.e2b[r] = 0.0f;
            if (!FR || (il < h && ja + 1 < w)) {
                ld2g(p1_tile + (long long)il * P1 + ja, A.e1a[r], A.e1b[r]);
                ld2g(p2_tile + (long long)il * P2 + ja, A.e2a[r], A.e2b[r]);
            } else if (il < h && ja < w) {  // framed: the tile's last column alone
                A.e1a[r] = p1_tile[(long long)il * P1 + ja];
                if (in_col && ja + 1 == w) ld2g(p2_tile + (long long)il * P2 + ja, A.e2a[r], A.e2b[r]);
                else A.e2a[r] = p2_tile[(long long)il * P2 + ja];
            } else if (in_col && il < h && ja == w) {  // the right edges in column w
                A.e2a[r] = p2_tile[(long long)il * P2 + ja];
            } else if (in_row && il == h) {  // the bottom edges in row h
                if (ja + 1 < w) ld2g(p1_tile + (long long)il * P1 + ja, A.e1a[r], A.e1b[r]);
                else if (ja < w) A.e1a[r] = p1_tile[(long long)il * P1 + ja];
            }
        }
        if (fc.last && (!FR || (h == kFusedMax && ja + 1 < w))) {
            ld2g(p1_tile + (long long)kFusedMax * P1 + ja, A.ba, A.bb);
        } else if (fc.last && h == kFusedMax && ja < w) {  // framed: the tile's last column alone
            A.ba = p1_tile[(long long)kFusedMax * P1 + ja];
        }
        if (lane < kR)
            S.rx[0][il0 + lane] = (!FR || (w == kFusedMax && il0 + lane < h))
                                      ? p2_tile[(long long)(il0 + lane) * P2 + kFusedMax]
                                      : 0.0f;
    }
    if (side_lane) {
        const int si = (s & 1) * 64 + lane;
        const float *ls = a.fa.lam + im.lam + side_base;
        L.lam[side][si] = ls[si];
        L.prv[side][si] = ls[(side_s ? nlam : 2 * nlam) + si];
    }
    if constexpr (FR == 1) {
        // c' on the frame's first row and column outside the tile (the rebuild below skips the
        // whole row or column when the tile's side there is an interface); ordered before the
        // loop's writes by its first barrier
        if (s == 0) lds_st2(&S.c1[0][ja], 0.0f, 0.0f);
        if (lane == 0)
#pragma unroll
            for (int r = 0; r < kR; ++r) S.c2[il0 + r][0] = 0.0f;
    }
    if constexpr (FR != 0) {
        // c' of the frame's right column below the tile and of its bottom row right of the tile: the
        // rebuild below never writes them when the tile's side there is an interface (it writes the
        // tile's own copies only).  At 0 the edges there stay 0: they cannot reach the tile either
        // way, but the stopping rule sums every edge of the frame.
        if (lane < kR && il0 + lane >= h) S.cr[il0 + lane] = 0.0f;
        if (s == 0) {
            if (ja >= w) S.cb[ja] = 0.0f;
            if (ja + 1 >= w) S.cb[ja + 1] = 0.0f;
        }
    }
    int rx_slot = 0;  // LDS slot of the right boundary column holding the current iterate
    bool ok = true;
    int steps_total = 0, steps_max = 0;  // adaptive stopping: local steps of this subdomain

    for (int n = 0; n < a.n_outer; ++n) {
        // ---- f of the strip's rows for the rebuild of c' (4a), issued first so that the loads
        // travel during the staging and the publication (the second iterate slot is dead here)
        // per outer step, so that the row addresses are formed here and not hoisted out of the loop
        const int jo = opaque(ja);
        // (a framed tile: 0 outside it.  The zeros are written in every lane before the loads
        // (pinned there): a zero written in the lanes that skip a load would otherwise wait for
        // the other lanes' load into the same register, and the loads would not overlap)
        float fra[kR], frb[kR];
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            fra[r] = frb[r] = 0.0f;
            if constexpr (FR != 0) pin4(fra[r], frb[r], fra[r], frb[r]);
            if (!FR || (il0 + r < h && ja + 1 < w)) ld2g(f_tile + (long long)(il0 + r) * W + jo, fra[r], frb[r]);
            else if (il0 + r < h && ja < w) fra[r] = f_tile[(long long)(il0 + r) * W + jo];
        }
        float fua = 0.0f, fub = 0.0f;  // f of the row above (0 above the tile)
        if constexpr (FR != 0) pin4(fua, fub, fua, fub);
        if (il0 > 0 && (!FR || (il0 - 1 < h && ja + 1 < w))) ld2g(f_tile + (long long)(il0 - 1) * W + jo, fua, fub);
        else if (FR && il0 > 0 && il0 - 1 < h && ja < w) fua = f_tile[(long long)(il0 - 1) * W + jo];

        // ---- (1) stage the current iterate on the top, bottom and left sides.  The staging rows
        // are LDS rows that the steps write but never read, so no barrier has to separate these
        // stores from the last step's reads: d of strip 15's last row (no strip below reads it),
        // the parity-0 top-edge row of strip 0 (no strip above reads it), and the last column's d
        // (each wave's own rows, written and read by that wave alone).
        if (s == 0) lds_st2(&S.dl[kWaves - 1][ja], A.e1a[0], A.e1b[0]);
        if (!in_row && fc.last) lds_st2(&S.yt[0][0][ja], A.ba, A.bb);
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < kR; ++r) S.dR[il0 + r] = A.e2a[r];
        }
        if constexpr (FR == 2) {
            // the bottom edges from row h, the right edges from column w (the parity-1 top-edge row
            // of strip 0, also written by the steps and never read)
            if (in_row && h >= il0 && h < il0 + kR) {  // the strip holding row h
#pragma unroll
                for (int r = 0; r < kR; ++r)
                    if (il0 + r == h) lds_st2(&S.yt[0][0][ja], A.e1a[r], A.e1b[r]);
            }
            if (in_col && ja == (w & ~1) && il0 < h) {  // the lane holding column w
                const bool odd = (w & 1) != 0;
#pragma unroll
                for (int r = 0; r < kR; ++r)
                    if (il0 + r < h) S.yt[1][0][il0 + r] = odd ? A.e2b[r] : A.e2a[r];
            }
        }
        if (threadIdx.x == 0) L.ok = 1;
        __syncthreads();
        // ---- (1b) publish q = 2 p^n - p^(n-1) on the tile's interface copies
        const int si = (s & 1) * 64 + opaque(lane);
        unsigned long long *xch = a.xch + (long long)(n & 1) * a.xch_stride + im.lam + side_base + si;
        float x_side = 0.0f, q_own = 0.0f;
        if (side_lane) {
            x_side = side == 3 ? (in_col ? S.yt[1][0][si] : S.rx[rx_slot][si])
                     : side == 0 ? S.dl[kWaves - 1][si] : side == 1 ? S.yt[0][0][si] : S.dR[si];
            q_own = 2.0f * x_side - L.prv[side][si];
            L.prv[side][si] = x_side;
            publish(xch + (side_s ? 0 : nlam), q_own, n);
        }
        // the right boundary column of the iterate goes to slot 0 (the first step reads it there)
        if (rx_slot == 1 && lane < kR) S.rx[0][il0 + lane] = S.rx[1][il0 + lane];

        // ---- (4a) while the neighbours' copies travel: c' of every edge from the anchor p^n and f,
        // as in the fused kernel's prologue, except the interface copies, which (4b) writes once
        // lambda^(n+1) is known; the two phases write disjoint entries, so no barrier separates them.
        // Every entry of a frame is written (0 outside the tile); without masks, the entries of the
        // first row and column outside the tile keep the zeros written before the loop.
        {
            const bool top_if = side_exists(im, tl, 0), bot_if = side_exists(im, tl, 1);
            const bool left_if = side_exists(im, tl, 2), right_if = side_exists(im, tl, 3);
            // a pair of entries, either of which may be an interface copy ((4b) writes those)
            auto st_pair = [](float *p, float x, float y, bool skx, bool sky) {
                if (!skx && !sky) lds_st2(p, x, y);
                else if (!skx) p[0] = x;
                else if (!sky) p[1] = y;
            };
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const int il = il0 + r;
                const float fva = fra[r], fvb = frb[r];
                const float fla = from_left(fvb);  // f of column a - 1 (lane 0: left of the tile, 0)
                // the interface rows: row 0 (top), row h < 128 (bottom, with masks); columns below w
                const bool if_row = (il == 0 && top_if) || (in_row && il == h && bot_if);
                const float c1a = fista_cprime(A.e1a[r], fua, fva, itau, invL);
                const float c1b = fista_cprime(A.e1b[r], fub, fvb, itau, invL);
                if (!if_row) lds_st2(&S.c1[il][ja], c1a, c1b);
                else if (FR == 2) st_pair(&S.c1[il][ja], c1a, c1b, ja < w, ja + 1 < w);  // outside the tile
                // the interface columns: column 0 (left), column w < 128 (right, with masks); rows below h
                const float c2a = fista_cprime(A.e2a[r], ja > 0 ? fla : 0.0f, fva, itau, invL);
                const float c2b = fista_cprime(A.e2b[r], fva, fvb, itau, invL);
                const bool if_a = il < h && ((ja == 0 && left_if) || (in_col && ja == w && right_if));
                const bool if_b = in_col && il < h && ja + 1 == w && right_if;
                if (FR < 2) {
                    if (ja == 0 && left_if) S.c2[il][1] = c2b;
                    else lds_st2(&S.c2[il][ja], c2a, c2b);
                } else {
                    if (!(if_a || if_b)) lds_st2(&S.c2[il][ja], c2a, c2b);
                    else st_pair(&S.c2[il][ja], c2a, c2b, if_a, if_b);
                }
                // the frame's bottom edges and right column: the tile's boundary edges on the image
                // boundary, or (framed) outside the tile
                if (il == kFusedMax - 1 && (!bot_if || in_row))
                    lds_st2(&S.cb[ja], fista_cprime(A.ba, fva, 0.0f, itau, invL),
                            fista_cprime(A.bb, fvb, 0.0f, itau, invL));
                if (lane == 63 && (!right_if || in_col))
                    S.cr[il] = fista_cprime(S.rx[0][il], fvb, 0.0f, itau, invL);
                fua = fva;
                fub = fvb;
            }
        }

        // ---- (2) the neighbour's copy of each interface edge, (3) lambda^(n+1), (4b) c' of the
        // interface copies from phat = p^n -/+ tau lambda^(n+1) (t copies +, s copies -)
        if (side_lane) {
            // the pixel of the tile next to the edge (its f enters the edge's c')
            const int pi = side == 0 ? 0 : side == 1 ? h - 1 : si;
            const int pj = side == 2 ? 0 : side == 3 ? w - 1 : si;
            const float fp = f_tile[(long long)pi * W + pj];
            float q_oth = 0.0f;
            if (fetch(xch + (side_s ? nlam : 0), n, q_oth, a.spin_limit)) {
                const float qs = side_s ? q_own : q_oth, qt = side_s ? q_oth : q_own;
                const float lam = L.lam[side][si] + a.sigma * (qs - qt);
                L.lam[side][si] = lam;
                if (side == 0) S.c1[0][si] = fista_cprime(fmaf(tau, lam, x_side), 0.0f, fp, itau, invL);
                else if (side == 2) S.c2[si][0] = fista_cprime(fmaf(tau, lam, x_side), 0.0f, fp, itau, invL);
                else if (side == 1)
                    (in_row ? S.c1[h][si] : S.cb[si]) = fista_cprime(fmaf(-tau, lam, x_side), fp, 0.0f, itau, invL);
                else
                    (in_col ? S.c2[si][w] : S.cr[si]) = fista_cprime(fmaf(-tau, lam, x_side), fp, 0.0f, itau, invL);
            } else {
                L.ok = 0;
                atomicOr(a.err, 1);
            }
        }
        __syncthreads();
        ok = L.ok != 0;
        if (!ok) break;  // a neighbour stopped publishing: leave (the host reports the error)

        // ---- (5) the local FISTA solves
        if constexpr (ADAPT) {
            int taken = 0;
            if constexpr (FR)
                rx_slot = run_steps_adaptive<FramedStep<FR>>(fc, S, A, B, a.fa.n_inner, a.fa.beta_dev, a.fa.tol2, L.red,
                                                             taken);
            else
                rx_slot = run_steps_adaptive<FullStep>(fc, S, A, B, a.fa.n_inner, a.fa.beta_dev, a.fa.tol2, L.red,
                                                       taken);
            steps_total += taken;
            steps_max = max(steps_max, taken);
        } else if constexpr (KF > 0) {
            rx_slot = full_steps_fixed<KF, false, FR>(fc, S, A, B, a.fa.beta);
            if constexpr (KF & 1) copy_slot(A, B);
        } else if constexpr (FR) {
            rx_slot = run_steps<FramedStep<FR>>(fc, S, A, B, a.fa.n_inner, a.fa.beta);
        } else {
            rx_slot = run_steps<FullStep>(fc, S, A, B, a.fa.n_inner, a.fa.beta);
        }
    }

    // ---- store p~^N and the lambda state (lambda^N and the copies of the last multiplier update)
    __syncthreads();
    {
        float *q1_tile = a.fa.out1 + im.p1 + row1 * P1 + tl.ca;
        float *q2_tile = a.fa.out2 + im.p2 + (long long)tl.ra * P2 + col2;
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int il = il0 + r;
            if (!FR || (il < h && ja + 1 < w)) {
                st2g(q1_tile + (long long)il * P1 + ja, A.e1a[r], A.e1b[r]);
                st2g(q2_tile + (long long)il * P2 + ja, A.e2a[r], A.e2b[r]);
            } else if (il < h && ja < w) {  // framed: the tile's last column alone
                q1_tile[(long long)il * P1 + ja] = A.e1a[r];
                if (in_col && ja + 1 == w) st2g(q2_tile + (long long)il * P2 + ja, A.e2a[r], A.e2b[r]);
                else q2_tile[(long long)il * P2 + ja] = A.e2a[r];
            } else if (in_col && il < h && ja == w) {  // the right edges in column w
                q2_tile[(long long)il * P2 + ja] = A.e2a[r];
            } else if (in_row && il == h) {  // the bottom edges in row h
                if (ja + 1 < w) st2g(q1_tile + (long long)il * P1 + ja, A.e1a[r], A.e1b[r]);
                else if (ja < w) q1_tile[(long long)il * P1 + ja] = A.e1a[r];
            }
        }
        // the frame's bottom row and right column: a framed tile's own only when it spans the frame
        if (fc.last && (!FR || (h == kFusedMax && ja + 1 < w)))
            st2g(q1_tile + (long long)kFusedMax * P1 + ja, A.ba, A.bb);
        else if (fc.last && h == kFusedMax && ja < w)
            q1_tile[(long long)kFusedMax * P1 + ja] = A.ba;
        if (lane < kR && (!FR || (w == kFusedMax && il0 + lane < h)))
            q2_tile[(long long)(il0 + lane) * P2 + kFusedMax] = S.rx[rx_slot][il0 + lane];
    }
    if constexpr (ADAPT) {
        if (threadIdx.x == 0) {  // the subdomain's only workgroup (adaptive: one launch, the plan's list)
            int *cnt = a.fa.counts + 2 * (long long)t;
            cnt[0] += steps_total;
            cnt[1] = max(cnt[1], steps_max);
        }
    }
    if (side_lane && ok) {
        const int si = (s & 1) * 64 + lane;
        float *ls = a.lam_out + im.lam + side_base;
        if (side_s) {
            ls[si] = L.lam[side][si];
            ls[nlam + si] = L.prv[side][si];
        } else {
            ls[2 * nlam + si] = L.prv[side][si];
        }
    }
}

// Every outer step of the subdomains subs[0, gridDim.x) in one cooperative launch, one
// workgroup per subdomain.  FRAMES > 0: some of them are framed tiles (smaller than 128 x 128,
// FRAMES = 1 when all of those have their short sides on the image boundary, 2 otherwise); then
// every tile takes the framed path, which on a 128 x 128 tile does what the full-tile path does
// (one path per kernel keeps the registers of the other out of its loop).
template <int KF, bool ADAPT = false, int FRAMES = 0>
__global__ __launch_bounds__(1024) void k_persist_fista(PersistArgs a)
{
    __shared__ PersistLds L;
    persist_tile<KF, ADAPT, FRAMES>(a, L, xcd_remap(blockIdx.x, gridDim.x));
}

bool persist_supported(int device)
{
    int coop = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess) return false;
    return coop != 0;
}

namespace {

using PersistKernel = void (*)(PersistArgs);

// kernels with the inner step count unrolled, for the common counts
template <int... Ks>
struct PersistTable {
    template <int FRM>
    static PersistKernel get(int K)
    {
        PersistKernel k = nullptr;
        ((K == Ks ? (k = k_persist_fista<Ks, false, FRM>, 0) : 0), ...);
        return k ? k : k_persist_fista<0, false, FRM>;
    }
    static PersistKernel get(int K, int frames)
    {
        return frames == 2 ? get<2>(K) : frames == 1 ? get<1>(K) : get<0>(K);
    }
};
using Persist = PersistTable<1, 2, 3, 4, 5, 6, 7, 8, 10>;

}  // namespace

int persist_capacity(int device)
{
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist_fista<0>, 1024, 0) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    return per_cu * cus;
}

hipError_t launch_persist_fista(const PersistArgs &a, int nsub, int frames, hipStream_t s)
{
    if (nsub <= 0 || a.n_outer <= 0) return hipSuccess;
    const bool adapt = a.fa.tol2 > 0.0;
    if (a.fa.n_inner < 1 || a.fa.n_inner > (adapt ? kMaxAdaptiveInner : kMaxFusedInner)) return hipErrorInvalidValue;
    if (adapt && (!a.fa.beta_dev || !a.fa.counts)) return hipErrorInvalidValue;
    PersistArgs arg = a;
    void *args[] = {&arg};
    if (frames < 0 || frames > 2) return hipErrorInvalidValue;
    const PersistKernel k = !adapt ? Persist::get(a.fa.n_inner, frames)
                            : frames == 2 ? k_persist_fista<0, true, 2>
                            : frames == 1 ? k_persist_fista<0, true, 1>
                                          : k_persist_fista<0, true, 0>;
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k), dim3(nsub), dim3(1024), args, 0, s);
}

}  // namespace dtv
