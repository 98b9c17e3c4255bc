// Fused schedule of the local FISTA solves (Lee & Park, arXiv 1901.00682,
// Algorithm 1, the "in parallel" local problems of eq. DD_local_dual for ROF):
// one 1024-thread workgroup owns one subdomain of at most 128 x 128 pixels
// and runs all n_inner projected-FISTA steps of an outer iteration on chip.
//
// Layout on chip.  Wave s (0..15) owns pixel rows il = 8 s .. 8 s + 7 of the
// tile; lane l owns columns 2l ("a") and 2l + 1 ("b") of those rows, so a
// wave covers a full tile row and every column neighbour is in the same wave
// (DPP wave shifts).  Each thread owns the top and left edges of its 16
// pixels; the tile's bottom boundary edges belong to the wave holding the last
// row, and the right boundary column of edges (one per row) to the lane
// holding the last column, kept in LDS.
//   VGPRs: the two iterate slots (x_{k-1} and x_{k-2}, then y, then x_k) on
//          the owned edges, 8 x 8 values.
//   LDS:   c' of every edge (128 KB) -- the per-edge constant that carries the
//          anchor phat and the image f (fista_ops.h) -- plus one exchange row
//          per strip for y and for the divergence d.
// A step: (1) y on every owned edge, publish the first row's top-edge y;
// barrier; (2) d of the strip's last row, publish it; barrier; (3) sweep the
// 8 rows: d of the row, projected step on the row's edges.
//
// The arithmetic per edge is that of the streaming kernel (fista_ops.h), so
// both schedules give bitwise identical results.
#include "fused_common.h"

namespace dtv {

using namespace fused;



// One workgroup's work on subdomain t.  LS holds lambda^(n+1) on the top, bottom, left and
// right sides; red is the reduction buffer of the adaptive rule (2 kWaves doubles).
// FR (with kFull): a framed tile, smaller than 128 x 128, run by the full-tile step in a
// 128 x 128 frame (full_step<.., FR>): FR = 1 when its short sides lie on the image boundary,
// FR = 2 for any tile of at most 128 x 128 (its bottom edges sit in frame row h and its right
// edges in frame column w, interface copies or not).
template <bool kFull, int KF, bool REC, bool ADAPT, int FR = 0>
__device__ __forceinline__ void fused_tile(const FusedArgs &a, int t, FusedLds &S, float (&LS)[4][kFusedMax],
                                           double *red)
{
    const SubTile tl = a.subs[t];
    const ImgDev im = a.imgs[tl.img];
    Ctx c;
    c.s = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform strip index
    c.lane = threadIdx.x & 63;
    c.ja = 2 * c.lane;
    c.jb = c.ja + 1;
    c.il0 = kR * c.s;
    constexpr bool kShape = kFull && !FR;  // the tile is 128 x 128 (known at compile time)
    c.h = kShape ? kFusedMax : tl.h;
    c.w = kShape ? kFusedMax : tl.w;
    c.acta = c.ja < c.w;
    c.actb = c.jb < c.w;
    c.lastcol_a = c.ja == c.w - 1;
    c.lastcol_b = c.jb == c.w - 1;
    const int H = im.H, W = im.W;
    c.top_bnd = tl.ra == 0;
    c.bot_bnd = tl.ra + c.h == H;
    c.left_bnd = tl.ca == 0;
    c.right_bnd = tl.ca + c.w == W;
    c.rb = c.h - 1 - c.il0;
    c.has_bottom = c.rb >= 0 && c.rb < kR;
    c.ak = im.a_keep;
    c.kL = im.kL;
    const int h = c.h, w = c.w, il0 = c.il0, ja = c.ja, jb = c.jb;
    const long long P1 = im.pitch1, P2 = im.pitch2;
    const long long row1 = (long long)tl.ra + tl.r;  // P1 row of the tile's edge row 0
    const long long col2 = (long long)tl.ca + tl.c;  // P2 column of the tile's edge column 0
    const float *b1 = a.base1 + im.p1, *b2 = a.base2 + im.p2;
    float *o1 = a.out1 + im.p1, *o2 = a.out2 + im.p2;
    const float *f = a.f + im.px;
    const float tau = a.tau, itau = a.inv_tau, invL = im.invL;

    Slot A, B;
    A.ba = A.bb = 0.0f;

    // ---- load p~^n and build c' (anchor phat = p~^n -/+ tau lambda on interface copies).
    // Every load of the thread is issued first and consumed afterwards, so the
    // tile arrives in one memory latency instead of one per row.  Each lane
    // reads its two adjacent columns with 8-byte accesses; f of the row above
    // is carried down the strip and f of the column to the left comes from the
    // neighbouring lane.
    auto ld2 = [](const float *p, float &x, float &y) {
        float2 v;
        __builtin_memcpy(&v, p, 8);
        x = v.x;
        y = v.y;
    };
    // uniform (per wave) row pointers; lanes index them with their column ja
    const float *f_tile = f + (long long)tl.ra * W + tl.ca;                 // pixel (0, 0) of the tile
    const float *p1_tile = b1 + row1 * P1 + tl.ca;                          // edge above pixel (0, 0)
    const float *p2_tile = b2 + (long long)tl.ra * P2 + col2;               // edge left of pixel (0, 0)
    const bool lastcol = c.lastcol_a || c.lastcol_b;
    // columns of the left edges held in registers: 0 .. w - 1, and w (the right edges) when a
    // framed tile with masks is narrower than the frame
    const bool l2a = FR == 2 ? ja <= w : c.acta, l2b = FR == 2 ? jb <= w : c.actb;
    float fva[kR], fvb[kR];  // f of the strip's rows at columns a and b
    float xr[kR];            // right boundary edges of the rows (last-column lane)
    float fua = 0.0f, fub = 0.0f;  // f of the row above (0 above the tile)
    // the rows' edges and image values first (unconditional on full tiles) ...
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int il = il0 + r;
        float x1a = 0.0f, x1b = 0.0f, x2a = 0.0f, x2b = 0.0f;
        fva[r] = fvb[r] = xr[r] = 0.0f;
        // (the zeros of the edges are written in every lane before the loads, pinned there:
        // written only in the lanes that skip a load, a zero would wait for the other lanes' load
        // into the same register, and the rows' loads would not overlap)
        if constexpr (!kShape) pin4(x1a, x1b, x2a, x2b);
        if (kShape || il < h) {  // (always on full tiles)
            const float *p1r = p1_tile + (long long)il * P1;
            const float *p2r = p2_tile + (long long)il * P2;
            const float *fr = f_tile + (long long)il * W;
            if (c.actb) {
                ld2(p1r + ja, x1a, x1b);
                ld2(p2r + ja, x2a, x2b);
                ld2(fr + ja, fva[r], fvb[r]);
            } else if (c.acta) {
                x1a = p1r[ja];
                fva[r] = fr[ja];
                if (l2b) ld2(p2r + ja, x2a, x2b);
                else x2a = p2r[ja];
            } else if (l2a) {
                x2a = p2r[ja];
            }
        } else if (FR == 2 && il == h) {  // the tile's bottom edges, in frame row h < 128
            const float *p1r = p1_tile + (long long)il * P1;
            if (c.actb) ld2(p1r + ja, x1a, x1b);
            else if (c.acta) x1a = p1r[ja];
        }
        A.e1a[r] = x1a; A.e2a[r] = x2a; A.e1b[r] = x1b; A.e2b[r] = x2b;
    }
    // ... then the conditional ones (waiting on one of these waits on everything issued before it)
    if (il0 > 0 && (il0 < h || (FR == 2 && il0 == h))) {
        const float *fr = f_tile + (long long)(il0 - 1) * W;
        if (c.actb) ld2(fr + ja, fua, fub);
        else if (c.acta) fua = fr[ja];
    }
    if (c.has_bottom && (!FR || h == kFusedMax)) {  // bottom boundary edges (the frame's own when framed)
        const float *pb = p1_tile + (long long)h * P1;
        if (c.acta) A.ba = pb[ja];
        if (c.actb) A.bb = pb[jb];
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int il = il0 + r;
        if ((kShape || il < h) && lastcol && (!FR || w == kFusedMax))
            xr[r] = p2_tile[(long long)il * P2 + w];  // right boundary edge of the row
    }

    // ---- (a1) lambda^(n+1) = lambda^n + sigma [(2 p_s^n - p_s^(n-1)) - (2 p_t^n - p_t^(n-1))] on the
    // tile's interface edges, with the operations of the multiplier kernel (the two tiles of an
    // interface compute the same value).  Waves 0..7 take the top, bottom, left and right sides
    // (two waves each).  The new lambda state goes to lam_out: lambda^(n+1) and p_s^n by the s
    // side (bottom, right), p_t^n by the t side (top, left).
    {
        const int side = c.s >> 1, si = (c.s & 1) * 64 + c.lane;
        bool has = false;
        long long e = 0, ips = 0, ipt = 0;  // lambda index; P1 or P2 offsets of the s and t copies
        if (c.s < 2 * 4 && si < (side < 2 ? w : h)) {
            const long long rs = (long long)(tl.ra + si) * P2;  // P2 row of a left / right edge
            switch (side) {
            case 0:  // top: the tile above holds the s copy
                has = tl.r > 0;
                e = (long long)(tl.r - 1) * W + tl.ca + si;
                ips = (row1 - 1) * P1 + tl.ca + si;
                ipt = row1 * P1 + tl.ca + si;
                break;
            case 1:  // bottom: the tile below holds the t copy
                has = tl.r < im.ny - 1;
                e = (long long)tl.r * W + tl.ca + si;
                ips = (row1 + h) * P1 + tl.ca + si;
                ipt = (row1 + h + 1) * P1 + tl.ca + si;
                break;
            case 2:  // left: the tile on the left holds the s copy
                has = tl.c > 0;
                e = im.nlh + (long long)(tl.c - 1) * H + tl.ra + si;
                ips = rs + col2 - 1;
                ipt = rs + col2;
                break;
            default:  // right: the tile on the right holds the t copy
                has = tl.c < im.nx - 1;
                e = im.nlh + (long long)tl.c * H + tl.ra + si;
                ips = rs + col2 + w;
                ipt = rs + col2 + w + 1;
                break;
            }
        }
        if (has) {
            const float *pp = side < 2 ? b1 : b2;
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
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int il = il0 + r;
        const float fla = from_left(fvb[r]);  // f of column a - 1 (lane 0: left of the tile, 0)
        if constexpr (FR) {
            // every c' entry of the frame written once: the tile's edges as below, 0 outside it
            // (with masks, row h < 128 holds the tile's bottom edges and column w < 128 its right
            // edges: s copies of an interface, anchored with -tau lambda, unless on the image
            // boundary; f is 0 below and right of the tile)
            float c1a = 0.0f, c1b = 0.0f, c2a = 0.0f, c2b = 0.0f;
            if (il < h || (FR == 2 && il == h)) {
                float ata = A.e1a[r], atb = A.e1b[r];
                if (il == 0 && tl.r > 0) {
                    if (c.acta) ata = fmaf(tau, LS[0][ja], ata);
                    if (c.actb) atb = fmaf(tau, LS[0][jb], atb);
                }
                if (FR == 2 && il == h && !c.bot_bnd) {
                    if (c.acta) ata = fmaf(-tau, LS[1][ja], ata);
                    if (c.actb) atb = fmaf(-tau, LS[1][jb], atb);
                }
                if (c.acta) c1a = fista_cprime(ata, fua, fva[r], itau, invL);
                if (c.actb) c1b = fista_cprime(atb, fub, fvb[r], itau, invL);
            }
            if (il < h) {
                float ala = A.e2a[r], alb = A.e2b[r];
                if (ja == 0 && tl.c > 0) ala = fmaf(tau, LS[2][il], ala);
                if (FR == 2 && !c.right_bnd) {
                    if (ja == w) ala = fmaf(-tau, LS[3][il], ala);
                    if (jb == w) alb = fmaf(-tau, LS[3][il], alb);
                }
                if (l2a) c2a = fista_cprime(ala, ja > 0 ? fla : 0.0f, fva[r], itau, invL);
                if (l2b) c2b = fista_cprime(alb, fva[r], fvb[r], itau, invL);
            }
            lds_st2(&S.c1[il][ja], c1a, c1b);
            lds_st2(&S.c2[il][ja], c2a, c2b);
            if (il == kFusedMax - 1) {  // the frame's bottom edges: the tile's when h = 128
                float cba = 0.0f, cbb = 0.0f;
                if (h == kFusedMax) {
                    if (c.acta) cba = fista_cprime(c.bot_bnd ? A.ba : fmaf(-tau, LS[1][ja], A.ba), fva[r], 0.0f, itau,
                                                   invL);
                    if (c.actb) cbb = fista_cprime(c.bot_bnd ? A.bb : fmaf(-tau, LS[1][jb], A.bb), fvb[r], 0.0f, itau,
                                                   invL);
                }
                lds_st2(&S.cb[ja], cba, cbb);
            }
            if (c.lane == 63) {  // the frame's right edges: the tile's when w = 128
                float xv = 0.0f, cv = 0.0f;
                if (w == kFusedMax && il < h) {
                    xv = xr[r];
                    cv = fista_cprime(c.right_bnd ? xr[r] : fmaf(-tau, LS[3][il], xr[r]), fvb[r], 0.0f, itau, invL);
                }
                S.rx[0][il] = xv;
                S.rx[1][il] = xv;
                S.cr[il] = cv;
            }
        } else if (kShape || il < h) {  // (always on full tiles)
            // top edges (t copies of an interface on the tile's first row)
            float ata = A.e1a[r], atb = A.e1b[r];
            if (il == 0 && tl.r > 0) {
                if (c.acta) ata = fmaf(tau, LS[0][ja], ata);
                if (c.actb) atb = fmaf(tau, LS[0][jb], atb);
            }
            // left edge (t copy of an interface on the tile's first column)
            float ala = A.e2a[r];
            if (ja == 0 && tl.c > 0) ala = fmaf(tau, LS[2][il], ala);
            if (c.acta) {
                S.c1[il][ja] = fista_cprime(ata, fua, fva[r], itau, invL);
                S.c2[il][ja] = fista_cprime(ala, ja > 0 ? fla : 0.0f, fva[r], itau, invL);
            }
            if (c.actb) {
                S.c1[il][jb] = fista_cprime(atb, fub, fvb[r], itau, invL);
                S.c2[il][jb] = fista_cprime(A.e2b[r], fva[r], fvb[r], itau, invL);
            }
            if (il == h - 1) {  // bottom boundary edges (s copies unless on the image boundary)
                if (c.acta) {
                    const float ab = c.bot_bnd ? A.ba : fmaf(-tau, LS[1][ja], A.ba);
                    S.cb[ja] = fista_cprime(ab, fva[r], 0.0f, itau, invL);
                }
                if (c.actb) {
                    const float ab = c.bot_bnd ? A.bb : fmaf(-tau, LS[1][jb], A.bb);
                    S.cb[jb] = fista_cprime(ab, fvb[r], 0.0f, itau, invL);
                }
            }
            if (lastcol) {  // right boundary edge of this row
                S.rx[0][il] = xr[r];
                S.rx[1][il] = xr[r];
                const float ar = c.right_bnd ? xr[r] : fmaf(-tau, LS[3][il], xr[r]);
                S.cr[il] = fista_cprime(ar, c.lastcol_a ? fva[r] : fvb[r], 0.0f, itau, invL);
            }
        }
        fua = fva[r];
        fub = fvb[r];
    }
    B = A;
    __syncthreads();

    // steps 1 and 2 have no momentum (beta = 0); x_K ends in slot A
    const int K = a.n_inner;
    int rx_slot = 0;  // LDS slot of the right boundary edges holding x_K
    int taken = K;    // steps taken (adaptive stopping)
    if constexpr (kFull) {
        FullCtx fc;
        fc.s = c.s;
        fc.lane = c.lane;
        fc.ja = ja;
        fc.il0 = il0;
        fc.oc = il0 * kFusedMax + ja;
        fc.oy = c.s * kFusedMax + ja;
        fc.olr = il0 + c.lane;
        fc.last = c.s == kWaves - 1;
        fc.right_bnd = c.right_bnd;
        const bool tb = c.top_bnd && c.s == 0, lb = c.left_bnd && c.lane == 0;
        fc.lo1 = tb ? 0.0f : -1.0f;
        fc.hi1 = tb ? 0.0f : 1.0f;
        fc.lo2a = lb ? 0.0f : -1.0f;
        fc.hi2a = lb ? 0.0f : 1.0f;
        fc.lob = c.bot_bnd ? 0.0f : -1.0f;
        fc.hib = c.bot_bnd ? 0.0f : 1.0f;
        fc.ak = c.ak;
        fc.kL = c.kL;
        fc.qa = (float)(-im.dA * (double)a.inv_tau);
        fc.qb = (float)(-im.dB);
        fc.lo2b = -1.0f;
        fc.hi2b = 1.0f;
        fc.zrows = 0u;
        fc.mrows = 0xFFu;
        fc.lva = fc.lvb = true;
        if constexpr (FR) {
            // the boundary lines of a framed tile: the left edges of column w, the top edges of
            // row h; clamped when on the image boundary (always, without masks)
            const bool rz = FR == 1 || c.right_bnd, bz = FR == 1 || c.bot_bnd;
            const bool za = rz && w < kFusedMax && ja == w, zb = rz && w < kFusedMax && jb == w;
            fc.lo2a = za ? 0.0f : fc.lo2a;
            fc.hi2a = za ? 0.0f : fc.hi2a;
            fc.lo2b = zb ? 0.0f : -1.0f;
            fc.hi2b = zb ? 0.0f : 1.0f;
            const int zr = h - il0;
            fc.zrows = (bz && h < kFusedMax && zr >= 0 && zr < kR) ? 1u << zr : 0u;
            fc.right_bnd = c.right_bnd || w < kFusedMax;  // the frame's right column lies outside the tile
            // the pixels inside the tile: rows il0 .. h - 1 of the strip, columns below w
            fc.mrows = zr >= kR ? 0xFFu : zr <= 0 ? 0u : (1u << zr) - 1u;
            fc.lva = c.acta;
            fc.lvb = c.actb;
        }
        if constexpr (ADAPT) {
            rx_slot = run_steps_adaptive<FullStep>(fc, S, A, B, K, a.beta_dev, a.tol2, red, taken);
        } else if constexpr (FR && KF > 0) {
            rx_slot = full_steps_fixed<KF, false, FR>(fc, S, A, B, a.beta);
            if constexpr (KF & 1) copy_slot(A, B);
        } else if constexpr (FR) {
            rx_slot = run_steps<FramedStep<FR>>(fc, S, A, B, K, a.beta);
        } else if constexpr (KF > 0) {
            if constexpr (REC) {
                const long long rec_step = (long long)gridDim.x * kRecGroups * kRecThreads;
                float4 *rec = a.rec + (long long)t * kRecGroups * kRecThreads + threadIdx.x;
                rx_slot = full_steps_fixed<KF, true>(fc, S, A, B, a.beta, rec, rec_step);
            } else {
                rx_slot = full_steps_fixed<KF>(fc, S, A, B, a.beta);
            }
            if constexpr (KF & 1) copy_slot(A, B);
        } else {
            rx_slot = run_steps<FullStep>(fc, S, A, B, K, a.beta);
        }
    } else if constexpr (ADAPT) {
        rx_slot = run_steps_adaptive<GenericStep>(c, S, A, B, K, a.beta_dev, a.tol2, red, taken);
    } else {
        rx_slot = run_steps<GenericStep>(c, S, A, B, K, a.beta);
    }
    if constexpr (ADAPT) {
        if (threadIdx.x == 0) {  // the only workgroup of this subdomain in this launch
            int *cnt = a.counts + 2 * (long long)t;
            cnt[0] += taken;
            cnt[1] = max(cnt[1], taken);
        }
    }

    // ---- store x_K (now in slot A) as p~^(n+1)
    auto st2 = [](float *p, float x, float y) {
        const float2 v = make_float2(x, y);
        __builtin_memcpy(p, &v, 8);
    };
    float *q1_tile = o1 + row1 * P1 + tl.ca;
    float *q2_tile = o2 + (long long)tl.ra * P2 + col2;
    // the recording kernel: the row bases are uniform and the thread's column enters as one 32-bit
    // byte offset, formed here (a column offset kept from the prologue stays live through the
    // recorded steps, in scratch); the other kernels address the row plus the column
    unsigned jo4 = 0;
    if constexpr (REC) jo4 = (unsigned)opaque(ja) * 4u;
    auto at = [jo4, ja](float *row) { return REC ? (float *)((char *)row + jo4) : row + ja; };
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int il = il0 + r;
        if (il < h) {
            float *q1 = q1_tile + (long long)il * P1;
            float *q2 = q2_tile + (long long)il * P2;
            if (c.actb) {
                st2(at(q1), A.e1a[r], A.e1b[r]);
                st2(at(q2), A.e2a[r], A.e2b[r]);
            } else if (c.acta) {
                *at(q1) = A.e1a[r];
                if (l2b) st2(at(q2), A.e2a[r], A.e2b[r]);
                else *at(q2) = A.e2a[r];
            } else if (l2a) {
                *at(q2) = A.e2a[r];
            }
            // the right boundary edge: a framed tile narrower than 128 holds it in column w with
            // masks, and has it on the image boundary without
            if ((c.lastcol_a || c.lastcol_b) && (!FR || w == kFusedMax)) q2[w] = S.rx[rx_slot][il];
        } else if (FR == 2 && il == h) {  // the bottom edges of a framed tile lower than 128
            float *q1 = q1_tile + (long long)il * P1;
            if (c.actb) st2(at(q1), A.e1a[r], A.e1b[r]);
            else if (c.acta) *at(q1) = A.e1a[r];
        }
    }
    if (c.has_bottom && (!FR || h == kFusedMax)) {
        float *qb = q1_tile + (long long)h * P1;
        if (c.actb) st2(at(qb), A.ba, A.bb);
        else if (c.acta) *at(qb) = A.ba;
    }
}

// kFull: every tile of the launch is 128 x 128 (the list holds the full
// tiles first; the full launch takes that prefix, the other launch the rest).
// KF > 0: full tiles with n_inner = KF (steps unrolled); KF = 0: any n_inner.
// REC: also record every step for reverse mode (full tiles, KF > 0; a.rec).
// ADAPT: stop each subdomain's steps by the relative-change rule (a.tol2, KF = 0).
template <bool kFull, int KF, bool REC = false, bool ADAPT = false>
__global__ __launch_bounds__(1024) void k_fused_fista(FusedArgs a, int first)
{
    __shared__ FusedLds S;
    __shared__ float LS[4][kFusedMax];
    __shared__ double red[ADAPT ? 2 * kWaves : 1];
    fused_tile<kFull, KF, REC, ADAPT>(a, first + xcd_remap(blockIdx.x, gridDim.x), S, LS, red);
}

// Full tiles, fixed n_inner, in a launch of many rounds (more subdomains than the device holds at
// once).  A workgroup's LDS fills a CU, so a tile's loads and stores never overlap its own steps,
// and workgroups that start together stay in step: every CU loads, then every CU computes while
// HBM idles.  Blocks [0, a.stagger_blocks) hold their CU for a.stagger_ticks of the 100 MHz
// constant clock and leave, so that those CUs start their first tile later; from then on one
// half of the CUs loads and stores while the other half runs its steps.  (The delaying blocks
// are dealt to the XCDs round-robin like any others, half the CUs of each.)
template <int KF>
__global__ __launch_bounds__(1024) void k_fused_fista_staggered(FusedArgs a)
{
    __shared__ FusedLds S;
    __shared__ float LS[4][kFusedMax];
    __shared__ double red[1];
    const int b = blockIdx.x, nd = a.stagger_blocks;
    if (b < nd) {
        if (threadIdx.x == 0) {
            const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
            while (__builtin_amdgcn_s_memrealtime() - t0 < (unsigned long long)a.stagger_ticks)
                __builtin_amdgcn_s_sleep(4);
        }
        __syncthreads();
        return;
    }
    fused_tile<true, KF, false, false>(a, xcd_remap(b - nd, gridDim.x - nd), S, LS, red);
}

// Every kind of tile in one launch (fixed n_inner, no recording).  The list holds the full
// tiles first, then the framed ones (short sides on the image boundary), then the others, which
// run framed with masks; blocks [0, gpad) take the other tiles, [gpad, gpad + fpad) the framed
// ones (gpad, fpad: the counts rounded up to a multiple of 8; the extra blocks exit at once),
// the rest the full tiles.  The slower kinds are
// dispatched first, spread over the XCDs; the full tiles keep the XCD-aware order, and no launch
// boundary separates the kinds.
template <int KF>
__global__ __launch_bounds__(1024) void k_fused_fista_mixed(FusedArgs a, int nfull, int nframed, int ngen)
{
    __shared__ FusedLds S;
    __shared__ float LS[4][kFusedMax];
    __shared__ double red[1];
    const int gpad = (ngen + 7) & ~7, fpad = (nframed + 7) & ~7;
    const int b = blockIdx.x;
    if (b < gpad) {
        if (b < ngen) fused_tile<true, KF, false, false, 2>(a, nfull + nframed + b, S, LS, red);
    } else if (b < gpad + fpad) {
        if (b - gpad < nframed) fused_tile<true, KF, false, false, 1>(a, nfull + b - gpad, S, LS, red);
    } else {
        fused_tile<true, KF, false, false>(a, xcd_remap(b - gpad - fpad, gridDim.x - gpad - fpad), S, LS, red);
    }
}

namespace {

using FusedKernel = void (*)(FusedArgs, int);

// full-tile kernels with the inner step count unrolled, for the common counts;
// the recording ones exist only there
template <int... Ks>
struct FullTable {
    static FusedKernel get(int K, bool rec)
    {
        FusedKernel k = nullptr;
        ((K == Ks ? (k = rec ? k_fused_fista<true, Ks, true> : k_fused_fista<true, Ks>, 0) : 0), ...);
        return k ? k : rec ? nullptr : k_fused_fista<true, 0>;
    }
};
using Full = FullTable<1, 2, 3, 4, 5, 6, 7, 8, 10>;

using MixedKernel = void (*)(FusedArgs, int, int, int);
using FusedKernel1 = void (*)(FusedArgs);

template <int... Ks>
struct MixedTable {
    static MixedKernel get(int K)
    {
        MixedKernel k = nullptr;
        ((K == Ks ? (k = k_fused_fista_mixed<Ks>, 0) : 0), ...);
        return k ? k : k_fused_fista_mixed<0>;
    }
};
using Mixed = MixedTable<1, 2, 3, 4, 5, 6, 7, 8, 10>;

template <int... Ks>
struct StaggerTable {
    static FusedKernel1 get(int K)
    {
        FusedKernel1 k = nullptr;
        ((K == Ks ? (k = k_fused_fista_staggered<Ks>, 0) : 0), ...);
        return k ? k : k_fused_fista_staggered<0>;
    }
};
using Stagger = StaggerTable<1, 2, 3, 4, 5, 6, 7, 8, 10>;

}  // namespace

bool fused_record_supported(int K) { return Full::get(K, true) != nullptr; }

int fused_capacity(int device)
{
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused_fista<true, 0>, 1024, 0) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    return per_cu * cus;
}

namespace {

}  // namespace

hipError_t launch_fused_fista(const FusedArgs &a, int nsub, int nfull, int nframed, hipStream_t s, hipEvent_t e0,
                              hipEvent_t e1)
{
    if (nsub <= 0) return hipSuccess;
    const bool adapt = a.tol2 > 0.0;
    if (a.n_inner < 1 || (!adapt && a.n_inner > kMaxFusedInner) || nfull < 0 || nfull > nsub)
        return hipErrorInvalidValue;
    const int npart = nsub - nfull;
    if (a.rec && (adapt || npart > 0 || !Full::get(a.n_inner, true))) return hipErrorInvalidValue;
    if (adapt && (!a.beta_dev || !a.counts)) return hipErrorInvalidValue;
    if (adapt) {
        if (nfull > 0) {
            hipEvent_t stop = npart > 0 ? nullptr : e1;
            if (e0)
                hipExtLaunchKernelGGL((k_fused_fista<true, 0, false, true>), dim3(nfull), dim3(1024), 0, s, e0, stop,
                                      0, a, 0);
            else
                hipLaunchKernelGGL((k_fused_fista<true, 0, false, true>), dim3(nfull), dim3(1024), 0, s, a, 0);
        }
        if (npart > 0) {
            hipEvent_t start = nfull > 0 ? nullptr : e0;
            if (e0)
                hipExtLaunchKernelGGL((k_fused_fista<false, 0, false, true>), dim3(npart), dim3(1024), 0, s, start,
                                      e1, 0, a, nfull);
            else
                hipLaunchKernelGGL((k_fused_fista<false, 0, false, true>), dim3(npart), dim3(1024), 0, s, a, nfull);
        }
        return hipGetLastError();
    }
    if (nframed < 0 || nframed > npart) return hipErrorInvalidValue;
    if (npart > 0 && !a.rec) {  // one launch for every kind of tile
        const MixedKernel km = Mixed::get(a.n_inner);
        const int ngen = npart - nframed;
        const int grid = ((ngen + 7) & ~7) + ((nframed + 7) & ~7) + nfull;
        if (e0)
            hipExtLaunchKernelGGL(km, dim3(grid), dim3(1024), 0, s, e0, e1, 0, a, nfull, nframed, ngen);
        else
            hipLaunchKernelGGL(km, dim3(grid), dim3(1024), 0, s, a, nfull, nframed, ngen);
        return hipGetLastError();
    }
    if (npart == 0 && !a.rec && a.stagger_blocks > 0) {  // many rounds of full tiles
        const FusedKernel1 k = Stagger::get(a.n_inner);
        const int grid = nfull + a.stagger_blocks;
        if (e0)
            hipExtLaunchKernelGGL(k, dim3(grid), dim3(1024), 0, s, e0, e1, 0, a);
        else
            hipLaunchKernelGGL(k, dim3(grid), dim3(1024), 0, s, a);
        return hipGetLastError();
    }
    // the timing events bracket both launches
    if (nfull > 0) {
        const FusedKernel kf = Full::get(a.n_inner, a.rec != nullptr);
        hipEvent_t stop = npart > 0 ? nullptr : e1;
        if (e0)
            hipExtLaunchKernelGGL(kf, dim3(nfull), dim3(1024), 0, s, e0, stop, 0, a, 0);
        else
            hipLaunchKernelGGL(kf, dim3(nfull), dim3(1024), 0, s, a, 0);
    }
    if (npart > 0) {
        hipEvent_t start = nfull > 0 ? nullptr : e0;
        if (e0)
            hipExtLaunchKernelGGL((k_fused_fista<false, 0>), dim3(npart), dim3(1024), 0, s, start, e1, 0, a, nfull);
        else
            hipLaunchKernelGGL((k_fused_fista<false, 0>), dim3(npart), dim3(1024), 0, s, a, nfull);
    }
    return hipGetLastError();
}

}  // namespace dtv
