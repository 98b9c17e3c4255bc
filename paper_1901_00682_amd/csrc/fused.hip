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
#include "dtvdd_internal.h"
#include "fista_ops.h"

namespace dtv {

namespace {

constexpr int kR = 8;         // rows per wave
constexpr int kWaves = 16;    // 128 / kR

struct FusedLds {
    float c1[kFusedMax][kFusedMax];  // c' of the edge above pixel (il, jl)
    float c2[kFusedMax][kFusedMax];  // c' of the edge left of pixel (il, jl)
    float cb[kFusedMax];             // c' of the bottom boundary edges (per column)
    float cr[kFusedMax];             // c' of the right boundary edges (per row)
    float rx[2][kFusedMax];          // right boundary edges: the two iterate slots (per row)
    float yt[2][kWaves][kFusedMax];  // y on the top edges of each strip's first row, one buffer per
                                     // step parity: a strip may start the next step while the strip
                                     // above still reads the current row
    float dl[kWaves][kFusedMax];     // d of each strip's last row
};

// lane i receives lane i - 1 (lane 0 receives 0)
__device__ __forceinline__ float from_left(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xF, 0xF, false));
}

// lane i receives lane i + 1 (lane 63 receives 0)
__device__ __forceinline__ float from_right(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xF, 0xF, false));
}

}  // namespace

// iterate slot of one thread: its top (1) and left (2) edges in columns a and
// b of its kR rows, and the bottom boundary edges of the tile (last strip)
struct Slot {
    float e1a[kR], e1b[kR], e2a[kR], e2b[kR];
    float ba, bb;
};

struct Ctx {
    int s, lane, ja, jb, il0, h, w;
    int par;  // exchange-buffer parity of the current step
    bool acta, actb, lastcol_a, lastcol_b, top_bnd, bot_bnd, left_bnd, right_bnd, has_bottom;
    int rb;
    float ak, kL;
};

// y on the edge below row r of columns a and b
__device__ __forceinline__ void edge_below(const Ctx &c, const FusedLds &S, const Slot &Y, int r, float &ya, float &yb)
{
    const int il = c.il0 + r;
    if (il == c.h - 1) {
        ya = Y.ba;
        yb = Y.bb;
    } else if (r < kR - 1) {
        ya = Y.e1a[r + 1];
        yb = Y.e1b[r + 1];
    } else {
        const int sn = c.s < kWaves - 1 ? c.s + 1 : c.s;
        ya = S.yt[c.par][sn][c.ja];
        yb = S.yt[c.par][sn][c.jb];
    }
}

// unscaled divergence of the two pixels of row r
__device__ __forceinline__ void row_div(const Ctx &c, const Slot &Y, const float *RY, int r, float ya_below,
                                        float yb_below, float &da, float &db)
{
    const int il = c.il0 + r;
    float yra = Y.e2b[r];                // right edge of column a = left edge of column b
    float yrb = from_right(Y.e2a[r]);    // right edge of column b = left edge of the next lane's column a
    if (c.lastcol_a) yra = RY[il];
    if (c.lastcol_b) yrb = RY[il];
    const bool on = il < c.h;
    da = (on && c.acta) ? div4(Y.e1a[r], ya_below, Y.e2a[r], yra) : 0.0f;
    db = (on && c.actb) ? div4(Y.e1b[r], yb_below, Y.e2b[r], yrb) : 0.0f;
}

// One projected-FISTA step.  On entry X holds x_{k-1} and Y holds x_{k-2};
// on exit Y holds x_k.  sx selects the LDS slot of the right boundary edges
// that plays the role of X.
__device__ __forceinline__ void copy_slot(Slot &dst, const Slot &src)
{
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        dst.e1a[r] = src.e1a[r];
        dst.e1b[r] = src.e1b[r];
        dst.e2a[r] = src.e2a[r];
        dst.e2b[r] = src.e2b[r];
    }
    dst.ba = src.ba;
    dst.bb = src.bb;
}

template <bool mom>
__device__ __forceinline__ void fused_step(const Ctx &c0, FusedLds &S, const Slot &X, Slot &Y, int sx, float beta)
{
    Ctx c = c0;
    c.par = sx;
    const float *RX = S.rx[sx];
    float *RY = S.rx[sx ^ 1];
    const bool lastcol = c.lastcol_a || c.lastcol_b;
    // (1) y on every owned edge
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        Y.e1a[r] = mom ? fista_y(X.e1a[r], Y.e1a[r], beta) : X.e1a[r];
        Y.e1b[r] = mom ? fista_y(X.e1b[r], Y.e1b[r], beta) : X.e1b[r];
        Y.e2a[r] = mom ? fista_y(X.e2a[r], Y.e2a[r], beta) : X.e2a[r];
        Y.e2b[r] = mom ? fista_y(X.e2b[r], Y.e2b[r], beta) : X.e2b[r];
        const int il = c.il0 + r;
        if (lastcol && il < c.h) RY[il] = mom ? fista_y(RX[il], RY[il], beta) : RX[il];
    }
    Y.ba = mom ? fista_y(X.ba, Y.ba, beta) : X.ba;
    Y.bb = mom ? fista_y(X.bb, Y.bb, beta) : X.bb;
    if (c.s > 0 && c.il0 < c.h) {
        S.yt[sx][c.s][c.ja] = Y.e1a[0];
        S.yt[sx][c.s][c.jb] = Y.e1b[0];
    }
    __syncthreads();

    // (2) publish d of the strip's last row
    {
        float ya, yb, da, db;
        edge_below(c, S, Y, kR - 1, ya, yb);
        row_div(c, Y, RY, kR - 1, ya, yb, da, db);
        S.dl[c.s][c.ja] = da;
        S.dl[c.s][c.jb] = db;
    }
    __syncthreads();

    // (3) sweep the rows: d of the row, then the projected step on its edges
    float dua = 0.0f, dub = 0.0f;  // d of the row above (0 above the tile: one-sided copy)
    if (c.s > 0) {
        dua = S.dl[c.s - 1][c.ja];
        dub = S.dl[c.s - 1][c.jb];
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int il = c.il0 + r;
        float ya, yb, da, db;
        edge_below(c, S, Y, r, ya, yb);
        row_div(c, Y, RY, r, ya, yb, da, db);
        const float dlb = from_left(db);  // d of column a - 1 (lane 0: left of the tile, 0)
        if (il < c.h) {
            if (!(il == 0 && c.top_bnd)) {
                if (c.acta) Y.e1a[r] = fista_edge(Y.e1a[r], dua, da, S.c1[il][c.ja], c.ak, c.kL);
                if (c.actb) Y.e1b[r] = fista_edge(Y.e1b[r], dub, db, S.c1[il][c.jb], c.ak, c.kL);
            }
            if (c.acta && !(c.ja == 0 && c.left_bnd)) Y.e2a[r] = fista_edge(Y.e2a[r], dlb, da, S.c2[il][c.ja], c.ak, c.kL);
            if (c.actb) Y.e2b[r] = fista_edge(Y.e2b[r], da, db, S.c2[il][c.jb], c.ak, c.kL);
            if (c.has_bottom && r == c.rb && !c.bot_bnd) {
                if (c.acta) Y.ba = fista_edge(Y.ba, da, 0.0f, S.cb[c.ja], c.ak, c.kL);
                if (c.actb) Y.bb = fista_edge(Y.bb, db, 0.0f, S.cb[c.jb], c.ak, c.kL);
            }
            if (!c.right_bnd) {
                if (c.lastcol_a) RY[il] = fista_edge(RY[il], da, 0.0f, S.cr[il], c.ak, c.kL);
                if (c.lastcol_b) RY[il] = fista_edge(RY[il], db, 0.0f, S.cr[il], c.ak, c.kL);
            }
        }
        dua = da;
        dub = db;
    }
}

__global__ __launch_bounds__(1024) void k_fused_fista(FusedArgs a)
{
    __shared__ FusedLds S;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const SubTile tl = a.subs[t];
    const ImgDev im = a.imgs[tl.img];
    Ctx c;
    c.s = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform strip index
    c.lane = threadIdx.x & 63;
    c.ja = 2 * c.lane;
    c.jb = c.ja + 1;
    c.il0 = kR * c.s;
    c.h = tl.h;
    c.w = tl.w;
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
    const float *lam = a.lam + im.lam;
    const float *f = a.f + im.px;
    const float tau = a.tau, itau = a.inv_tau, invL = im.invL;

    Slot A, B;
    A.ba = A.bb = 0.0f;

    // ---- load p~^n and build c' (anchor phat = p~^n -/+ tau lambda on interface copies).
    // Each lane reads its two adjacent columns with 8-byte accesses; f of the
    // row above is carried down the strip and f of the column to the left comes
    // from the neighbouring lane.
    auto ld2 = [](const float *p, float &x, float &y) {
        float2 v;
        __builtin_memcpy(&v, p, 8);
        x = v.x;
        y = v.y;
    };
    float fua = 0.0f, fub = 0.0f;  // f of the row above (0 above the tile)
    // uniform (per wave) row pointers; lanes index them with their column ja
    const float *f_tile = f + (long long)tl.ra * W + tl.ca;                 // pixel (0, 0) of the tile
    const float *p1_tile = b1 + row1 * P1 + tl.ca;                          // edge above pixel (0, 0)
    const float *p2_tile = b2 + (long long)tl.ra * P2 + col2;               // edge left of pixel (0, 0)
    if (il0 > 0 && il0 < h) {
        const float *fr = f_tile + (long long)(il0 - 1) * W;
        if (c.actb) ld2(fr + ja, fua, fub);
        else if (c.acta) fua = fr[ja];
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int il = il0 + r;
        float x1a = 0.0f, x1b = 0.0f, x2a = 0.0f, x2b = 0.0f, fva = 0.0f, fvb = 0.0f;
        const float *p1r = p1_tile + (long long)il * P1;
        const float *p2r = p2_tile + (long long)il * P2;
        const float *fr = f_tile + (long long)il * W;
        if (il < h) {
            if (c.actb) {
                ld2(p1r + ja, x1a, x1b);
                ld2(p2r + ja, x2a, x2b);
                ld2(fr + ja, fva, fvb);
            } else if (c.acta) {
                x1a = p1r[ja];
                x2a = p2r[ja];
                fva = fr[ja];
            }
        }
        const float fla = from_left(fvb);  // f of column a - 1 (lane 0: left of the tile, 0)
        if (il < h) {
            const long long gi = tl.ra + il;
            // top edges (t copies of an interface on the tile's first row)
            float ata = x1a, atb = x1b;
            if (il == 0 && tl.r > 0) {
                const float *lr = lam + (long long)(tl.r - 1) * W + tl.ca;
                if (c.acta) ata = fmaf(tau, lr[ja], ata);
                if (c.actb) atb = fmaf(tau, lr[jb], atb);
            }
            // left edge (t copy of an interface on the tile's first column)
            float ala = x2a;
            if (ja == 0 && tl.c > 0) ala = fmaf(tau, lam[im.nlh + (long long)(tl.c - 1) * H + gi], ala);
            if (c.acta) {
                S.c1[il][ja] = fista_cprime(ata, fua, fva, itau, invL);
                S.c2[il][ja] = fista_cprime(ala, ja > 0 ? fla : 0.0f, fva, itau, invL);
            }
            if (c.actb) {
                S.c1[il][jb] = fista_cprime(atb, fub, fvb, itau, invL);
                S.c2[il][jb] = fista_cprime(x2b, fva, fvb, itau, invL);
            }
            if (il == h - 1) {  // bottom boundary edges (s copies unless on the image boundary)
                const float *pb = p1_tile + (long long)h * P1;
                const float *lb = lam + (long long)tl.r * W + tl.ca;
                if (c.acta) {
                    const float xb = pb[ja];
                    A.ba = xb;
                    const float ab = c.bot_bnd ? xb : fmaf(-tau, lb[ja], xb);
                    S.cb[ja] = fista_cprime(ab, fva, 0.0f, itau, invL);
                }
                if (c.actb) {
                    const float xb = pb[jb];
                    A.bb = xb;
                    const float ab = c.bot_bnd ? xb : fmaf(-tau, lb[jb], xb);
                    S.cb[jb] = fista_cprime(ab, fvb, 0.0f, itau, invL);
                }
            }
            if (c.lastcol_a || c.lastcol_b) {  // right boundary edge of this row
                const float xr = p2r[w];
                S.rx[0][il] = xr;
                S.rx[1][il] = xr;
                const float ar = c.right_bnd ? xr : fmaf(-tau, lam[im.nlh + (long long)tl.c * H + gi], xr);
                S.cr[il] = fista_cprime(ar, c.lastcol_a ? fva : fvb, 0.0f, itau, invL);
            }
        }
        A.e1a[r] = x1a; A.e2a[r] = x2a; A.e1b[r] = x1b; A.e2b[r] = x2b;
        fua = fva;
        fub = fvb;
    }
    B = A;
    __syncthreads();

    // steps 1 and 2 have no momentum (beta = 0); x_K ends in slot A
    const int K = a.n_inner;
    int rx_slot = 0;  // LDS slot of the right boundary edges holding x_K
    if (K == 1) {
        fused_step<false>(c, S, A, B, 0, 0.0f);
        copy_slot(A, B);
        rx_slot = 1;
    } else {
        fused_step<false>(c, S, A, B, 0, 0.0f);
        fused_step<false>(c, S, B, A, 1, 0.0f);
        int k = 3;
        for (; k + 1 <= K; k += 2) {
            fused_step<true>(c, S, A, B, 0, a.beta[k]);
            fused_step<true>(c, S, B, A, 1, a.beta[k + 1]);
        }
        if (k == K) {
            fused_step<true>(c, S, A, B, 0, a.beta[K]);
            copy_slot(A, B);
            rx_slot = 1;
        }
    }

    // ---- store x_K (now in slot A) as p~^(n+1)
    auto st2 = [](float *p, float x, float y) {
        const float2 v = make_float2(x, y);
        __builtin_memcpy(p, &v, 8);
    };
    float *q1_tile = o1 + row1 * P1 + tl.ca;
    float *q2_tile = o2 + (long long)tl.ra * P2 + col2;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int il = il0 + r;
        if (il < h) {
            float *q1 = q1_tile + (long long)il * P1;
            float *q2 = q2_tile + (long long)il * P2;
            if (c.actb) {
                st2(q1 + ja, A.e1a[r], A.e1b[r]);
                st2(q2 + ja, A.e2a[r], A.e2b[r]);
            } else if (c.acta) {
                q1[ja] = A.e1a[r];
                q2[ja] = A.e2a[r];
            }
            if (c.lastcol_a || c.lastcol_b) q2[w] = S.rx[rx_slot][il];
        }
    }
    if (c.has_bottom) {
        float *qb = q1_tile + (long long)h * P1;
        if (c.actb) st2(qb + ja, A.ba, A.bb);
        else if (c.acta) qb[ja] = A.ba;
    }
}

hipError_t launch_fused_fista(const FusedArgs &a, int nsub, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (nsub <= 0) return hipSuccess;
    if (a.n_inner < 1 || a.n_inner > kMaxFusedInner) return hipErrorInvalidValue;
    if (e0)
        hipExtLaunchKernelGGL(k_fused_fista, dim3(nsub), dim3(1024), 0, s, e0, e1, 0, a);
    else
        hipLaunchKernelGGL(k_fused_fista, dim3(nsub), dim3(1024), 0, s, a);
    return hipGetLastError();
}

}  // namespace dtv
