// Device code shared by the fused and the persistent FISTA kernels: the
// on-chip layout of one subdomain tile (LDS and register slots) and one
// projected-FISTA step over the tile.  See fused.hip for the layout.
#pragma once

#include "dtvdd_internal.h"
#include "fista_ops.h"

namespace dtv {
namespace fused {

constexpr int kR = 8;         // rows per wave
constexpr int kWaves = 16;    // 128 / kR

struct FusedLds {
    // the small arrays first, so that their offsets fit the 16-bit immediate of LDS instructions
    float cb[kFusedMax];             // c' of the bottom boundary edges (per column)
    float cr[kFusedMax];             // c' of the right boundary edges (per row)
    float rx[2][kFusedMax];          // right boundary edges: the two iterate slots (per row)
    float yt[2][kWaves][kFusedMax];  // y on the top edges of each strip's first row, one buffer per
                                     // step parity: a strip may start the next step while the strip
                                     // above still reads the current row
    float dl[kWaves][kFusedMax];     // d of each strip's last row
    float dR[kFusedMax];             // full tiles: d of the last column, per row
    float c1[kFusedMax][kFusedMax];  // c' of the edge above pixel (il, jl)
    float c2[kFusedMax][kFusedMax];  // c' of the edge left of pixel (il, jl)
};

// lane i receives lane i - 1 (lane 0 receives 0); the zero comes from the
// bound control, so the move can fold into the instruction that consumes it
__device__ __forceinline__ float from_left(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xF, 0xF, true));
}

// lane i receives lane i + 1 (lane 63 receives 0)
__device__ __forceinline__ float from_right(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xF, 0xF, false));
}

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

// ---- full tiles (h = w = 128) ----------------------------------------------
// Every thread owns two columns inside the tile and eight rows inside it, so
// the per-element guards of fused_step drop out and the few special edges are
// handled without divergent branches: the tile's top row (strip 0) and bottom
// row (strip 15) by wave-uniform branches, the left edges of column 0 by
// clamp bounds that collapse to 0 on the image boundary, and the right
// boundary column by lanes 0..7 of each strip after the row sweep (lane r
// updates row 8 s + r from the last column's d, passed through LDS).

struct FullCtx {
    int s, lane, ja, il0;
    // LDS element offsets il0 * 128 + ja, s * 128 + ja and il0 + lane.  full_step
    // passes them through opaque() once per step, so that each LDS access is a
    // base register plus an immediate offset computed inside the step, rather
    // than an address register hoisted out of the step loop and kept live.
    int oc, oy, olr;
    bool last;       // strip 15: owns the tile's bottom boundary edges
    bool right_bnd;  // the tile's right boundary edges lie on the image boundary
    // clamp bounds, (-1, 1) or (0, 0) for edges on the image boundary: the
    // top edges of the strip's first row, the left edge of column a, the
    // tile's bottom edges
    float lo1, hi1, lo2a, hi2a, lob, hib;
    float ak, kL;
    float qa, qb;  // recording: the weights of y and of d_b - d_a in the record word q
    // framed tiles only (a subdomain smaller than 128 x 128 run in a 128 x 128 frame): clamp
    // bounds of the left edge of column b, the strip's rows whose top edges are the tile's bottom
    // boundary on the image boundary (bit r: row 8 s + r), and, with masks, the strip's rows inside
    // the tile and whether columns a and b are inside it
    float lo2b, hi2b;
    unsigned zrows;
    unsigned mrows;
    bool lva, lvb;
};

__device__ __forceinline__ int opaque(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Marks four values as used here: their computation cannot sink below this
// point (the compiler otherwise moves every row update next to its use in the
// following step and keeps all rows' temporaries alive at once).
__device__ __forceinline__ void pin4(float &a, float &b, float &c, float &d)
{
    asm volatile("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d));
}

// 8-byte LDS access; p is 8-byte aligned (an even column of a row)
__device__ __forceinline__ void lds_ld2(const float *p, float &x, float &y)
{
    const float2 v = *reinterpret_cast<const float2 *>(__builtin_assume_aligned(p, 8));
    x = v.x;
    y = v.y;
}

__device__ __forceinline__ void lds_st2(float *p, float x, float y)
{
    *reinterpret_cast<float2 *>(__builtin_assume_aligned(p, 8)) = make_float2(x, y);
}

// lane i receives lane i + 1; lane 63 receives edge
__device__ __forceinline__ float from_right_or(float x, float edge)
{
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(x), 0x130, 0xF, 0xF, false));
}

// unscaled divergence of the two pixels of row r of a full tile; ry is y on
// the right boundary edge of the row
__device__ __forceinline__ void full_row_div(const Slot &Y, float ry, int r, float ya_below, float yb_below,
                                             float &da, float &db)
{
    const float yrb = from_right_or(Y.e2a[r], ry);
    da = div4(Y.e1a[r], ya_below, Y.e2a[r], Y.e2b[r]);
    db = div4(Y.e1b[r], yb_below, Y.e2b[r], yrb);
}

// fused_step on a full tile; same arithmetic per edge, hence the same result
// Record of one step on a full tile (reverse mode): kRecGroups groups of four
// words per thread of the workgroup (group g of thread t is the float4 at
// rec4[g * kRecThreads + t], dtvdd_internal.h):
//   g = 0..7  q = qa y + qb (d_b - d_a) on the edges e1a, e1b, e2a, e2b of row r = g:
//             the alpha derivative of z is (dA/tau)(phat - y) - dA (f_b - f_a)
//             - dB (d_b - d_a), and q carries its y-dependent part (qa = -dA/tau,
//             qb = -dB)
//   g = 8     q on the bottom boundary edges a, b (strip 15) and on the right
//             boundary edge of row 8 s + lane (lanes 0..7), each a NaN where the
//             projection is not differentiable there (|z| >= 1, an edge that is not a
//             variable, or a thread that holds no such edge), and the projection mask
//             of the 32 other edges (bit 4 r + i set when -1 < z < 1 on an edge that
//             is a variable)

// a framed tile with masks: d is 0 on the pixels outside the tile (row r of the strip)
__device__ __forceinline__ void dmask(const FullCtx &c, int r, float &da, float &db)
{
    const bool row = ((c.mrows >> r) & 1u) != 0;
    da = (row && c.lva) ? da : 0.0f;
    db = (row && c.lvb) ? db : 0.0f;
}

// projected step value and, when recording, the mask bit of its derivative
template <bool REC>
__device__ __forceinline__ float proj(float z, float lo, float hi, unsigned &m, int bit)
{
    if constexpr (REC) m |= (z > lo && z < hi) ? (1u << bit) : 0u;
    return __builtin_amdgcn_fmed3f(z, lo, hi);
}

// FR: a framed tile.  The tile's h x w pixels sit at the top left of the 128 x 128 frame; its
// bottom edges are the top edges of frame row h and its right edges the left edges of frame
// column w (the frame's own bottom row and right column when h or w is 128).  Outside the tile
// every edge starts at 0 with c' = 0.  A side on the image boundary is clamped to 0.
//   FR = 1: the short sides (h or w below 128) lie on the image boundary; their clamped edges
//           keep d = 0 on the pixels outside, so the tile's edges see exactly the values of a
//           tile of its own size.
//   FR = 2: any tile; d of the pixels outside is set to 0 (masks), so a short side may be an
//           interface whose copies are updated in the frame.
template <bool mom, bool REC = false, int FR = 0>
__device__ __forceinline__ void full_step(const FullCtx &c, FusedLds &S, const Slot &X, Slot &Y, int sx, float beta,
                                          float4 *rec = nullptr)
{
    // The phases are written without branches wherever a select does the job:
    // a branch splits the step into blocks and the compiler then sinks the row
    // updates towards their next use, keeping every row's temporaries alive.
    const int oc = opaque(c.oc), oy = opaque(c.oy), olr = opaque(c.olr), orow = opaque(c.il0);
    const float *RX = S.rx[sx];
    float *RY = S.rx[sx ^ 1];
    const float ak = c.ak, kL = c.kL;
    // (1) y on every owned edge; lanes 0..7 take the right boundary edges of the strip's rows
    if (c.lane < kR) RY[olr] = mom ? fista_y(RX[olr], RY[olr], beta) : RX[olr];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        Y.e1a[r] = mom ? fista_y(X.e1a[r], Y.e1a[r], beta) : X.e1a[r];
        Y.e1b[r] = mom ? fista_y(X.e1b[r], Y.e1b[r], beta) : X.e1b[r];
        Y.e2a[r] = mom ? fista_y(X.e2a[r], Y.e2a[r], beta) : X.e2a[r];
        Y.e2b[r] = mom ? fista_y(X.e2b[r], Y.e2b[r], beta) : X.e2b[r];
        pin4(Y.e1a[r], Y.e1b[r], Y.e2a[r], Y.e2b[r]);
    }
    if (REC || c.last) {  // the bottom boundary edges (strip 15)
        Y.ba = mom ? fista_y(X.ba, Y.ba, beta) : X.ba;
        Y.bb = mom ? fista_y(X.bb, Y.bb, beta) : X.bb;
    }
    float *yt = &S.yt[sx][0][0] + oy;  // this strip's row of the exchange buffer (strip 0's is unused)
    lds_st2(yt, Y.e1a[0], Y.e1b[0]);
    __syncthreads();

    // (2) d of the strip's last row, published for the strip below
    const float *RYr = RY + orow;  // y on the right boundary edges of the strip's rows (lane 63 uses them)
    float ya7, yb7;  // y on the edges below the last row
    lds_ld2(yt + kFusedMax, ya7, yb7);  // strip 15 reads a neighbouring array here and discards it
    ya7 = c.last ? Y.ba : ya7;
    yb7 = c.last ? Y.bb : yb7;
    float *dl = &S.dl[0][0] + oy;
    float da7, db7;  // d of the last row (the row sweep reuses it)
    full_row_div(Y, RYr[kR - 1], kR - 1, ya7, yb7, da7, db7);
    if constexpr (FR == 2) dmask(c, kR - 1, da7, db7);
    lds_st2(dl, da7, db7);
    __syncthreads();

    // (3) row sweep
    float dua, dub;  // d of the row above (0 above the tile)
    lds_ld2(dl - kFusedMax, dua, dub);  // strip 0 reads a neighbouring array here and discards it
    dua = c.s > 0 ? dua : 0.0f;
    dub = c.s > 0 ? dub : 0.0f;
    const float *c1 = &S.c1[0][0] + oc, *c2 = &S.c2[0][0] + oc;
    unsigned m0 = 0, m1 = 0;               // projection masks (recording)
    float qba = 0.0f, qbb = 0.0f, qr = 0.0f;  // q of the bottom and right boundary edges (recording)
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        __builtin_amdgcn_sched_barrier(0);  // one row at a time: bounds the registers in flight
        float da = da7, db = db7;
        if (r < kR - 1) {
            full_row_div(Y, RYr[r], r, Y.e1a[r + 1], Y.e1b[r + 1], da, db);
            if constexpr (FR == 2) dmask(c, r, da, db);
        }
        const float dlb = from_left(db);
        if constexpr (REC)
            rec[r * kRecThreads] =
                make_float4(fmaf(c.qb, dua - da, c.qa * Y.e1a[r]), fmaf(c.qb, dub - db, c.qa * Y.e1b[r]),
                            fmaf(c.qb, dlb - da, c.qa * Y.e2a[r]), fmaf(c.qb, da - db, c.qa * Y.e2b[r]));
        float c1a, c1b, c2a, c2b;
        lds_ld2(c1 + r * kFusedMax, c1a, c1b);
        lds_ld2(c2 + r * kFusedMax, c2a, c2b);
        // the top edges of the tile collapse to 0 on the image boundary (bounds lo1, hi1 on row 0),
        // and in a framed tile on its bottom boundary line
        float lo1 = r == 0 ? c.lo1 : -1.0f, hi1 = r == 0 ? c.hi1 : 1.0f;
        if constexpr (FR) {
            const bool zr = ((c.zrows >> r) & 1u) != 0;
            lo1 = zr ? 0.0f : lo1;
            hi1 = zr ? 0.0f : hi1;
        }
        Y.e1a[r] = proj<REC>(fista_z(Y.e1a[r], dua, da, c1a, ak, kL), lo1, hi1, m0, 4 * r + 0);
        Y.e1b[r] = proj<REC>(fista_z(Y.e1b[r], dub, db, c1b, ak, kL), lo1, hi1, m0, 4 * r + 1);
        Y.e2a[r] = proj<REC>(fista_z(Y.e2a[r], dlb, da, c2a, ak, kL), c.lo2a, c.hi2a, m0, 4 * r + 2);
        Y.e2b[r] = proj<REC>(fista_z(Y.e2b[r], da, db, c2b, ak, kL), FR ? c.lo2b : -1.0f, FR ? c.hi2b : 1.0f, m0,
                             4 * r + 3);
        // bottom boundary edges of the tile (strip 15; 0 on the image boundary).  The branch is
        // wave-uniform; the recording step keeps the straight line (fewer registers live).
        if (r == kR - 1 && (REC || c.last)) {
            float cba, cbb;
            lds_ld2(S.cb + (oy - c.s * kFusedMax), cba, cbb);
            if constexpr (REC) {
                qba = fmaf(c.qb, da, c.qa * Y.ba);
                qbb = fmaf(c.qb, db, c.qa * Y.bb);
            }
            // they collapse to 0 on the image boundary
            Y.ba = proj<REC>(fista_z(Y.ba, da, 0.0f, cba, ak, kL), c.lob, c.hib, m1, 0);
            Y.bb = proj<REC>(fista_z(Y.bb, db, 0.0f, cbb, ak, kL), c.lob, c.hib, m1, 1);
        }
        pin4(Y.e1a[r], Y.e1b[r], Y.e2a[r], Y.e2b[r]);
        // the last column's d, for the right boundary edges; stored after the row's updates so
        // that the lane shift of d above stays in one block with its use and folds into it
        if (c.lane == 63) S.dR[orow + r] = db;
        dua = da;
        dub = db;
    }
    if (c.lane < kR) {
        if constexpr (REC) qr = fmaf(c.qb, S.dR[olr], c.qa * RY[olr]);
        if (!c.right_bnd) {
            const float z = fista_z(RY[olr], S.dR[olr], 0.0f, S.cr[olr], ak, kL);
            RY[olr] = proj<REC>(z, -1.0f, 1.0f, m1, 2);
        }
    }
    if constexpr (REC) {
        const float nan = __builtin_nanf("");
        rec[8 * kRecThreads] = make_float4((m1 & 1u) ? qba : nan, (m1 & 2u) ? qbb : nan, (m1 & 4u) ? qr : nan,
                                           __uint_as_float(m0));
    }
}

struct GenericStep {
    template <bool mom>
    __device__ __forceinline__ static void step(const Ctx &c, FusedLds &S, const Slot &X, Slot &Y, int sx, float beta)
    {
        fused_step<mom>(c, S, X, Y, sx, beta);
    }
};

struct FullStep {
    template <bool mom>
    __device__ __forceinline__ static void step(const FullCtx &c, FusedLds &S, const Slot &X, Slot &Y, int sx,
                                                float beta)
    {
        full_step<mom>(c, S, X, Y, sx, beta);
    }
};

template <int FR>
struct FramedStep {
    template <bool mom>
    __device__ __forceinline__ static void step(const FullCtx &c, FusedLds &S, const Slot &X, Slot &Y, int sx,
                                                float beta)
    {
        full_step<mom, false, FR>(c, S, X, Y, sx, beta);
    }
};

// ---- adaptive inner stopping -------------------------------------------------
// The local solve of a subdomain stops after step k once
//   |x_k - x_{k-1}|_2 < tol |x_k|_2   (or x_k = x_{k-1})
// over all of the subdomain's edge dofs, or after the cap K.  Each thread sums
// its own edges in FP32; the sums are reduced per wave and over the 16 waves
// in FP64, in a fixed order, and every thread takes the same decision.

// Partial sums of |x_k - x_{k-1}|^2 and |x_k|^2 over the thread's edges: N
// holds x_k, O holds x_{k-1}; the right boundary edges are in LDS slots so ^ 1
// (x_k) and so (x_{k-1}).
__device__ __forceinline__ void conv_acc(float n, float o, float &dd, float &nn)
{
    const float d = n - o;
    dd = fmaf(d, d, dd);
    nn = fmaf(n, n, nn);
}

__device__ __forceinline__ void conv_sums(const Ctx &c, const FusedLds &S, const Slot &O, const Slot &N, int so,
                                          float &dd, float &nn)
{
#pragma unroll
    for (int r = 0; r < kR; ++r) {  // edges outside the tile hold 0 in both slots
        conv_acc(N.e1a[r], O.e1a[r], dd, nn);
        conv_acc(N.e1b[r], O.e1b[r], dd, nn);
        conv_acc(N.e2a[r], O.e2a[r], dd, nn);
        conv_acc(N.e2b[r], O.e2b[r], dd, nn);
    }
    if (c.has_bottom) {
        if (c.acta) conv_acc(N.ba, O.ba, dd, nn);
        if (c.actb) conv_acc(N.bb, O.bb, dd, nn);
    }
    if (c.lastcol_a || c.lastcol_b)
#pragma unroll
        for (int r = 0; r < kR; ++r)
            if (c.il0 + r < c.h) conv_acc(S.rx[so ^ 1][c.il0 + r], S.rx[so][c.il0 + r], dd, nn);
}

__device__ __forceinline__ void conv_sums(const FullCtx &c, const FusedLds &S, const Slot &O, const Slot &N, int so,
                                          float &dd, float &nn)
{
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        conv_acc(N.e1a[r], O.e1a[r], dd, nn);
        conv_acc(N.e1b[r], O.e1b[r], dd, nn);
        conv_acc(N.e2a[r], O.e2a[r], dd, nn);
        conv_acc(N.e2b[r], O.e2b[r], dd, nn);
    }
    if (c.last) {  // the bottom boundary edges are meaningful in strip 15 only
        conv_acc(N.ba, O.ba, dd, nn);
        conv_acc(N.bb, O.bb, dd, nn);
    }
    if (c.lane < kR) conv_acc(S.rx[so ^ 1][c.olr], S.rx[so][c.olr], dd, nn);  // lanes 0..7: right column
}

__device__ __forceinline__ double wave_sum_f64(double x)
{
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// red: 2 doubles per wave of LDS.  Reading red after the barrier is safe against
// the next step's writes: those come after the two barriers of that step.
__device__ __forceinline__ bool block_converged(int s, int lane, float dd, float nn, double tol2, double *red)
{
    const double d = wave_sum_f64((double)dd), n = wave_sum_f64((double)nn);
    if (lane == 0) {
        red[2 * s] = d;
        red[2 * s + 1] = n;
    }
    __syncthreads();
    double D = 0.0, N = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        D += red[2 * w];
        N += red[2 * w + 1];
    }
    return D == 0.0 || D < tol2 * N;
}

// Up to K steps from x_0 in A (B holds a copy) with the stopping rule above
// (tol2 = tol^2); x_k ends in A.  beta: the momentum table (beta[k], k >= 3).
// Returns the LDS slot of the right boundary edges holding x_k; taken = k.
template <class Step, class C>
__device__ __forceinline__ int run_steps_adaptive(const C &c, FusedLds &S, Slot &A, Slot &B, int K, const float *beta,
                                                  double tol2, double *red, int &taken)
{
    int k = 1;
    for (;; ++k) {
        float dd = 0.0f, nn = 0.0f;
        if (k & 1) {  // x_{k-1} in A (slot 0), x_k into B
            if (k >= 3) Step::template step<true>(c, S, A, B, 0, beta[k]);
            else Step::template step<false>(c, S, A, B, 0, 0.0f);
            if (k == K) break;
            conv_sums(c, S, A, B, 0, dd, nn);
        } else {      // x_{k-1} in B (slot 1), x_k into A
            if (k >= 3) Step::template step<true>(c, S, B, A, 1, beta[k]);
            else Step::template step<false>(c, S, B, A, 1, 0.0f);
            if (k == K) break;
            conv_sums(c, S, B, A, 1, dd, nn);
        }
        if (block_converged(c.s, c.lane, dd, nn, tol2, red)) break;
    }
    taken = k;
    if (k & 1) {
        copy_slot(A, B);
        return 1;
    }
    return 0;
}

// K projected-FISTA steps from x_0 in A (B holds a copy); x_K ends in A.
// Steps 1 and 2 have no momentum (beta = 0).  Returns the LDS slot of the
// right boundary edges that holds x_K.
template <class Step, class C>
__device__ __forceinline__ int run_steps(const C &c, FusedLds &S, Slot &A, Slot &B, int K, const float *beta)
{
    if (K == 1) {
        Step::template step<false>(c, S, A, B, 0, 0.0f);
        copy_slot(A, B);
        return 1;
    }
    Step::template step<false>(c, S, A, B, 0, 0.0f);
    Step::template step<false>(c, S, B, A, 1, 0.0f);
    int k = 3;
    for (; k + 1 <= K; k += 2) {
        Step::template step<true>(c, S, A, B, 0, beta[k]);
        Step::template step<true>(c, S, B, A, 1, beta[k + 1]);
    }
    if (k == K) {
        Step::template step<true>(c, S, A, B, 0, beta[K]);
        copy_slot(A, B);
        return 1;
    }
    return 0;
}

// The same K steps on a full tile with K known at compile time: fully
// unrolled, so the two slots never swap roles across a loop back-edge (which
// costs register copies, and spills where the caller keeps more state live).
// x_K ends in A when K is even and in B when K is odd; returns the LDS slot of
// the right boundary column holding it (K & 1).
template <int K, bool REC = false, int FR = 0, int k = 1>
__device__ __forceinline__ int full_steps_fixed(const FullCtx &c, FusedLds &S, Slot &X, Slot &Y, const float *beta,
                                                float4 *rec = nullptr, long long rec_step = 0)
{
    if constexpr (k <= K) {
        full_step<(k >= 3), REC, FR>(c, S, X, Y, (k - 1) & 1, k >= 3 ? beta[k] : 0.0f,
                                     REC ? rec + (k - 1) * rec_step : nullptr);
        return full_steps_fixed<K, REC, FR, k + 1>(c, S, Y, X, beta, rec, rec_step);
    } else {
        return K & 1;
    }
}

}  // namespace fused
}  // namespace dtv
