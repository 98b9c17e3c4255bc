// S consecutive local projected-FISTA steps k .. k + S - 1 (S = 2 .. 5) on the
// local dual ROF problems (eq. DD_local_dual, Sec. 5, Lee & Park, arXiv
// 1901.00682; FISTA of Beck and Teboulle) in one streaming launch over every
// subdomain.
//
// The one-step kernel (kernels.hip, k_fista_step) reads x_{k-1}, x_{k-2} and
// c' and writes x_k at every step (32 bytes per pixel and step).  Here the
// steps of a launch pass their iterates to each other in registers: a launch
// reads x_{k-1}, x_{k-2} and c' once (at k = 1: p~^n, the multipliers and f,
// from which it forms c') and writes its last iterate, the one before it when
// another launch of the outer step follows, and c' when the launch starts the
// outer step and is not its only one.  With all five steps of an outer step in
// one launch that is 20 bytes per pixel, the fused kernel's traffic, for
// subdomains of any size.
//
// Work decomposition and row sweep as in the multi-step primal-dual kernel
// (cp2_multi.hip): level L runs step k + L one row behind level L - 1, whose
// iterate on a row's bottom edge is the next row's top edge; the divergence
// d = div_s y of a level plays the part of u there (the level's update of a
// pixel's top edge needs d of the row above, of its left edge d of the lane to
// the left).  A wave stores the 65 - 2S columns of lanes S .. 64 - S; level L
// starts S - L rows above the strip and level 0 ends S - 1 rows below it.
//
// The per-element arithmetic is that of the one-step kernel (fista_ops.h), in
// the same order, so an S-step launch equals S one-step launches bitwise.
#include "fista_multi.h"
#include "fista_ops.h"

namespace dtv {

namespace {

// everything one row of the strip loads (the one-step kernel's row)
struct FistaMultiRow {
    int rw;                                   // row info word
    float xt, xtp, xb, xbp, xl, xlp, xr, xrp;  // x_{k-1}, x_{k-2} on the top, bottom, left, right edges
    float fv;                                 // f (k = 1)
    float lt, ll, lb, lr;                     // lambda on the interface copies among the edges (k = 1)
    float ct, cl, cb, cr;                     // c' of the four edges (k >= 2)
};

// what a level leaves of a row for the next level: its step's iterate (x_new), the iterate it read
// (x_old) and c' of the four edges
struct FistaMultiMid {
    int rw;                  // row info word
    float kt, kl, kb, kr;    // x_new on the top, left, bottom (last row), right (last column) edges
    float mt, ml, mb, mr;    // x_old on the top, left, bottom and right edges
    float ct, cl, cb, cr;
};

// element at byte offset off of a row base (one address register per lane: scalar base plus a
// 32-bit offset)
template <class T>
__device__ __forceinline__ T &fm_at(T *base, unsigned off)
{
    return *(T *)((char *)base + off);
}
template <class T>
__device__ __forceinline__ const T &fm_at(const T *base, unsigned off)
{
    return *(const T *)((const char *)base + off);
}

// waves per SIMD asked of an S-step kernel (the most whose registers hold every value)
constexpr int fista_multi_waves(int S) { return S <= 2 ? 5 : (S == 3 ? 4 : 3); }

}  // namespace

// MODE: the first step's kind (kFistaFirst: k = 1, forms c'; kFistaPlain: k = 2; kFistaMomentum:
// k >= 3, extrapolates).  Step k + L extrapolates when k + L >= 3, which MODE fixes for every level.
template <int R, int S, int MODE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(fista_multi_waves(S)))) void k_fista_multi(
    FistaMultiArgs a)
{
    constexpr bool FIRST = MODE == kFistaFirst, EXT = MODE == kFistaMomentum;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const StreamTile tile = a.tiles[t];
    const ImgDev im = a.imgs[tile.img];
    const int lane = threadIdx.x;
    const int H = im.H, W = im.W;
    const int j = tile.j0 - S + lane;
    const bool colok = (j >= 0) && (j < W);
    const int cw = colok ? a.info[im.cinfo + j] : 0;
    const int cs = info_sub(cw);
    const bool cfirst = info_first(cw), clast = info_last(cw);
    const int left = j + cs;
    const bool outlane = colok && lane >= S && lane <= 64 - S;
    // every access below is a row base shared by the wave plus one of these 32-bit byte offsets
    // (the loads and stores of lanes inside the image only, where they are nonnegative)
    const unsigned uj = 4u * (unsigned)j, ul = 4u * (unsigned)left;
    const long long P1 = im.pitch1, P2 = im.pitch2;

    // the outputs alias none of the inputs (distinct buffers)
    const float *__restrict__ xa1 = a.xa1 + im.p1;
    const float *__restrict__ xa2 = a.xa2 + im.p2;
    const float *__restrict__ xb1 = EXT ? a.xb1 + im.p1 : nullptr;
    const float *__restrict__ xb2 = EXT ? a.xb2 + im.p2 : nullptr;
    const float *__restrict__ lam = a.lam + im.lam;
    const float *__restrict__ f = a.f + im.px;
    float *__restrict__ c1 = a.c1 + im.p1;
    float *__restrict__ c2 = a.c2 + im.p2;
    float *__restrict__ ka1 = a.outk1 + im.p1;
    float *__restrict__ ka2 = a.outk2 + im.p2;
    float *__restrict__ kb1 = a.outn1 + im.p1;
    float *__restrict__ kb2 = a.outn2 + im.p2;
    const float tau = a.tau, itau = a.inv_tau;
    const float invL = im.invL, ak = im.a_keep, kL = im.kL;
    const bool store_c = FIRST && a.store_c != 0, store_prev = a.store_prev != 0;

    // y of level 0 (step k) and of level L from the two iterates on an edge
    auto yv0 = [&](float x, float xp) -> float {
        if constexpr (EXT) return fista_y(x, xp, a.beta[0]);
        return x;
    };
    auto yv = [&](int L, float x, float xp) -> float {
        const bool mom = MODE == kFistaFirst ? L >= 2 : (MODE == kFistaPlain ? L >= 1 : true);
        return mom ? fista_y(x, xp, a.beta[L]) : x;
    };

    const int i0 = tile.i0;
    const int iend = min(i0 + R, H);
    const int ra = max(i0 - S, 0);            // first row of level 0
    const int rb = min(iend + S - 2, H - 1);  // last row of level 0
    const int ilast = iend + S - 2;           // the last level reaches row iend - 1 here

    auto load_row = [&](int i, FistaMultiRow &r, bool top) {
        r.rw = a.info[im.rinfo + i];
        const int rs = info_sub(r.rw);
        const bool rfirst = info_first(r.rw), rlast = info_last(r.rw);
        const long long tp = i + rs;
        r.xt = r.xtp = r.xb = r.xbp = r.xl = r.xlp = r.xr = r.xrp = 0.0f;
        r.fv = r.lt = r.ll = r.lb = r.lr = 0.0f;
        r.ct = r.cl = r.cb = r.cr = 0.0f;
        if (colok) {
            if (rfirst || top) {
                r.xt = fm_at(xa1 + tp * P1, uj);
                if constexpr (EXT) r.xtp = fm_at(xb1 + tp * P1, uj);
            }
            r.xb = fm_at(xa1 + (tp + 1) * P1, uj);
            r.xl = fm_at(xa2 + i * P2, ul);
            r.xr = fm_at(xa2 + i * P2 + 1, ul);
            if constexpr (EXT) {
                r.xbp = fm_at(xb1 + (tp + 1) * P1, uj);
                r.xlp = fm_at(xb2 + i * P2, ul);
                r.xrp = fm_at(xb2 + i * P2 + 1, ul);
            }
            if constexpr (FIRST) {
                r.fv = fm_at(f + (long long)i * W, uj);
                if (rfirst && i > 0) r.lt = fm_at(lam + (long long)(rs - 1) * W, uj);
                if (cfirst && j > 0) r.ll = fm_at(lam + im.nlh + i, 4u * (unsigned)((cs - 1) * H));
                if (rlast && i < H - 1) r.lb = fm_at(lam + (long long)rs * W, uj);
                if (clast && j < W - 1) r.lr = fm_at(lam + im.nlh + i, 4u * (unsigned)(cs * H));
            } else {
                r.ct = fm_at(c1 + tp * P1, uj);
                r.cb = fm_at(c1 + (tp + 1) * P1, uj);
                r.cl = fm_at(c2 + i * P2, ul);
                r.cr = fm_at(c2 + i * P2 + 1, ul);
            }
        }
    };

    float d_up[S];  // per level: d of the row above
#pragma unroll
    for (int L = 0; L < S; ++L) d_up[L] = 0.0f;

    // level L >= 1 (step k + L) on row q from level L - 1's values of the row (m) and its new iterate
    // on the row's bottom edge (kbot: the next row's top edge, or the row's own bottom edge at the
    // last row of a subdomain); the last level stores its iterate (and the one it read, when the
    // next launch extrapolates from it) for rows inside the strip, the others fill o for the level
    // after them.  Every lane computes: the lanes outside the image feed no lane inside it, since
    // column 0 is a first column and column W - 1 a last one, and they store nothing.
    auto level = [&](int L, int q, const FistaMultiMid &m, float kbot, FistaMultiMid &o) {
        const int rw = m.rw;
        const bool rfirst = info_first(rw), rlast = info_last(rw);
        const long long tp = q + info_sub(rw);
        if (rfirst) d_up[L] = 0.0f;
        // x_old of this level on the right edge: the next lane's left edge, or the column's own at a
        // subdomain's last column
        const float kr_next = __shfl_down(m.kl, 1, 64);
        const float krr = clast ? m.kr : kr_next;
        const float yt = yv(L, m.kt, m.mt), yb = yv(L, kbot, m.mb);
        const float yl = yv(L, m.kl, m.ml), yr = yv(L, krr, m.mr);
        const float d = div4(yt, yb, yl, yr);
        float d_left = __shfl_up(d, 1, 64);
        if (cfirst) d_left = 0.0f;
        const float nt = q > 0 ? clamp1(fista_z(yt, d_up[L], d, m.ct, ak, kL)) : 0.0f;
        const float nl = j > 0 ? clamp1(fista_z(yl, d_left, d, m.cl, ak, kL)) : 0.0f;
        const float nb = (rlast && q < H - 1) ? clamp1(fista_z(yb, d, 0.0f, m.cb, ak, kL)) : 0.0f;
        const float nr = (clast && j < W - 1) ? clamp1(fista_z(yr, d, 0.0f, m.cr, ak, kL)) : 0.0f;
        if (L == S - 1) {
            if (outlane && q >= i0 && q < iend) {
                if (q > 0) {
                    fm_at(kb1 + tp * P1, uj) = nt;
                    if (store_prev) fm_at(ka1 + tp * P1, uj) = m.kt;
                }
                if (j > 0) {
                    fm_at(kb2 + q * P2, ul) = nl;
                    if (store_prev) fm_at(ka2 + q * P2, ul) = m.kl;
                }
                if (rlast && q < H - 1) {
                    fm_at(kb1 + (tp + 1) * P1, uj) = nb;
                    if (store_prev) fm_at(ka1 + (tp + 1) * P1, uj) = m.kb;
                }
                if (clast && j < W - 1) {
                    fm_at(kb2 + q * P2 + 1, ul) = nr;
                    if (store_prev) fm_at(ka2 + q * P2 + 1, ul) = m.kr;
                }
            }
        } else {
            o.rw = m.rw;
            o.kt = nt;
            o.kl = nl;
            o.kb = nb;
            o.kr = nr;
            o.mt = m.kt;
            o.ml = m.kl;
            o.mb = kbot;
            o.mr = krr;
            o.ct = m.ct;
            o.cl = m.cl;
            o.cb = m.cb;
            o.cr = m.cr;
        }
        d_up[L] = d;
    };

    float y_carry = 0.0f, x_carry = 0.0f, f_up = 0.0f;  // level 0: y, x_{k-1} and f of the row above
    bool have = false;
    FistaMultiMid prev[S];  // prev[L], L >= 1: level L - 1's row waiting for level L
    bool pend[S];
#pragma unroll
    for (int L = 0; L < S; ++L) pend[L] = false;

    // levels 1 .. S - 1 at iteration i: level L on row i - L, now that level L - 1's iterate on its
    // bottom edge is known (mo: the row level 0 produced at this iteration, if has)
    auto levels = [&](int i, FistaMultiMid mo, bool has) {
#pragma unroll
        for (int L = 1; L < S; ++L) {
            FistaMultiMid out;
            bool has_out = false;
            if (pend[L]) {
                // the image's last row is the last row of its subdomain: past the image's end, no
                // level needs the level before it
                const float kbot = info_last(prev[L].rw) ? prev[L].kb : mo.kt;
                level(L, i - L, prev[L], kbot, out);
                has_out = L < S - 1;
            }
            if (has) prev[L] = mo;
            pend[L] = has && i - L + 1 >= max(i0 - (S - L), 0);
            mo = out;
            has = has_out;
        }
    };

    FistaMultiRow cur, nxt;
    load_row(ra, cur, true);
    for (int i = ra; i <= rb; ++i) {
        // ---- level 0 (step k) on row i
        if (i + 1 <= rb) load_row(i + 1, nxt, false);
        const int rs = info_sub(cur.rw);
        const bool rfirst = info_first(cur.rw), rlast = info_last(cur.rw);
        const long long tp = i + rs;
        if (rfirst) {
            have = false;
            d_up[0] = 0.0f;
            f_up = 0.0f;
        }
        float d = 0.0f, yt = 0.0f, yb = 0.0f, yl = 0.0f, yr = 0.0f, xt = cur.xt;
        if (colok) {
            yt = have ? y_carry : yv0(cur.xt, cur.xtp);
            if (have) xt = x_carry;
            yb = yv0(cur.xb, cur.xbp);
            yl = yv0(cur.xl, cur.xlp);
            yr = yv0(cur.xr, cur.xrp);
            d = div4(yt, yb, yl, yr);
        }
        float d_left = __shfl_up(d, 1, 64);
        float f_left = 0.0f;
        if constexpr (FIRST) f_left = __shfl_up(cur.fv, 1, 64);
        if (cfirst) {
            d_left = 0.0f;
            f_left = 0.0f;
        }
        FistaMultiMid mo;
        mo.rw = cur.rw;
        if constexpr (FIRST) {
            // c' from the anchor phat = p~^n -/+ tau lambda on the t / s copies of interface edges
            mo.ct = fista_cprime(rfirst ? fmaf(tau, cur.lt, yt) : yt, f_up, cur.fv, itau, invL);
            mo.cl = fista_cprime(cfirst ? fmaf(tau, cur.ll, yl) : yl, f_left, cur.fv, itau, invL);
            mo.cb = fista_cprime(fmaf(-tau, cur.lb, yb), cur.fv, 0.0f, itau, invL);
            mo.cr = fista_cprime(fmaf(-tau, cur.lr, yr), cur.fv, 0.0f, itau, invL);
            if (store_c && outlane && i >= i0 && i < iend) {
                if (i > 0) fm_at(c1 + tp * P1, uj) = mo.ct;
                if (j > 0) fm_at(c2 + i * P2, ul) = mo.cl;
                if (rlast && i < H - 1) fm_at(c1 + (tp + 1) * P1, uj) = mo.cb;
                if (clast && j < W - 1) fm_at(c2 + i * P2 + 1, ul) = mo.cr;
            }
        } else {
            mo.ct = cur.ct;
            mo.cl = cur.cl;
            mo.cb = cur.cb;
            mo.cr = cur.cr;
        }
        mo.kt = i > 0 ? clamp1(fista_z(yt, d_up[0], d, mo.ct, ak, kL)) : 0.0f;
        mo.kl = j > 0 ? clamp1(fista_z(yl, d_left, d, mo.cl, ak, kL)) : 0.0f;
        mo.kb = (rlast && i < H - 1) ? clamp1(fista_z(yb, d, 0.0f, mo.cb, ak, kL)) : 0.0f;
        mo.kr = (clast && j < W - 1) ? clamp1(fista_z(yr, d, 0.0f, mo.cr, ak, kL)) : 0.0f;
        mo.mt = xt;
        mo.ml = cur.xl;
        mo.mb = cur.xb;
        mo.mr = cur.xr;
        d_up[0] = d;
        y_carry = yb;
        x_carry = cur.xb;
        f_up = cur.fv;
        have = true;
        cur = nxt;
        levels(i, mo, true);
    }
    // the strip reaches the image's last row: the later levels finish the rows below their lag
    for (int i = rb + 1; i <= ilast; ++i) levels(i, FistaMultiMid{}, false);
}

namespace {

template <int R, int S, int MODE>
hipError_t fm_launch(const FistaMultiArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    auto k = k_fista_multi<R, S, MODE>;
    if (e0 || e1)
        hipExtLaunchKernelGGL(k, dim3(a.ntiles), dim3(64), 0, s, e0, e1, 0, a);
    else
        hipLaunchKernelGGL(k, dim3(a.ntiles), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <int R, int S>
hipError_t fm_mode(const FistaMultiArgs &a, int mode, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    switch (mode) {
    case kFistaFirst: return fm_launch<R, S, kFistaFirst>(a, s, e0, e1);
    case kFistaPlain: return fm_launch<R, S, kFistaPlain>(a, s, e0, e1);
    default: return fm_launch<R, S, kFistaMomentum>(a, s, e0, e1);
    }
}

template <int R>
hipError_t fm_steps(const FistaMultiArgs &a, int mode, int steps, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    switch (steps) {
    case 2: return fm_mode<R, 2>(a, mode, s, e0, e1);
    case 3: return fm_mode<R, 3>(a, mode, s, e0, e1);
    case 4: return fm_mode<R, 4>(a, mode, s, e0, e1);
    case 5: return fm_mode<R, 5>(a, mode, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_fista_multi(const FistaMultiArgs &a, int mode, int rows, int steps, hipStream_t s, hipEvent_t e0,
                              hipEvent_t e1)
{
    if (a.ntiles <= 0) return hipSuccess;
    switch (rows) {
    case 4: return fm_steps<4>(a, mode, steps, s, e0, e1);
    case 8: return fm_steps<8>(a, mode, steps, s, e0, e1);
    case 16: return fm_steps<16>(a, mode, steps, s, e0, e1);
    case 32: return fm_steps<32>(a, mode, steps, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace dtv
