// S consecutive local steps k .. k + S - 1 (S = 2 .. 5) of the accelerated
// primal-dual solver (Chambolle-Pock Alg. 2 on the local saddle problems
// eq. (local) of Sec. 5, Lee & Park, arXiv 1901.00682) in one streaming launch
// over every subdomain.
//
// The one-step kernel (kernels.hip) reads x_{k-1}, x_{k-2}, the anchor, u, f
// and the mask and writes x_k and u_k at every step.  Here the steps of a
// launch pass their results to each other in registers: per launch the kernel
// reads that input once and writes x_{k+S-1}, u_{k+S-1} and, when another
// launch of the outer step follows (it extrapolates from the last two
// iterates), x_{k+S-2}: about 53 bytes per pixel for any S, 29 for all five
// steps of an outer step in one launch, against 45 per step for one-step
// launches.
//
// Work decomposition as in the one-step kernel: a 64-lane wave owns a strip
// of R rows and 64 consecutive columns.  Level L of the launch runs step
// k + L.  At a pixel it needs level L - 1's iterate on the pixel's right edge
// (the left edge of the next lane's pixel), and its iterate on a pixel's left
// edge needs its u of the lane to the left, so each level loses one lane on
// the right and one on the left: lanes 0 .. S - 1 are halo columns, lanes
// above 64 - S compute only what the lanes left of them read, and each wave
// writes the 65 - 2S columns of lanes S .. 64 - S.  Rows are swept top to
// bottom; level L runs L rows behind level 0, since level L - 1's iterate on
// a row's bottom edge is the top edge of the row below.  Level L starts
// S - L rows above the strip (the last level needs u of the row above the
// strip, which needs level S - 2 on two rows above it, ...) and level 0 ends
// S - 1 rows below it; those halo rows are computed and not stored.
// Subdomain boundaries inside a strip reset the carried values exactly as in
// the one-step kernel.
//
// The per-element arithmetic is that of the one-step kernel (cp2_ops.h), in
// the same order, so an S-step launch equals S one-step launches bitwise.
//
// With S = 5 a wave keeps four rows in flight besides the one being loaded
// (about 150 VGPRs, three waves per SIMD), so the launch is bound by issue and
// latency rather than by HBM: the fidelity is a template parameter (no branch
// on it in any level), the levels after the first compute on every lane
// without a branch, and every load and store addresses a wave-uniform row base
// plus a 32-bit lane offset, one address register per lane instead of a
// 64-bit address per array.
#include "cp2_multi.h"
#include "cp2_ops.h"
#include "dtvdd.h"
#include "fista_ops.h"

namespace dtv {

namespace {

// everything one row of the strip loads (the one-step kernel's row)
struct MultiRow {
    int rw;                                   // row info word
    float xt, xtp, xb, xbp, xl, xlp, xr, xrp;  // x_{k-1}, x_{k-2} on the top, bottom, left, right edges
    float uv, fv;                             // u_{k-1}, f
    float at, al, ab, ar;                     // anchors p~^n of the four edges
    float lt, ll, lb, lr;                     // lambda on the interface copies among them
    unsigned mv;                              // observed (mask byte)
};

// what a level leaves of a row for the next level: its step's u and iterate (x_new) and the iterate
// it read (x_old)
struct MultiMid {
    int rw;                            // row info word, with bit 31 set when the pixel is observed
    float u;
    float kt, kl, kb, kr;              // x_new on the top, left, bottom (last row), right (last column) edges
    float mt, ml, mb, mr;              // x_old on the top, left, bottom and right edges
    float fv;
    float at, al, ab, ar;              // the anchors phat of the four edges (-/+ tau lambda on interface copies)
};

// element at byte offset off of a row base: with the base the same for the whole wave and a 32-bit
// offset the access takes one address register per lane (scalar base plus offset)
template <class T>
__device__ __forceinline__ T &at_byte(T *base, unsigned off)
{
    return *(T *)((char *)base + off);
}
template <class T>
__device__ __forceinline__ const T &at_byte(const T *base, unsigned off)
{
    return *(const T *)((const char *)base + off);
}

// waves per SIMD asked of an S-step kernel: the launch is bound by memory latency, and each level
// keeps a row of values in registers
constexpr int multi_waves(int S) { return S <= 2 ? 5 : (S == 3 ? 4 : 3); }

}  // namespace

// EXT: step k extrapolates xbar_{k-1} = x_{k-1} + theta_{k-1} (x_{k-1} - x_{k-2}) (k >= 2); every
// later level always extrapolates the iterate of the level before it.  FID: the fidelity (DTV_L2,
// DTV_L1, DTV_CV), fixed at compile time so that no level branches on it.
template <int R, bool EXT, int S, int FID>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(multi_waves(S)))) void k_cp2_multi(
    Cp2MultiArgs a)
{
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
    const float *__restrict__ b1 = a.base1 + im.p1;
    const float *__restrict__ b2 = a.base2 + im.p2;
    const float *__restrict__ lam = a.lam + im.lam;
    const float *__restrict__ f = a.f + im.px;
    const uint8_t *__restrict__ mk = a.mask ? a.mask + im.px : nullptr;
    const float *__restrict__ uin = a.u_in + im.px;
    float *__restrict__ uout = a.u_out + im.px;
    float *__restrict__ ka1 = a.outk1 + im.p1;
    float *__restrict__ ka2 = a.outk2 + im.p2;
    float *__restrict__ kb1 = a.outn1 + im.p1;
    float *__restrict__ kb2 = a.outn2 + im.p2;
    const float tau = a.tau;
    const float cv1 = a.cv_c1, cv2 = a.cv_c2;
    const bool store_prev = a.store_prev != 0;

    auto xbar0 = [&](float x, float xp) -> float {
        if constexpr (EXT) return fmaf(a.theta[0], x - xp, x);
        return x;
    };
    auto xbar = [&](int L, float x, float xp) -> float { return fmaf(a.theta[L], x - xp, x); };
    auto pup = [&](int L, float x, float du, float anchor) -> float {
        return clamp1(cp2_pre(x, du, anchor, a.tk[L], a.ck[L], a.ca[L]));
    };

    const int i0 = tile.i0;
    const int iend = min(i0 + R, H);
    const int ra = max(i0 - S, 0);            // first row of level 0
    const int rb = min(iend + S - 2, H - 1);  // last row of level 0
    const int ilast = iend + S - 2;           // the last level reaches row iend - 1 here

    auto load_row = [&](int i, MultiRow &r, bool top) {
        r.rw = a.info[im.rinfo + i];
        const int rs = info_sub(r.rw);
        const bool rfirst = info_first(r.rw), rlast = info_last(r.rw);
        const long long tp = i + rs;
        const long long row = (long long)i * W;
        r.xt = r.xtp = r.xb = r.xbp = r.xl = r.xlp = r.xr = r.xrp = 0.0f;
        r.uv = r.fv = r.at = r.al = r.ab = r.ar = 0.0f;
        r.lt = r.ll = r.lb = r.lr = 0.0f;
        r.mv = 1;
        if (colok) {
            if (mk) r.mv = (mk + row)[(unsigned)j];
            if (rfirst || top) {
                r.xt = at_byte(xa1 + tp * P1, uj);
                if constexpr (EXT) r.xtp = at_byte(xb1 + tp * P1, uj);
            }
            r.xb = at_byte(xa1 + (tp + 1) * P1, uj);
            r.xl = at_byte(xa2 + i * P2, ul);
            r.xr = at_byte(xa2 + i * P2 + 1, ul);
            if constexpr (EXT) {
                r.xbp = at_byte(xb1 + (tp + 1) * P1, uj);
                r.xlp = at_byte(xb2 + i * P2, ul);
                r.xrp = at_byte(xb2 + i * P2 + 1, ul);
            }
            r.uv = at_byte(uin + row, uj);
            r.fv = at_byte(f + row, uj);
            r.at = at_byte(b1 + tp * P1, uj);
            r.ab = at_byte(b1 + (tp + 1) * P1, uj);
            r.al = at_byte(b2 + i * P2, ul);
            r.ar = at_byte(b2 + i * P2 + 1, ul);
            if (rfirst && i > 0) r.lt = at_byte(lam + (long long)(rs - 1) * W, uj);
            if (cfirst && j > 0) r.ll = at_byte(lam + im.nlh + i, 4u * (unsigned)((cs - 1) * H));
            if (rlast && i < H - 1) r.lb = at_byte(lam + (long long)rs * W, uj);
            if (clast && j < W - 1) r.lr = at_byte(lam + im.nlh + i, 4u * (unsigned)(cs * H));
        }
    };

    float u_up[S];  // per level: u of the row above
#pragma unroll
    for (int L = 0; L < S; ++L) u_up[L] = 0.0f;

    // level L >= 1 (step k + L) on row q from level L - 1's values of the row (m) and its new iterate
    // on the row's bottom edge (kbot: the next row's top edge, or the row's own bottom edge at the
    // last row of a subdomain); the last level stores u, x_old and x_new of rows inside the strip,
    // the others fill o for the level after them.  Every lane computes (no branch): the lanes
    // outside the image feed no lane inside it, since column 0 is a first column and column W - 1 a
    // last one, and they store nothing.
    auto level = [&](int L, int q, const MultiMid &m, float kbot, MultiMid &o) {
        const int rw = m.rw & 0x7FFFFFFF;
        const bool rfirst = info_first(rw), rlast = info_last(rw);
        const long long tp = q + info_sub(rw);
        if (rfirst) u_up[L] = 0.0f;
        // x_old of this level on the right edge: the next lane's left edge, or the column's own at a
        // subdomain's last column
        const float kr_next = __shfl_down(m.kl, 1, 64);
        const float krr = clast ? m.kr : kr_next;
        const float bxt = xbar(L, m.kt, m.mt);
        const float bxb = xbar(L, kbot, m.mb);
        const float d = (bxb - bxt) + (xbar(L, krr, m.mr) - xbar(L, m.kl, m.ml));
        const float u1 = cp2_u(FID, m.u, d, a.sk[L], m.fv, m.rw < 0, a.sk[L] * im.alpha, cv1, cv2);
        float u_left = __shfl_up(u1, 1, 64);
        if (cfirst) u_left = 0.0f;
        const float nt = q > 0 ? pup(L, m.kt, u_up[L] - u1, m.at) : 0.0f;
        const float nl = j > 0 ? pup(L, m.kl, u_left - u1, m.al) : 0.0f;
        const float nb = (rlast && q < H - 1) ? pup(L, m.kb, u1, m.ab) : 0.0f;
        const float nr = (clast && j < W - 1) ? pup(L, m.kr, u1, m.ar) : 0.0f;
        if (L == S - 1) {
            if (outlane && q >= i0 && q < iend) {
                at_byte(uout + (long long)q * W, uj) = u1;
                if (q > 0) {
                    if (store_prev) at_byte(ka1 + tp * P1, uj) = m.kt;
                    at_byte(kb1 + tp * P1, uj) = nt;
                }
                if (j > 0) {
                    if (store_prev) at_byte(ka2 + q * P2, ul) = m.kl;
                    at_byte(kb2 + q * P2, ul) = nl;
                }
                if (rlast && q < H - 1) {
                    if (store_prev) at_byte(ka1 + (tp + 1) * P1, uj) = m.kb;
                    at_byte(kb1 + (tp + 1) * P1, uj) = nb;
                }
                if (clast && j < W - 1) {
                    if (store_prev) at_byte(ka2 + q * P2 + 1, ul) = m.kr;
                    at_byte(kb2 + q * P2 + 1, ul) = nr;
                }
            }
        } else {
            o.rw = m.rw;
            o.u = u1;
            o.kt = nt;
            o.kl = nl;
            o.kb = nb;
            o.kr = nr;
            o.mt = m.kt;
            o.ml = m.kl;
            o.mb = kbot;
            o.mr = krr;
            o.fv = m.fv;
            o.at = m.at;
            o.al = m.al;
            o.ab = m.ab;
            o.ar = m.ar;
        }
        u_up[L] = u1;
    };

    float xbar_carry = 0.0f, x_carry = 0.0f;  // level 0: xbar and x_{k-1} on the bottom edge of the row above
    bool have = false;
    MultiMid prev[S];  // prev[L], L >= 1: level L - 1's row waiting for level L
    bool pend[S];
#pragma unroll
    for (int L = 0; L < S; ++L) pend[L] = false;

    // levels 1 .. S - 1 at iteration i: level L on row i - L, now that level L - 1's iterate on its
    // bottom edge is known (mo: the row level 0 produced at this iteration, if has)
    auto levels = [&](int i, MultiMid mo, bool has) {
#pragma unroll
        for (int L = 1; L < S; ++L) {
            MultiMid out;
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

    MultiRow cur, nxt;
    load_row(ra, cur, true);
    for (int i = ra; i <= rb; ++i) {
        // ---- level 0 (step k) on row i: u_k of the pixel from xbar_{k-1} on its four edges
        if (i + 1 <= rb) load_row(i + 1, nxt, false);
        const bool rfirst = info_first(cur.rw), rlast = info_last(cur.rw);
        if (rfirst) {
            have = false;
            u_up[0] = 0.0f;
        }
        float u = 0.0f, bxb = 0.0f, xt = cur.xt;
        if (colok) {
            const float bxt = have ? xbar_carry : xbar0(cur.xt, cur.xtp);
            if (have) xt = x_carry;
            bxb = xbar0(cur.xb, cur.xbp);
            const float d = (bxb - bxt) + (xbar0(cur.xr, cur.xrp) - xbar0(cur.xl, cur.xlp));
            u = cp2_u(FID, cur.uv, d, a.sk[0], cur.fv, cur.mv != 0, a.sk[0] * im.alpha, cv1, cv2);
        }
        float u_left = __shfl_up(u, 1, 64);
        if (cfirst) u_left = 0.0f;
        // x_k on the row's edges (0 on the image boundary, where the buffers hold 0)
        MultiMid mo;
        mo.rw = cur.rw | (cur.mv != 0 ? (int)0x80000000u : 0);
        mo.u = u;
        // the anchors of every level: t copies + tau lambda, s copies - tau lambda
        mo.at = rfirst ? fmaf(tau, cur.lt, cur.at) : cur.at;
        mo.al = cfirst ? fmaf(tau, cur.ll, cur.al) : cur.al;
        mo.ab = fmaf(-tau, cur.lb, cur.ab);
        mo.ar = fmaf(-tau, cur.lr, cur.ar);
        mo.kt = i > 0 ? pup(0, xt, u_up[0] - u, mo.at) : 0.0f;
        mo.kl = j > 0 ? pup(0, cur.xl, u_left - u, mo.al) : 0.0f;
        mo.kb = (rlast && i < H - 1) ? pup(0, cur.xb, u, mo.ab) : 0.0f;
        mo.kr = (clast && j < W - 1) ? pup(0, cur.xr, u, mo.ar) : 0.0f;
        mo.mt = xt;
        mo.ml = cur.xl;
        mo.mb = cur.xb;
        mo.mr = cur.xr;
        mo.fv = cur.fv;
        u_up[0] = u;
        xbar_carry = bxb;
        x_carry = cur.xb;
        have = true;
        cur = nxt;
        levels(i, mo, true);
    }
    // the strip reaches the image's last row: the later levels finish the rows below their lag
    for (int i = rb + 1; i <= ilast; ++i) levels(i, MultiMid{}, false);
}

namespace {

template <int R, int S, int FID>
hipError_t multi_launch(const Cp2MultiArgs &a, bool ext, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    auto k = ext ? k_cp2_multi<R, true, S, FID> : k_cp2_multi<R, false, S, FID>;
    if (e0 || e1)
        hipExtLaunchKernelGGL(k, dim3(a.ntiles), dim3(64), 0, s, e0, e1, 0, a);
    else
        hipLaunchKernelGGL(k, dim3(a.ntiles), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <int R, int S>
hipError_t multi_fid(const Cp2MultiArgs &a, bool ext, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    switch (a.fidelity) {
    case DTV_L2: return multi_launch<R, S, DTV_L2>(a, ext, s, e0, e1);
    case DTV_L1: return multi_launch<R, S, DTV_L1>(a, ext, s, e0, e1);
    case DTV_CV: return multi_launch<R, S, DTV_CV>(a, ext, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

template <int R>
hipError_t multi_rows(const Cp2MultiArgs &a, bool ext, int steps, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    switch (steps) {
    case 2: return multi_fid<R, 2>(a, ext, s, e0, e1);
    case 3: return multi_fid<R, 3>(a, ext, s, e0, e1);
    case 4: return multi_fid<R, 4>(a, ext, s, e0, e1);
    case 5: return multi_fid<R, 5>(a, ext, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_cp2_multi(const Cp2MultiArgs &a, bool extrapolate, int rows, int steps, hipStream_t s, hipEvent_t e0,
                            hipEvent_t e1)
{
    if (a.ntiles <= 0) return hipSuccess;
    switch (rows) {
    case 4: return multi_rows<4>(a, extrapolate, steps, s, e0, e1);
    case 8: return multi_rows<8>(a, extrapolate, steps, s, e0, e1);
    case 16: return multi_rows<16>(a, extrapolate, steps, s, e0, e1);
    case 32: return multi_rows<32>(a, extrapolate, steps, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace dtv
