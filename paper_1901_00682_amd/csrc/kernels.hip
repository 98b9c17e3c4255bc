// HIP kernels of libdtvdd.so for gfx950: the streaming schedule of
// Algorithm 1 (Lee & Park, arXiv 1901.00682, Sec. 4) -- one launch per inner
// step over every subdomain of every image -- plus the multiplier update,
// the primal recovery and the FP64 diagnostics.
//
// Work decomposition of the step kernels: one 64-lane wave owns a strip of
// R pixel rows and 64 consecutive columns; lane 0 is a halo column whose
// values are only used by lane 1, so each wave writes 63 columns and all
// loads and stores of a row are coalesced.  Rows are swept top to bottom so
// the edge shared by two vertically adjacent pixels of the same subdomain is
// loaded once and the value of the pixel above stays in a register; the
// value of the left neighbour comes from the lane to the left by a shuffle.
// Subdomain membership comes from per-row / per-column info words, so tiles
// of any size (ragged ones included) need no special cases.
//
// Arithmetic is FP32 with explicit fmaf where a fused multiply-add is meant
// (the library is built with -ffp-contract=off so that the streaming and
// fused schedules round identically).
#include <algorithm>

#include "dtvdd_internal.h"
#include "cp2_ops.h"
#include "fista_ops.h"

namespace dtv {

// ---------------------------------------------------------------------------
// (a1) multiplier update, one thread per interface dof:
//   lambda_e += sigma ((2 p_s - prev_s) - (2 p_t - prev_t)),  prev <- p.
__global__ __launch_bounds__(256) void k_lambda(const ImgDev *imgs, const int *info, const float *p1,
                                                const float *p2, float *lam, float sigma)
{
    const ImgDev im = imgs[blockIdx.y];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= im.nlam) return;
    float ps, pt;
    if (e < im.nlh) {
        const int r = e / im.W + 1, j = e - (r - 1) * im.W;
        const int cut = info[im.rcut + r];
        // side s: bottom copy of subdomain row r-1 at P1 row cut + r - 1; side t: row cut + r
        ps = p1[im.p1 + (long long)(cut + r - 1) * im.pitch1 + j];
        pt = p1[im.p1 + (long long)(cut + r) * im.pitch1 + j];
    } else {
        const int q = e - im.nlh;
        const int c = q / im.H + 1, i = q - (c - 1) * im.H;
        const int cut = info[im.ccut + c];
        ps = p2[im.p2 + (long long)i * im.pitch2 + cut + c - 1];
        pt = p2[im.p2 + (long long)i * im.pitch2 + cut + c];
    }
    float *L = lam + im.lam;
    const float prev_s = L[im.nlam + e], prev_t = L[2 * im.nlam + e];
    L[e] = L[e] + sigma * ((2.0f * ps - prev_s) - (2.0f * pt - prev_t));
    L[im.nlam + e] = ps;
    L[2 * im.nlam + e] = pt;
}

hipError_t launch_lambda(const ImgDev *imgs, int nimg, int max_nlam, const int *info, const float *p1,
                         const float *p2, float *lam, float sigma, hipStream_t s)
{
    if (max_nlam <= 0) return hipSuccess;
    dim3 grid((max_nlam + 255) / 256, nimg);
    hipLaunchKernelGGL(k_lambda, grid, dim3(256), 0, s, imgs, info, p1, p2, lam, sigma);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// (a3) one projected-FISTA step on every local dual problem (ROF), in the
// form of fista_ops.h.  The first step of an outer iteration (MODE first)
// starts from y = x_0 = p~^n and also builds c' from the anchor
// phat = p~^n -/+ tau lambda on the s / t copies of interface edges
// (Algorithm 1: phat = p~ - tau B^* lambda) and from f; later steps read c'.
template <int R, int MODE>
__global__ __launch_bounds__(64) void k_fista_step(FistaStepArgs a)
{
    constexpr bool FIRST = MODE == kFistaFirst, MOM = MODE == kFistaMomentum;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const StreamTile tile = a.tiles[t];
    const ImgDev im = a.imgs[tile.img];
    const int lane = threadIdx.x;
    const int H = im.H, W = im.W;
    const int j = tile.j0 - 1 + lane;
    const bool colok = (j >= 0) && (j < W);
    const int cw = colok ? a.info[im.cinfo + j] : 0;
    const int cs = info_sub(cw);
    const bool cfirst = info_first(cw), clast = info_last(cw);
    const int left = j + cs;
    const bool outlane = colok && lane >= 1;
    const long long P1 = im.pitch1, P2 = im.pitch2;

    // the outputs (new iterate, c' in the first step, pre-projection records) alias none of the
    // inputs, so every load of a row is issued before the row's stores
    const float *__restrict__ xa1 = a.xa1 + im.p1;
    const float *__restrict__ xa2 = a.xa2 + im.p2;
    const float *__restrict__ xb1 = MOM ? a.xb1 + im.p1 : nullptr;
    const float *__restrict__ xb2 = MOM ? a.xb2 + im.p2 : nullptr;
    float *__restrict__ c1 = a.c1 + im.p1;
    float *__restrict__ c2 = a.c2 + im.p2;
    const float *__restrict__ lam = a.lam + im.lam;
    const float *__restrict__ f = a.f + im.px;
    float *__restrict__ o1 = a.out1 + im.p1;
    float *__restrict__ o2 = a.out2 + im.p2;
    const bool rec = a.z1 != nullptr;
    float *__restrict__ zr1 = rec ? a.z1 + im.p1 : nullptr;
    float *__restrict__ zr2 = rec ? a.z2 + im.p2 : nullptr;
    const float beta = a.beta, tau = a.tau, itau = a.inv_tau;
    const float invL = im.invL, ak = im.a_keep, kL = im.kL;

    // y = x + beta (x - x_prev) from the two loaded values
    auto yv = [&](float x, float xp) -> float {
        if constexpr (MOM) return fista_y(x, xp, beta);
        return x;
    };

    const int i0 = tile.i0;
    const int iend = min(i0 + R, H);
    float d_up = 0.0f, y_carry = 0.0f, f_up = 0.0f;
    bool have = false;
    if (i0 > 0 && !info_first(a.info[im.rinfo + i0])) {
        // halo row: divergence of the pixel above the strip, same subdomain
        const int i = i0 - 1;
        const long long top = i + info_sub(a.info[im.rinfo + i]);
        if (colok) {
            const float xt = xa1[top * P1 + j], xb = xa1[(top + 1) * P1 + j];
            const float xl = xa2[i * P2 + left], xr = xa2[i * P2 + left + 1];
            float xtp = 0.0f, xbp = 0.0f, xlp = 0.0f, xrp = 0.0f;
            if constexpr (MOM) {
                xtp = xb1[top * P1 + j];
                xbp = xb1[(top + 1) * P1 + j];
                xlp = xb2[i * P2 + left];
                xrp = xb2[i * P2 + left + 1];
            }
            if constexpr (FIRST) f_up = f[(long long)i * W + j];
            const float yb = yv(xb, xbp);
            d_up = div4(yv(xt, xtp), yb, yv(xl, xlp), yv(xr, xrp));
            y_carry = yb;
        }
        have = true;
    }
    for (int i = i0; i < iend; ++i) {
        const int rw = a.info[im.rinfo + i];
        const int rs = info_sub(rw);
        const bool rfirst = info_first(rw), rlast = info_last(rw);
        const long long top = i + rs;
        if (rfirst) {
            have = false;
            d_up = 0.0f;
            f_up = 0.0f;
        }
        // ---- every load of the row first
        float xt = 0.0f, xtp = 0.0f, xb = 0.0f, xbp = 0.0f, xl = 0.0f, xlp = 0.0f, xr = 0.0f, xrp = 0.0f;
        float fv = 0.0f, ct = 0.0f, cl = 0.0f, cb = 0.0f, cr = 0.0f, lt = 0.0f, ll = 0.0f, lb = 0.0f, lr = 0.0f;
        if (colok) {
            if (!have) {
                xt = xa1[top * P1 + j];
                if constexpr (MOM) xtp = xb1[top * P1 + j];
            }
            xb = xa1[(top + 1) * P1 + j];
            xl = xa2[i * P2 + left];
            xr = xa2[i * P2 + left + 1];
            if constexpr (MOM) {
                xbp = xb1[(top + 1) * P1 + j];
                xlp = xb2[i * P2 + left];
                xrp = xb2[i * P2 + left + 1];
            }
            if constexpr (FIRST) {
                fv = f[(long long)i * W + j];
                if (rfirst && i > 0) lt = lam[(long long)(rs - 1) * W + j];
                if (cfirst && j > 0) ll = lam[im.nlh + (long long)(cs - 1) * H + i];
                if (rlast && i < H - 1) lb = lam[(long long)rs * W + j];
                if (clast && j < W - 1) lr = lam[im.nlh + (long long)cs * H + i];
            } else {
                ct = c1[top * P1 + j];
                cl = c2[i * P2 + left];
                cb = c1[(top + 1) * P1 + j];
                cr = c2[i * P2 + left + 1];
            }
        }
        float d = 0.0f, yt = 0.0f, yb = 0.0f, yl = 0.0f, yr = 0.0f;
        if (colok) {
            yt = have ? y_carry : yv(xt, xtp);
            yb = yv(xb, xbp);
            yl = yv(xl, xlp);
            yr = yv(xr, xrp);
            d = div4(yt, yb, yl, yr);
        }
        float d_left = __shfl_up(d, 1, 64);
        float f_left = 0.0f;
        if constexpr (FIRST) f_left = __shfl_up(fv, 1, 64);
        if (cfirst) {
            d_left = 0.0f;
            f_left = 0.0f;
        }
        if (outlane) {
            if (i > 0) {  // edge above the pixel (interior, or t copy of an interface)
                float c = ct;
                if constexpr (FIRST) {
                    c = fista_cprime(rfirst ? fmaf(tau, lt, yt) : yt, f_up, fv, itau, invL);
                    c1[top * P1 + j] = c;
                }
                const float z = fista_z(yt, d_up, d, c, ak, kL);
                o1[top * P1 + j] = clamp1(z);
                if (rec) zr1[top * P1 + j] = z;
            }
            if (j > 0) {  // edge left of the pixel
                float c = cl;
                if constexpr (FIRST) {
                    c = fista_cprime(cfirst ? fmaf(tau, ll, yl) : yl, f_left, fv, itau, invL);
                    c2[i * P2 + left] = c;
                }
                const float z = fista_z(yl, d_left, d, c, ak, kL);
                o2[i * P2 + left] = clamp1(z);
                if (rec) zr2[i * P2 + left] = z;
            }
            if (rlast && i < H - 1) {  // s copy below the last row of the subdomain
                float c = cb;
                if constexpr (FIRST) {
                    c = fista_cprime(fmaf(-tau, lb, yb), fv, 0.0f, itau, invL);
                    c1[(top + 1) * P1 + j] = c;
                }
                const float z = fista_z(yb, d, 0.0f, c, ak, kL);
                o1[(top + 1) * P1 + j] = clamp1(z);
                if (rec) zr1[(top + 1) * P1 + j] = z;
            }
            if (clast && j < W - 1) {  // s copy right of the last column
                float c = cr;
                if constexpr (FIRST) {
                    c = fista_cprime(fmaf(-tau, lr, yr), fv, 0.0f, itau, invL);
                    c2[i * P2 + left + 1] = c;
                }
                const float z = fista_z(yr, d, 0.0f, c, ak, kL);
                o2[i * P2 + left + 1] = clamp1(z);
                if (rec) zr2[i * P2 + left + 1] = z;
            }
        }
        d_up = d;
        y_carry = yb;
        f_up = fv;
        have = true;
    }
}

// launch with optional start / stop events recorded by the dispatch itself
template <typename... Args>
static void launch_timed(void (*kern)(Args...), dim3 grid, dim3 block, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                         Args... args)
{
    if (e0)
        hipExtLaunchKernelGGL(kern, grid, block, 0, s, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kern, grid, block, 0, s, args...);
}

template <int R>
static hipError_t fista_rows(const FistaStepArgs &a, int mode, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    switch (mode) {
    case kFistaFirst: launch_timed(k_fista_step<R, kFistaFirst>, dim3(a.ntiles), dim3(64), s, e0, e1, a); break;
    case kFistaPlain: launch_timed(k_fista_step<R, kFistaPlain>, dim3(a.ntiles), dim3(64), s, e0, e1, a); break;
    default: launch_timed(k_fista_step<R, kFistaMomentum>, dim3(a.ntiles), dim3(64), s, e0, e1, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_fista_step(const FistaStepArgs &a, int mode, int rows, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (a.ntiles <= 0) return hipSuccess;
    switch (rows) {
    case 4: return fista_rows<4>(a, mode, s, e0, e1);
    case 8: return fista_rows<8>(a, mode, s, e0, e1);
    case 16: return fista_rows<16>(a, mode, s, e0, e1);
    case 32: return fista_rows<32>(a, mode, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// (a3) one step of the accelerated primal-dual method (Chambolle-Pock 2011,
// Alg. 2) on every local saddle problem eq. (local) of Sec. 5:
//   xbar = x_{k-1} + theta_prev (x_{k-1} - x_{k-2})
//   u_k  = prox_{sigma_k alpha F}(u_{k-1} + sigma_k div_s xbar)   (per pixel)
//   x_k  = clamp((tau (x_{k-1} - tau_k div_s^* u_k) + tau_k phat) / (tau + tau_k))
template <int R, bool EXT>
__global__ __launch_bounds__(64) void k_cp2_step(Cp2StepArgs a)
{
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const StreamTile tile = a.tiles[t];
    const ImgDev im = a.imgs[tile.img];
    const int lane = threadIdx.x;
    const int H = im.H, W = im.W;
    const int j = tile.j0 - 1 + lane;
    const bool colok = (j >= 0) && (j < W);
    const int cw = colok ? a.info[im.cinfo + j] : 0;
    const int cs = info_sub(cw);
    const bool cfirst = info_first(cw), clast = info_last(cw);
    const int left = j + cs;
    const bool outlane = colok && lane >= 1;
    const long long P1 = im.pitch1, P2 = im.pitch2;

    // the outputs alias none of the inputs (distinct buffers), so every load of a
    // row can be issued before the previous row's stores complete
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
    float *__restrict__ o1 = a.out1 + im.p1;
    float *__restrict__ o2 = a.out2 + im.p2;
    const float th = a.theta_prev, sk = a.sk, tk = a.tk, tau = a.tau;
    const float ck = a.c_keep, ca = a.c_anchor, sa = a.sk * im.alpha;
    const int fid = a.fidelity;
    const float cv1 = a.cv_c1, cv2 = a.cv_c2;

    // xbar = x + theta (x - x_prev) from the two loaded values
    auto xbar = [&](float x, float xp) -> float {
        if constexpr (EXT) return fmaf(th, x - xp, x);
        return x;
    };
    auto pupdate = [&](float x, float du, float anchor) -> float { return clamp1(cp2_pre(x, du, anchor, tk, ck, ca)); };

    const int i0 = tile.i0;
    const int iend = min(i0 + R, H);
    float u_up = 0.0f, xbar_carry = 0.0f, x_carry = 0.0f;
    bool have = false;
    if (i0 > 0 && !info_first(a.info[im.rinfo + i0])) {  // the row above, in the same subdomain
        const int i = i0 - 1;
        const long long top = i + info_sub(a.info[im.rinfo + i]);
        if (colok) {
            const long long px = (long long)i * W + j;
            const float xt = xa1[top * P1 + j], xb = xa1[(top + 1) * P1 + j];
            const float xl = xa2[i * P2 + left], xr = xa2[i * P2 + left + 1];
            float xtp = 0.0f, xbp = 0.0f, xlp = 0.0f, xrp = 0.0f;
            if constexpr (EXT) {
                xtp = xb1[top * P1 + j];
                xbp = xb1[(top + 1) * P1 + j];
                xlp = xb2[i * P2 + left];
                xrp = xb2[i * P2 + left + 1];
            }
            const float uv = uin[px], fv = f[px];
            const bool obs = mk ? mk[px] != 0 : true;
            const float bt = xbar(xt, xtp), bb = xbar(xb, xbp);
            const float d = (bb - bt) + (xbar(xr, xrp) - xbar(xl, xlp));
            u_up = cp2_u(fid, uv, d, sk, fv, obs, sa, cv1, cv2);
            xbar_carry = bb;
            x_carry = xb;
        }
        have = true;
    }
    // Every load of a row, issued one row ahead (software pipeline): row i + 1's loads are in
    // flight while row i is computed and stored.  The top edge of a row is the bottom edge of the
    // row above, carried in registers, except at the first row of a subdomain.
    struct Row {
        int rw;
        float xt, xtp, xb, xbp, xl, xlp, xr, xrp, uv, fv, at, al, ab, ar, lt, ll, lb, lr;
        unsigned mv;
    };
    auto load_row = [&](int i, Row &r) {
        r.rw = a.info[im.rinfo + i];
        const int rs = info_sub(r.rw);
        const bool rfirst = info_first(r.rw), rlast = info_last(r.rw);
        const long long top = i + rs;
        const long long px = (long long)i * W + j;
        r.xt = r.xtp = r.xb = r.xbp = r.xl = r.xlp = r.xr = r.xrp = 0.0f;
        r.uv = r.fv = r.at = r.al = r.ab = r.ar = 0.0f;
        r.lt = r.ll = r.lb = r.lr = 0.0f;
        r.mv = 1;
        if (colok) {
            if (mk) r.mv = mk[px];  // first: loads complete in order, so its use waits on it alone
            if (rfirst) {
                r.xt = xa1[top * P1 + j];
                if constexpr (EXT) r.xtp = xb1[top * P1 + j];
            }
            r.xb = xa1[(top + 1) * P1 + j];
            r.xl = xa2[i * P2 + left];
            r.xr = xa2[i * P2 + left + 1];
            if constexpr (EXT) {
                r.xbp = xb1[(top + 1) * P1 + j];
                r.xlp = xb2[i * P2 + left];
                r.xrp = xb2[i * P2 + left + 1];
            }
            r.uv = uin[px];
            r.fv = f[px];
            // anchors p~^n of the four edges, and lambda on the interface copies
            r.at = b1[top * P1 + j];
            r.ab = b1[(top + 1) * P1 + j];
            r.al = b2[i * P2 + left];
            r.ar = b2[i * P2 + left + 1];
            if (rfirst && i > 0) r.lt = lam[(long long)(rs - 1) * W + j];
            if (cfirst && j > 0) r.ll = lam[im.nlh + (long long)(cs - 1) * H + i];
            if (rlast && i < H - 1) r.lb = lam[(long long)rs * W + j];
            if (clast && j < W - 1) r.lr = lam[im.nlh + (long long)cs * H + i];
        }
    };
    Row cur, nxt;
    load_row(i0, cur);
    for (int i = i0; i < iend; ++i) {
        if (i + 1 < iend) load_row(i + 1, nxt);
        const int rs = info_sub(cur.rw);
        const bool rfirst = info_first(cur.rw), rlast = info_last(cur.rw);
        const long long top = i + rs;
        const long long px = (long long)i * W + j;
        if (rfirst) {
            have = false;
            u_up = 0.0f;
        }
        // ---- u_k of the pixel from xbar_{k-1} on its four edges
        float u = 0.0f, bxb = 0.0f, xt = cur.xt;
        if (colok) {
            const float bxt = have ? xbar_carry : xbar(cur.xt, cur.xtp);
            if (have) xt = x_carry;
            bxb = xbar(cur.xb, cur.xbp);
            const float d = (bxb - bxt) + (xbar(cur.xr, cur.xrp) - xbar(cur.xl, cur.xlp));
            u = cp2_u(fid, cur.uv, d, sk, cur.fv, cur.mv != 0, sa, cv1, cv2);
        }
        float u_left = __shfl_up(u, 1, 64);
        if (cfirst) u_left = 0.0f;
        // ---- x_k on the pixel's top and left edges, and on its bottom / right edges at the
        // subdomain's last row / column (anchors -/+ tau lambda on the interface copies)
        if (outlane) {
            uout[px] = u;
            if (i > 0) o1[top * P1 + j] = pupdate(xt, u_up - u, rfirst ? fmaf(tau, cur.lt, cur.at) : cur.at);
            if (j > 0) o2[i * P2 + left] = pupdate(cur.xl, u_left - u, cfirst ? fmaf(tau, cur.ll, cur.al) : cur.al);
            if (rlast && i < H - 1) o1[(top + 1) * P1 + j] = pupdate(cur.xb, u, fmaf(-tau, cur.lb, cur.ab));
            if (clast && j < W - 1) o2[i * P2 + left + 1] = pupdate(cur.xr, u, fmaf(-tau, cur.lr, cur.ar));
        }
        u_up = u;
        xbar_carry = bxb;
        x_carry = cur.xb;
        have = true;
        cur = nxt;
    }
}

template <int R>
static hipError_t cp2_rows(const Cp2StepArgs &a, bool ext, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (ext)
        launch_timed(k_cp2_step<R, true>, dim3(a.ntiles), dim3(64), s, e0, e1, a);
    else
        launch_timed(k_cp2_step<R, false>, dim3(a.ntiles), dim3(64), s, e0, e1, a);
    return hipGetLastError();
}

hipError_t launch_cp2_step(const Cp2StepArgs &a, bool extrapolate, int rows, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (a.ntiles <= 0) return hipSuccess;
    switch (rows) {
    case 4: return cp2_rows<4>(a, extrapolate, s, e0, e1);
    case 8: return cp2_rows<8>(a, extrapolate, s, e0, e1);
    case 16: return cp2_rows<16>(a, extrapolate, s, e0, e1);
    case 32: return cp2_rows<32>(a, extrapolate, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// (a4) primal recovery for ROF: u = f + div_s p~ / alpha on every pixel.
__global__ __launch_bounds__(256) void k_u_from_p(const ImgDev *imgs, const int *info, const float *p1,
                                                  const float *p2, const float *f, float *u)
{
    const ImgDev im = imgs[blockIdx.z];
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= im.H || j >= im.W) return;
    const long long top = i + info_sub(info[im.rinfo + i]);
    const long long left = j + info_sub(info[im.cinfo + j]);
    const float *q1 = p1 + im.p1, *q2 = p2 + im.p2;
    const float yt = q1[top * im.pitch1 + j], yb = q1[(top + 1) * im.pitch1 + j];
    const float yl = q2[i * (long long)im.pitch2 + left], yr = q2[i * (long long)im.pitch2 + left + 1];
    const long long px = im.px + (long long)i * im.W + j;
    u[px] = fmaf((yb - yt) + (yr - yl), im.inv_alpha, f[px]);
}

hipError_t launch_u_from_p(const ImgDev *imgs, int nimg, int maxH, int maxW, const int *info, const float *p1,
                           const float *p2, const float *f, float *u, hipStream_t s)
{
    dim3 grid((maxW + 63) / 64, (maxH + 3) / 4, nimg);
    hipLaunchKernelGGL(k_u_from_p, grid, dim3(256), 0, s, imgs, info, p1, p2, f, u);
    return hipGetLastError();
}

// Boundary edges of the image carry no dof: keep them at zero.
// Zero fill of `words` 32-bit words (every buffer the solver clears is a
// multiple of 4 bytes and 4-byte aligned).  A kernel rather than
// hipMemsetAsync, so that a caller may capture the whole solve in a hipGraph
// without memset nodes.
__global__ __launch_bounds__(256) void k_fill_zero(unsigned *p, long long words)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < words; k += stride) p[k] = 0u;
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s)
{
    const long long words = (long long)(bytes / 4);
    if (words == 0) return hipSuccess;
    const long long blocks = std::min<long long>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, (unsigned *)p, words);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero_boundary(const ImgDev *imgs, float *p1, float *p2)
{
    const ImgDev im = imgs[blockIdx.y];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < im.W) {
        p1[im.p1 + k] = 0.0f;
        p1[im.p1 + (long long)(im.H + im.ny - 1) * im.pitch1 + k] = 0.0f;
    }
    if (k < im.H) {
        p2[im.p2 + (long long)k * im.pitch2] = 0.0f;
        p2[im.p2 + (long long)k * im.pitch2 + im.W + im.nx - 1] = 0.0f;
    }
}

hipError_t launch_zero_boundary(const ImgDev *imgs, int nimg, int maxH, int maxW, float *p1, float *p2,
                                hipStream_t s)
{
    const int n = maxH > maxW ? maxH : maxW;
    hipLaunchKernelGGL(k_zero_boundary, dim3((n + 255) / 256, nimg), dim3(256), 0, s, imgs, p1, p2);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// (a5) FP64 diagnostics.  Per pixel, in double precision:
//   fidelity term, TV terms |u(i+1,j) - u(i,j)| + |u(i,j+1) - u(i,j)|,
//   d = div p_avg (interface dofs averaged over their two copies),
//   f d and d^2 (Chan-Vese: min(0, alpha g - d), the pixel's share of the dual
//   value), and |p_s - p_t|^2 for the interface edges below / right of the pixel.  Fixed-order reductions (wave shuffles, then a fixed tree), so
//   results are bitwise reproducible.
constexpr int kDiagRows = 32;  // rows per diagnostics block (4 rows per pass, 8 passes)

int diag_blocks_per_image(int maxH, int maxW) { return ((maxW + 63) / 64) * ((maxH + kDiagRows - 1) / kDiagRows); }

__device__ __forceinline__ double wave_sum(double x)
{
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__global__ __launch_bounds__(256) void k_diag(const ImgDev *imgs, const int *info, const float *p1,
                                              const float *p2, const float *f, const float *u,
                                              const uint8_t *mask, int fidelity, double cv_c1, double cv_c2,
                                              double *partials)
{
    const ImgDev im = imgs[blockIdx.z];
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int H = im.H, W = im.W;
    const float *q1 = p1 + im.p1, *q2 = p2 + im.p2;
    const long long P1 = im.pitch1, P2 = im.pitch2;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int pass = 0; pass < kDiagRows / 4; ++pass) {
        const int i = blockIdx.y * kDiagRows + pass * 4 + (threadIdx.x >> 6);
        if (i >= H || j >= W) continue;
        const int rw = info[im.rinfo + i], cw = info[im.cinfo + j];
        const long long top = i + info_sub(rw), left = j + info_sub(cw);
        const long long px = im.px + (long long)i * W + j;
        const double uv = u[px], fv = f[px];
        const bool obs = mask ? mask[px] != 0 : true;
        const double g = (fv - cv_c1) * (fv - cv_c1) - (fv - cv_c2) * (fv - cv_c2);
        if (fidelity == 2) {
            acc[0] += uv * g;
        } else if (obs) {
            const double d = uv - fv;
            acc[0] += fidelity == 0 ? 0.5 * d * d : fabs(d);
        }
        if (i + 1 < H) acc[1] += fabs((double)u[px + W] - uv);
        if (j + 1 < W) acc[1] += fabs((double)u[px + 1] - uv);
        // conforming average on the four edges of the pixel
        double et = q1[top * P1 + j], eb = q1[(top + 1) * P1 + j];
        double el = q2[i * P2 + left], er = q2[i * P2 + left + 1];
        if (info_first(rw) && i > 0) et = 0.5 * (et + (double)q1[(top - 1) * P1 + j]);
        if (info_last(rw) && i < H - 1) {
            const double t = q1[(top + 2) * P1 + j];
            acc[4] += (eb - t) * (eb - t);
            eb = 0.5 * (eb + t);
        }
        if (info_first(cw) && j > 0) el = 0.5 * (el + (double)q2[i * P2 + left - 1]);
        if (info_last(cw) && j < W - 1) {
            const double t = q2[i * P2 + left + 2];
            acc[4] += (er - t) * (er - t);
            er = 0.5 * (er + t);
        }
        const double d = (eb - et) + (er - el);
        acc[2] += fidelity == 2 ? fmin(0.0, (double)im.alpha * g - d) : fv * d;
        acc[3] += d * d;
        if (!isfinite(uv) || !isfinite(et) || !isfinite(el) || !isfinite(eb) || !isfinite(er)) acc[5] += 1.0;
    }
    __shared__ double red[4][6];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int q = 0; q < 6; ++q) {
        const double s = wave_sum(acc[q]);
        if (lane == 0) red[wave][q] = s;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int q = threadIdx.x;
        const double s = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
        const long long blk = (long long)blockIdx.z * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x;
        partials[blk * 6 + q] = s;
    }
}

__global__ __launch_bounds__(256) void k_diag_final(const double *partials, int nblk, double *out)
{
    const int img = blockIdx.x;
    const double *P = partials + (long long)img * nblk * 6;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += 256)
        for (int q = 0; q < 6; ++q) acc[q] += P[(long long)b * 6 + q];
    __shared__ double red[4][6];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int q = 0; q < 6; ++q) {
        const double s = wave_sum(acc[q]);
        if (lane == 0) red[wave][q] = s;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int q = threadIdx.x;
        out[img * 6 + q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
    }
}

hipError_t launch_diag(const ImgDev *imgs, int nimg, int maxH, int maxW, const int *info, const float *p1,
                       const float *p2, const float *f, const float *u, const uint8_t *mask, int fidelity,
                       double cv_c1, double cv_c2, double *partials, int nblk_per_img, double *out, hipStream_t s)
{
    dim3 grid((maxW + 63) / 64, (maxH + kDiagRows - 1) / kDiagRows, nimg);
    hipLaunchKernelGGL(k_diag, grid, dim3(256), 0, s, imgs, info, p1, p2, f, u, mask, fidelity, cv_c1, cv_c2,
                       partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_final, dim3(nimg), dim3(256), 0, s, partials, nblk_per_img, out);
    return hipGetLastError();
}

}  // namespace dtv
