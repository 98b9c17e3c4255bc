// Two consecutive local steps k and k + 1 of the accelerated primal-dual solver
// (Chambolle-Pock Alg. 2 on the local saddle problems eq. (local) of Sec. 5,
// Lee & Park, arXiv 1901.00682) in one streaming launch over every subdomain.
//
// The one-step kernel (kernels.hip) reads x_{k-1}, x_{k-2}, the anchor, u, f
// and the mask and writes x_k and u_k at every step.  Here step k's results
// stay in registers for step k + 1: per launch the kernel reads that input
// once and writes x_k, x_{k+1} and u_{k+1}, about 61 bytes per pixel for two
// steps against 90 for two one-step launches.
//
// Work decomposition as in the one-step kernel: a 64-lane wave owns a strip
// of R rows and 64 consecutive columns.  Step k + 1 at a pixel needs x_k on
// the pixel's right edge (the left edge of the next lane's pixel) and x_k of
// a lane needs u_k of the lane to its left, so lanes 0 and 1 are halo
// columns and lane 63 computes only what lane 62 reads: each wave writes the
// 61 columns of lanes 2..62.  Rows are swept top to bottom; step k + 1 runs
// one row behind step k, which supplies x_k on the row's bottom edge (the
// next row's top edge).  Step k starts two rows above the strip (u_k there
// is needed for x_k and u_(k+1) of the row above the strip) and ends one row
// below it; those halo rows are computed and not stored.  Subdomain
// boundaries inside a strip reset the carried values exactly as in the
// one-step kernel.
//
// The per-element arithmetic is that of the one-step kernel (cp2_ops.h), in
// the same order, so a pair launch equals two one-step launches bitwise.
#include "cp2_ops.h"
#include "cp2_pair.h"
#include "fista_ops.h"

namespace dtv {

namespace {

// everything one row of the strip loads (the one-step kernel's row)
struct PairRow {
    int rw;                                   // row info word
    float xt, xtp, xb, xbp, xl, xlp, xr, xrp;  // x_{k-1}, x_{k-2} on the top, bottom, left, right edges
    float uv, fv;                             // u_{k-1}, f
    float at, al, ab, ar;                     // anchors p~^n of the four edges
    float lt, ll, lb, lr;                     // lambda on the interface copies among them
    unsigned mv;                              // observed (mask byte)
};

// what step k leaves of a row for step k + 1
struct PairMid {
    int rw;                            // row info word, with bit 31 set when the pixel is observed
    float u;                           // u_k
    float kt, kl, kb, kr;              // x_k on the top, left, bottom (last row), right (last column) edges
    float mt, ml, mb, mr;              // x_{k-1} on the same edges (mb, mr: the bottom and right edges)
    float fv;
    float at, al, ab, ar;              // the anchors phat of the four edges (-/+ tau lambda on interface copies)
};

}  // namespace

// EXT: step k extrapolates xbar_{k-1} = x_{k-1} + theta_{k-1} (x_{k-1} - x_{k-2}) (k >= 2); step
// k + 1 always extrapolates xbar_k = x_k + theta_k (x_k - x_{k-1}).  The kernel is bound by memory
// latency, so it asks for five waves per SIMD (at most 96 VGPRs; the one value that then spills is
// stored before the row loop and reloaded after it).
template <int R, bool EXT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) void k_cp2_pair(Cp2PairArgs a)
{
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const StreamTile tile = a.tiles[t];
    const ImgDev im = a.imgs[tile.img];
    const int lane = threadIdx.x;
    const int H = im.H, W = im.W;
    const int j = tile.j0 - 2 + lane;
    const bool colok = (j >= 0) && (j < W);
    const int cw = colok ? a.info[im.cinfo + j] : 0;
    const int cs = info_sub(cw);
    const bool cfirst = info_first(cw), clast = info_last(cw);
    const int left = j + cs;
    const bool outlane = colok && lane >= 2 && lane <= 62;
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
    const float tha = a.theta_a, ska = a.sk_a, tka = a.tk_a, cka = a.ck_a, caa = a.ca_a, saa = a.sk_a * im.alpha;
    const float thb = a.theta_b, skb = a.sk_b, tkb = a.tk_b, ckb = a.ck_b, cab = a.ca_b, sab = a.sk_b * im.alpha;
    const int fid = a.fidelity;
    const float cv1 = a.cv_c1, cv2 = a.cv_c2;

    auto xbarA = [&](float x, float xp) -> float {
        if constexpr (EXT) return fmaf(tha, x - xp, x);
        return x;
    };
    auto xbarB = [&](float x, float xp) -> float { return fmaf(thb, x - xp, x); };
    auto pupA = [&](float x, float du, float anchor) -> float { return clamp1(cp2_pre(x, du, anchor, tka, cka, caa)); };
    auto pupB = [&](float x, float du, float anchor) -> float { return clamp1(cp2_pre(x, du, anchor, tkb, ckb, cab)); };

    const int i0 = tile.i0;
    const int iend = min(i0 + R, H);
    const int ra = max(i0 - 2, 0);  // first row of step k
    const int rb = min(iend, H - 1);  // last row of step k
    const int qa = max(i0 - 1, 0);  // first row of step k + 1

    auto load_row = [&](int i, PairRow &r, bool top) {
        r.rw = a.info[im.rinfo + i];
        const int rs = info_sub(r.rw);
        const bool rfirst = info_first(r.rw), rlast = info_last(r.rw);
        const long long tp = i + rs;
        const long long px = (long long)i * W + j;
        r.xt = r.xtp = r.xb = r.xbp = r.xl = r.xlp = r.xr = r.xrp = 0.0f;
        r.uv = r.fv = r.at = r.al = r.ab = r.ar = 0.0f;
        r.lt = r.ll = r.lb = r.lr = 0.0f;
        r.mv = 1;
        if (colok) {
            if (mk) r.mv = mk[px];
            if (rfirst || top) {
                r.xt = xa1[tp * P1 + j];
                if constexpr (EXT) r.xtp = xb1[tp * P1 + j];
            }
            r.xb = xa1[(tp + 1) * P1 + j];
            r.xl = xa2[i * P2 + left];
            r.xr = xa2[i * P2 + left + 1];
            if constexpr (EXT) {
                r.xbp = xb1[(tp + 1) * P1 + j];
                r.xlp = xb2[i * P2 + left];
                r.xrp = xb2[i * P2 + left + 1];
            }
            r.uv = uin[px];
            r.fv = f[px];
            r.at = b1[tp * P1 + j];
            r.ab = b1[(tp + 1) * P1 + j];
            r.al = b2[i * P2 + left];
            r.ar = b2[i * P2 + left + 1];
            if (rfirst && i > 0) r.lt = lam[(long long)(rs - 1) * W + j];
            if (cfirst && j > 0) r.ll = lam[im.nlh + (long long)(cs - 1) * H + i];
            if (rlast && i < H - 1) r.lb = lam[(long long)rs * W + j];
            if (clast && j < W - 1) r.lr = lam[im.nlh + (long long)cs * H + i];
        }
    };

    // step k + 1 on row q from step k's values of the row (m) and x_k, x_{k-1} on the row's
    // bottom edge (kbot, mbot: the next row's top edge, or the row's own bottom edge at the last
    // row of a subdomain); stores u_{k+1}, x_k and x_{k+1} of rows inside the strip
    float u_upB = 0.0f;
    auto step_b = [&](int q, const PairMid &m, float kbot, float mbot) {
        const int rw = m.rw & 0x7FFFFFFF;
        const bool rfirst = info_first(rw), rlast = info_last(rw);
        const long long tp = q + info_sub(rw);
        const long long px = (long long)q * W + j;
        if (rfirst) u_upB = 0.0f;
        // x_k on the right edge: the next lane's left edge, or the column's own at a subdomain's last column
        const float kr_next = __shfl_down(m.kl, 1, 64);
        float u1 = 0.0f;
        if (colok) {
            const float krr = clast ? m.kr : kr_next;
            const float bxt = xbarB(m.kt, m.mt);
            const float bxb = xbarB(kbot, mbot);
            const float d = (bxb - bxt) + (xbarB(krr, m.mr) - xbarB(m.kl, m.ml));
            u1 = cp2_u(fid, m.u, d, skb, m.fv, m.rw < 0, sab, cv1, cv2);
        }
        float u_left = __shfl_up(u1, 1, 64);
        if (cfirst) u_left = 0.0f;
        if (outlane && q >= i0 && q < iend) {
            uout[px] = u1;
            if (q > 0) {
                ka1[tp * P1 + j] = m.kt;
                kb1[tp * P1 + j] = pupB(m.kt, u_upB - u1, m.at);
            }
            if (j > 0) {
                ka2[q * P2 + left] = m.kl;
                kb2[q * P2 + left] = pupB(m.kl, u_left - u1, m.al);
            }
            if (rlast && q < H - 1) {
                ka1[(tp + 1) * P1 + j] = m.kb;
                kb1[(tp + 1) * P1 + j] = pupB(m.kb, u1, m.ab);
            }
            if (clast && j < W - 1) {
                ka2[q * P2 + left + 1] = m.kr;
                kb2[q * P2 + left + 1] = pupB(m.kr, u1, m.ar);
            }
        }
        u_upB = u1;
    };

    float u_upA = 0.0f, xbar_carry = 0.0f, x_carry = 0.0f;
    bool have = false;
    PairMid prev{};
    bool have_prev = false;
    PairRow cur, nxt;
    load_row(ra, cur, true);
    for (int i = ra; i <= rb; ++i) {
        if (i + 1 <= rb) load_row(i + 1, nxt, false);
        const bool rfirst = info_first(cur.rw), rlast = info_last(cur.rw);
        if (rfirst) {
            have = false;
            u_upA = 0.0f;
        }
        // ---- step k: u_k of the pixel from xbar_{k-1} on its four edges
        float u = 0.0f, bxb = 0.0f, xt = cur.xt;
        if (colok) {
            const float bxt = have ? xbar_carry : xbarA(cur.xt, cur.xtp);
            if (have) xt = x_carry;
            bxb = xbarA(cur.xb, cur.xbp);
            const float d = (bxb - bxt) + (xbarA(cur.xr, cur.xrp) - xbarA(cur.xl, cur.xlp));
            u = cp2_u(fid, cur.uv, d, ska, cur.fv, cur.mv != 0, saa, cv1, cv2);
        }
        float u_left = __shfl_up(u, 1, 64);
        if (cfirst) u_left = 0.0f;
        // x_k on the row's edges (0 on the image boundary, where the buffers hold 0)
        PairMid m;
        m.rw = cur.rw | (cur.mv != 0 ? (int)0x80000000u : 0);
        m.u = u;
        // the anchors of both steps: t copies + tau lambda, s copies - tau lambda
        m.at = rfirst ? fmaf(tau, cur.lt, cur.at) : cur.at;
        m.al = cfirst ? fmaf(tau, cur.ll, cur.al) : cur.al;
        m.ab = fmaf(-tau, cur.lb, cur.ab);
        m.ar = fmaf(-tau, cur.lr, cur.ar);
        m.kt = i > 0 ? pupA(xt, u_upA - u, m.at) : 0.0f;
        m.kl = j > 0 ? pupA(cur.xl, u_left - u, m.al) : 0.0f;
        m.kb = (rlast && i < H - 1) ? pupA(cur.xb, u, m.ab) : 0.0f;
        m.kr = (clast && j < W - 1) ? pupA(cur.xr, u, m.ar) : 0.0f;
        m.mt = xt;
        m.ml = cur.xl;
        m.mb = cur.xb;
        m.mr = cur.xr;
        m.fv = cur.fv;
        // ---- step k + 1 on the row above, now that x_k on its bottom edge is known
        if (have_prev) {
            const bool plast = info_last(prev.rw);
            step_b(i - 1, prev, plast ? prev.kb : m.kt, prev.mb);
        }
        prev = m;
        have_prev = i >= qa;
        u_upA = u;
        xbar_carry = bxb;
        x_carry = cur.xb;
        have = true;
        cur = nxt;
    }
    // the strip reaches the image's last row, which is the last row of its subdomain
    if (have_prev && rb == iend - 1) step_b(rb, prev, prev.kb, prev.mb);
}

namespace {

template <int R>
hipError_t pair_rows(const Cp2PairArgs &a, bool ext, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    auto k = ext ? k_cp2_pair<R, true> : k_cp2_pair<R, false>;
    if (e0 || e1)
        hipExtLaunchKernelGGL(k, dim3(a.ntiles), dim3(64), 0, s, e0, e1, 0, a);
    else
        hipLaunchKernelGGL(k, dim3(a.ntiles), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cp2_pair(const Cp2PairArgs &a, bool extrapolate, int rows, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (a.ntiles <= 0) return hipSuccess;
    switch (rows) {
    case 4: return pair_rows<4>(a, extrapolate, s, e0, e1);
    case 8: return pair_rows<8>(a, extrapolate, s, e0, e1);
    case 16: return pair_rows<16>(a, extrapolate, s, e0, e1);
    case 32: return pair_rows<32>(a, extrapolate, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace dtv
