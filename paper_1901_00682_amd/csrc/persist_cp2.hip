// Persistent schedule of Algorithm 1 (Lee & Park, arXiv 1901.00682) with the
// local accelerated primal-dual solver of Sec. 5 (any fidelity of Sec. 3):
// one cooperative launch runs every outer step.
//
// Each workgroup owns one full 128 x 128 subdomain for the whole solve; x, u
// and f stay in VGPRs (the layout of cp2_tile.h) from the first outer step to
// the last.  Per outer step n:
//   (1) each tile forms q = 2 p^n - p^(n-1) on its own interface copies and
//       publishes them (exchange.h);
//   (2) meanwhile it writes the anchors phat = p^n of every edge but the
//       interface copies to LDS;
//   (3) it waits for its neighbours' copies on the same edges, and both tiles
//       of an interface edge compute lambda^(n+1) = lambda^n + sigma (q_s - q_t)
//       with the operations of the multiplier-update kernel;
//   (4) the anchors of the interface copies, p^n -/+ tau lambda^(n+1);
//   (5) the n_inner primal-dual steps (cp2tile::solve).
// lambda^n and the tile's own previous copies live in LDS.
//
// The arithmetic per edge, pixel and multiplier is that of the streaming and
// fused schedules, so all three give bitwise identical results.
#include "cp2_tile.h"
#include "exchange.h"

namespace dtv {

using namespace fused;
using namespace cp2tile;
using namespace xchg;

namespace {

struct PersistCp2Lds {
    Cp2Lds t;
    float lam[kSides][kFusedMax];    // lambda on the tile's interface edges
    float prv[kSides][kFusedMax];    // the tile's own copies on those edges at the previous outer step
    float stage[kSides][kFusedMax];  // the current copies on the top, bottom and left sides
    int ok;                          // every wait of the current step completed
};

}  // namespace

// FID: the fidelity (0 L2, 1 L1, 2 convex Chan-Vese); MASK: an inpainting mask is given
// FR: some subdomains are framed tiles (smaller than 128 x 128, their short sides on the image
// boundary, run in a 128 x 128 frame as in the fused kernel); every tile then takes that path.
// ADAPT: every local solve stops by the relative-change rule (cp2_tile.h); the steps taken are
// counted per subdomain.
template <int FID, bool MASK, bool FR = false, bool ADAPT = false>
__global__ __launch_bounds__(1024) void k_persist_cp2(PersistCp2Args pa)
{
    __shared__ PersistCp2Lds L;
    Cp2Lds &S = L.t;
    const FusedCp2Args &a = pa.ca;
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
    float *p1_tile = a.p1 + im.p1 + row1 * P1 + tl.ca;
    float *p2_tile = a.p2 + im.p2 + (long long)tl.ra * P2 + col2;
    const long long px0 = im.px + (long long)tl.ra * W + tl.ca;
    const float *f_tile = a.f + px0;
    float *u_tile = a.u + px0;
    const float tau = a.tau;
    const long long nlam = im.nlam;

    Cp2Ctx cx;
    cx.s = s;
    cx.lane = lane;
    cx.ja = ja;
    cx.jb = jb;
    cx.il0 = il0;
    cx.last = last;
    cx.bot_bnd = bot_bnd;
    cx.right_bnd = right_bnd;
    cx.lo1 = (top_bnd && s == 0) ? 0.0f : -1.0f;
    cx.hi1 = -cx.lo1;
    cx.lo2a = (left_bnd && lane == 0) ? 0.0f : -1.0f;
    cx.hi2a = -cx.lo2a;
    cx.alpha = im.alpha;
    cx.cv1 = a.cv_c1;
    cx.cv2 = a.cv_c2;
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
    int steps_total = 0, steps_max = 0;  // adaptive stopping: local steps of this subdomain

    // side work (multiplier update): waves 0..7, side = wave / 2 (wave-uniform), edge
    // si = 64 (wave % 2) + lane; the lambda index is side_base + si
    const int side = s >> 1;
    const bool side_wave = s < 2 * kSides && side_exists(im, tl, side) &&
                           (!FR || (s & 1) * 64 + lane < (side < 2 ? w : h));  // (a framed tile's sides are shorter)
    const bool side_s = side == 1 || side == 3;  // s copies: bottom and right sides
    const long long side_base = side_wave ? side_edge(im, tl, side, 0) : 0;

    // ---- load p~^0, u, f and the lambda state
    Slot X;
    float ua[kR], ub[kR], fa[kR], fb[kR];
    unsigned obs = 0xFFFFu;  // observed pixels: bit 2r (column a), 2r + 1 (column b) of row r
    // (a framed tile: its own h x w pixels and edges; the rest of the frame starts at 0, the zeros
    // written in every lane before the loads)
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int il = il0 + r;
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
    if (lane < kR)
        S.rx[il0 + lane] = (!FR || (w == kFusedMax && il0 + lane < h))
                               ? p2_tile[(long long)(il0 + lane) * P2 + kFusedMax] : 0.0f;
    if constexpr (MASK) {
        const uint8_t *m_tile = a.mask + px0;
        obs = 0;  // (a framed tile: the pixels outside it are unobserved)
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            if (FR && il0 + r >= h) continue;
            const uint8_t *mr = m_tile + (long long)(il0 + r) * W + ja;
            if (!FR || ja < w) obs |= (mr[0] != 0 ? 1u : 0u) << (2 * r);
            if (!FR || ja + 1 < w) obs |= (mr[1] != 0 ? 1u : 0u) << (2 * r + 1);
        }
    }
    if constexpr (FR) {
        // anchors that the loop below never writes on a framed tile: the frame's first row and
        // column and its bottom row and right column outside the tile (the loop skips the rows
        // and columns that hold interface copies; (4) writes the tile's own entries); ordered
        // before the loop's reads by its barriers
        if (s == 0) lds_st2(&S.a1[0][ja], 0.0f, 0.0f);
        if (last) lds_st2(&S.ab[ja], 0.0f, 0.0f);
        if (lane == 0)
#pragma unroll
            for (int r = 0; r < kR; ++r) S.a2[il0 + r][0] = 0.0f;
        if (lane < kR) S.ar[il0 + lane] = 0.0f;
    }
    if (side_wave) {
        const int si = (s & 1) * 64 + lane;
        const float *ls = a.lam + im.lam + side_base;
        L.lam[side][si] = ls[si];
        L.prv[side][si] = ls[(side_s ? nlam : 2 * nlam) + si];
    }
    bool ok = true;

    for (int n = 0; n < pa.n_outer; ++n) {
        // ---- (1) stage the current iterate on the top, bottom and left sides (the right
        // boundary column is in S.rx).  The staging rows are read only by the publication below,
        // and the previous solve's barriers separate that read from these stores.
        if (s == 0) lds_st2(&L.stage[0][ja], X.e1a[0], X.e1b[0]);
        if (last) lds_st2(&L.stage[1][ja], X.ba, X.bb);
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < kR; ++r) L.stage[2][il0 + r] = X.e2a[r];
        }
        if (threadIdx.x == 0) L.ok = 1;
        __syncthreads();
        // ---- publish q = 2 p^n - p^(n-1) on the tile's interface copies
        const int si = (s & 1) * 64 + opaque(lane);
        unsigned long long *xch = pa.xch + (long long)(n & 1) * pa.xch_stride + im.lam + side_base + si;
        float x_side = 0.0f, q_own = 0.0f;
        if (side_wave) {
            x_side = side == 3 ? S.rx[si] : L.stage[side][si];
            q_own = 2.0f * x_side - L.prv[side][si];
            L.prv[side][si] = x_side;
            publish(xch + (side_s ? 0 : nlam), q_own, n);
        }

        // ---- (2) anchors phat = p^n while the neighbours' copies travel, on every edge but the
        // interface copies, which (4) writes with their multiplier term; the two phases write
        // disjoint entries, so no barrier separates them
        {
            const bool top_if = side_exists(im, tl, 0), bot_if = side_exists(im, tl, 1);
            const bool left_if = side_exists(im, tl, 2), right_if = side_exists(im, tl, 3);
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const int il = il0 + r;
                if (!(il == 0 && top_if)) lds_st2(&S.a1[il][ja], X.e1a[r], X.e1b[r]);
                if (ja == 0 && left_if) S.a2[il][1] = X.e2b[r];
                else lds_st2(&S.a2[il][ja], X.e2a[r], X.e2b[r]);
            }
            if (last && !bot_if) lds_st2(&S.ab[ja], X.ba, X.bb);
            if (lane < kR && !right_if) S.ar[il0 + lane] = S.rx[il0 + lane];
        }

        // ---- (3) the neighbour's copy of each interface edge, lambda^(n+1), and (4) the anchor of
        // the tile's copy: phat = p^n + tau lambda on t copies (top, left), - tau lambda on s copies
        if (side_wave) {
            float q_oth = 0.0f;
            if (fetch(xch + (side_s ? nlam : 0), n, q_oth, pa.spin_limit)) {
                const float qs = side_s ? q_own : q_oth, qt = side_s ? q_oth : q_own;
                const float lam = L.lam[side][si] + pa.sigma * (qs - qt);
                L.lam[side][si] = lam;
                if (side == 0) S.a1[0][si] = fmaf(tau, lam, x_side);
                else if (side == 2) S.a2[si][0] = fmaf(tau, lam, x_side);
                else if (side == 1) S.ab[si] = fmaf(-tau, lam, x_side);
                else S.ar[si] = fmaf(-tau, lam, x_side);
            } else {
                L.ok = 0;
                atomicOr(pa.err, 1);
            }
        }
        __syncthreads();
        ok = L.ok != 0;
        if (!ok) break;  // a neighbour stopped publishing: leave (the host reports the error)

        // ---- (5) the local primal-dual solve
        const int taken = solve<FID, FR, ADAPT>(cx, S, X, ua, ub, fa, fb, obs, a);
        if constexpr (ADAPT) {
            steps_total += taken;
            steps_max = max(steps_max, taken);
        }
    }

    // ---- store p~^N, u and the lambda state (lambda^N and the copies of the last multiplier update)
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int il = il0 + r;
        if (!FR || (il < h && ja + 1 < w)) {
            st2g(p1_tile + (long long)il * P1 + ja, X.e1a[r], X.e1b[r]);
            st2g(p2_tile + (long long)il * P2 + ja, X.e2a[r], X.e2b[r]);
            st2g(u_tile + (long long)il * W + ja, ua[r], ub[r]);
        } else if (il < h && ja < w) {  // framed: the tile's last column alone
            p1_tile[(long long)il * P1 + ja] = X.e1a[r];
            p2_tile[(long long)il * P2 + ja] = X.e2a[r];
            u_tile[(long long)il * W + ja] = ua[r];
        }
    }
    // the frame's bottom row and right column: a framed tile's own only when it spans the frame
    if (last && (!FR || (h == kFusedMax && ja + 1 < w))) st2g(p1_tile + (long long)kFusedMax * P1 + ja, X.ba, X.bb);
    else if (FR && last && h == kFusedMax && ja < w) p1_tile[(long long)kFusedMax * P1 + ja] = X.ba;
    if (lane < kR && (!FR || (w == kFusedMax && il0 + lane < h)))
        p2_tile[(long long)(il0 + lane) * P2 + kFusedMax] = S.rx[il0 + lane];
    if constexpr (ADAPT) {
        if (threadIdx.x == 0) {  // the subdomain's only workgroup (one launch holds every subdomain)
            int *cnt = a.counts + 2 * (long long)t;
            cnt[0] += steps_total;
            cnt[1] = max(cnt[1], steps_max);
        }
    }
    if (side_wave && ok) {
        const int si = (s & 1) * 64 + lane;
        float *ls = pa.lam_out + im.lam + side_base;
        if (side_s) {
            ls[si] = L.lam[side][si];
            ls[nlam + si] = L.prv[side][si];
        } else {
            ls[2 * nlam + si] = L.prv[side][si];
        }
    }
}

namespace {

using PersistCp2Kernel = void (*)(PersistCp2Args);

template <bool FR, bool AD>
PersistCp2Kernel persist_cp2_variant(int fidelity, bool mask)
{
    switch (fidelity) {
    case 0: return mask ? k_persist_cp2<0, true, FR, AD> : k_persist_cp2<0, false, FR, AD>;
    case 1: return mask ? k_persist_cp2<1, true, FR, AD> : k_persist_cp2<1, false, FR, AD>;
    case 2: return mask ? nullptr : k_persist_cp2<2, false, FR, AD>;
    default: return nullptr;
    }
}

PersistCp2Kernel persist_cp2_kernel(int fidelity, bool mask, bool frames, bool adapt)
{
    if (adapt)
        return frames ? persist_cp2_variant<true, true>(fidelity, mask) : persist_cp2_variant<false, true>(fidelity, mask);
    return frames ? persist_cp2_variant<true, false>(fidelity, mask) : persist_cp2_variant<false, false>(fidelity, mask);
}

}  // namespace

int persist_cp2_capacity(int device)
{
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist_cp2<1, true>, 1024, 0) != hipSuccess)
        return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    return per_cu * cus;
}

hipError_t launch_persist_cp2(const PersistCp2Args &a, int nsub, hipStream_t s)
{
    if (nsub <= 0 || a.n_outer <= 0) return hipSuccess;
    const bool adapt = a.ca.tol2 > 0.0;
    if (a.ca.n_inner < 1 || a.ca.n_inner > (adapt ? kMaxAdaptiveInner : kMaxFusedInner)) return hipErrorInvalidValue;
    if (adapt && (!a.ca.tab || !a.ca.counts)) return hipErrorInvalidValue;
    const PersistCp2Kernel k = persist_cp2_kernel(a.ca.fidelity, a.ca.mask != nullptr, a.ca.frames != 0, adapt);
    if (!k) return hipErrorInvalidValue;
    PersistCp2Args arg = a;
    void *args[] = {&arg};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k), dim3(nsub), dim3(1024), args, 0, s);
}

}  // namespace dtv
