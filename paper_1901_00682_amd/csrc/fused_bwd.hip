// Reverse mode of one outer step of Algorithm 1 (Lee & Park, arXiv 1901.00682,
// Sec. 4) with FISTA local steps, on full 128 x 128 subdomains: one 1024-thread
// workgroup per subdomain runs the n_inner reverse steps on chip.
//
// The forward step is x_k = P(z_k), z_k = a y_k + c' - kL div_s^*(div_s y_k)
// (fista_ops.h).  Its reverse, from xbar_k:
//   zbar = xbar_k * 1{-1 < z_k < 1}                 (mask recorded by the forward)
//   ybar = a zbar - kL div_s^*(div_s zbar)            (the linear part is self-adjoint)
//   xbar_{k-1} += (1 + beta_k) ybar,  xbar_{k-2} += -beta_k ybar   (steps k >= 3; else xbar_{k-1} += ybar)
// c' = (phat / tau - (f_b - f_a)) / L sends zbar / (L tau) to phat and
// -div_s zbar / L to f; summed over the steps these need only S = sum_k zbar_k,
// kept per edge in LDS.  The alpha derivative of z_k,
//   dA ((phat - y_k) / tau - (f_b - f_a)) - dB div_s^*(div_s y_k),
// with dA = 8 / (alpha L)^2 and dB = -1 / (tau (alpha L)^2), is collected as
//   sum_k <zbar_k, q_k> + dA/tau <phat, S> - dA <f, div S>,
// q_k = -dA/tau y_k - dB div_s^*(div_s y_k) per edge from the forward's record.
//
// The layout on chip is the forward's: wave s holds rows 8 s .. 8 s + 7, lane
// l columns 2 l and 2 l + 1, the two adjoint slots in VGPRs, the right
// boundary column in LDS, one exchange row per strip for zbar and one for
// div zbar; each step has two workgroup barriers.
#include "bwd.h"
#include "exchange.h"
#include "fused_common.h"

namespace dtv {

using namespace fused;

namespace {

struct BwdLds {
    float Sb[kFusedMax];             // S on the bottom boundary edges
    float Sr[kFusedMax];             // S on the right boundary edges
    float rx[2][kFusedMax];          // right boundary edges: the two adjoint slots
    float zt[2][kWaves][kFusedMax];  // zbar on each strip's first-row top edges, by step parity
    float dl[kWaves][kFusedMax];     // div zbar of each strip's last row
    float dR[kFusedMax];             // div zbar of the last column, per row
    double red[kWaves];              // per-wave partial sums of the alpha derivative
    float S1[kFusedMax][kFusedMax];  // S on the edge above pixel (il, jl)
    float S2[kFusedMax][kFusedMax];  // S on the edge left of pixel (il, jl)
};

struct BwdCtx {
    int s, lane, ja, il0;
    bool last;                 // strip 15: owns the tile's bottom boundary edges
    bool top_var, left_var;    // the strip's first-row top edges / lane's column-0 left edge are variables
    bool bot_var, right_var;   // the tile's bottom / right boundary edges are variables
    float ak, kL;
};

__device__ __forceinline__ void ld2(const float *p, float &x, float &y)
{
    float2 v;
    __builtin_memcpy(&v, p, 8);
    x = v.x;
    y = v.y;
}

__device__ __forceinline__ void st2(float *p, float x, float y)
{
    const float2 v = make_float2(x, y);
    __builtin_memcpy(p, &v, 8);
}

__device__ __forceinline__ double wave_sum_d(double x)
{
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// group g of this thread in a step record: rec is the subdomain's record of
// the step (uniform), tid the thread; the group base stays in scalar registers
__device__ __forceinline__ float4 rg(const float4 *rec, int g, int tid) { return (rec + g * kRecThreads)[tid]; }

// One reverse step.  On entry Z holds xbar_k (complete) and P xbar_{k-1}
// (partial); on exit P holds xbar_{k-1} (complete) and Z xbar_{k-2} (partial).
// sx: LDS slot of the right boundary column of Z.  rec: the subdomain's record
// of the step.
template <bool mom, int QD = 4>
__device__ __forceinline__ void bwd_step(const BwdCtx &c, BwdLds &L, Slot &Z, Slot &P, int sx, float beta,
                                         const float4 *rec, double &acc_q)
{
    float *RZ = L.rx[sx];
    float *RP = L.rx[sx ^ 1];
    const float ak = c.ak, kL = c.kL;
    // per step, so that addresses are formed here and not hoisted out of the step sequence
    const int tid = opaque(c.s * 64 + c.lane), oc = opaque(c.il0 * kFusedMax + c.ja);
    const int row = c.il0 + c.lane;  // lanes 0..7: right boundary edge of this row
    float *S1 = &L.S1[0][0] + oc, *S2 = &L.S2[0][0] + oc;
    // (1) zbar on every owned edge, S += zbar, <zbar, q>.  The step's record is
    // loaded in two halves: group 8 (boundary edges and mask) and rows 0..3 first,
    // rows 4..7 once rows 0..1 are consumed, so that at most five groups are held
    // at once (all nine at once take more registers than the slots leave).
    float4 q[QD];
    const float4 g8 = rg(rec, 8, tid);
#pragma unroll
    for (int g = 0; g < QD; ++g) q[g] = rg(rec, g, tid);
    const unsigned m0 = __float_as_uint(g8.w);
    // the step's dot product is summed in FP32 over the thread's 35 edges and then
    // added to the FP64 accumulator
    float zy = 0.0f;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        __builtin_amdgcn_sched_barrier(0);
        const float4 qr = q[r % QD];
        if constexpr (QD == 4) {
            if (r >= 2 && r < 6) q[(r + 2) & 3] = rg(rec, r + 2, tid);  // rows 4..7 into the registers of rows 0..3
        } else {
            if (r + QD < kR) q[r % QD] = rg(rec, r + QD, tid);  // row r + QD into the registers of row r
        }
        Z.e1a[r] = (m0 >> (4 * r + 0)) & 1u ? Z.e1a[r] : 0.0f;
        Z.e1b[r] = (m0 >> (4 * r + 1)) & 1u ? Z.e1b[r] : 0.0f;
        Z.e2a[r] = (m0 >> (4 * r + 2)) & 1u ? Z.e2a[r] : 0.0f;
        Z.e2b[r] = (m0 >> (4 * r + 3)) & 1u ? Z.e2b[r] : 0.0f;
        zy = fmaf(Z.e1a[r], qr.x, zy);
        zy = fmaf(Z.e1b[r], qr.y, zy);
        zy = fmaf(Z.e2a[r], qr.z, zy);
        zy = fmaf(Z.e2b[r], qr.w, zy);
        float s1a, s1b, s2a, s2b;
        lds_ld2(S1 + r * kFusedMax, s1a, s1b);
        lds_ld2(S2 + r * kFusedMax, s2a, s2b);
        lds_st2(S1 + r * kFusedMax, s1a + Z.e1a[r], s1b + Z.e1b[r]);
        lds_st2(S2 + r * kFusedMax, s2a + Z.e2a[r], s2b + Z.e2b[r]);
        pin4(Z.e1a[r], Z.e1b[r], Z.e2a[r], zy);
    }
    // bottom boundary edges (strip 15) and right boundary edges (lanes 0..7): q is a NaN where
    // the projection's derivative is 0
    const bool mba = !__builtin_isnan(g8.x), mbb = !__builtin_isnan(g8.y), mr = !__builtin_isnan(g8.z);
    Z.ba = c.last && mba ? Z.ba : 0.0f;
    Z.bb = c.last && mbb ? Z.bb : 0.0f;
    if (c.last) {
        zy = fmaf(Z.ba, mba ? g8.x : 0.0f, fmaf(Z.bb, mbb ? g8.y : 0.0f, zy));
        float sa, sb;
        lds_ld2(&L.Sb[c.ja], sa, sb);
        lds_st2(&L.Sb[c.ja], sa + Z.ba, sb + Z.bb);
    }
    if (c.lane < kR) {
        const float zr = mr ? RZ[row] : 0.0f;
        RZ[row] = zr;
        zy = fmaf(zr, mr ? g8.z : 0.0f, zy);
        L.Sr[row] += zr;
    }
    acc_q += (double)zy;
    lds_st2(&L.zt[sx][c.s][c.ja], Z.e1a[0], Z.e1b[0]);
    __syncthreads();

    // (2) div zbar of the strip's last row, published for the strip below
    const float *RZr = RZ + c.il0;
    float za7, zb7;  // zbar on the edges below the last row
    lds_ld2(&L.zt[sx][c.s < kWaves - 1 ? c.s + 1 : c.s][c.ja], za7, zb7);
    za7 = c.last ? Z.ba : za7;
    zb7 = c.last ? Z.bb : zb7;
    float da7, db7;
    full_row_div(Z, RZr[kR - 1], kR - 1, za7, zb7, da7, db7);
    lds_st2(&L.dl[c.s][c.ja], da7, db7);
    __syncthreads();

    // (3) row sweep: div zbar, ybar and the adjoint updates
    float dua = 0.0f, dub = 0.0f;  // div zbar of the row above (0 above the tile)
    if (c.s > 0) lds_ld2(&L.dl[c.s - 1][c.ja], dua, dub);
    const float bk = 1.0f + beta;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        __builtin_amdgcn_sched_barrier(0);  // one row at a time: bounds the registers in flight
        float da = da7, db = db7;
        if (r < kR - 1) full_row_div(Z, RZr[r], r, Z.e1a[r + 1], Z.e1b[r + 1], da, db);
        const float dlb = from_left(db);  // div zbar of column a - 1 (0 left of the tile)
        float y1a = fmaf(-kL, dua - da, ak * Z.e1a[r]);
        float y1b = fmaf(-kL, dub - db, ak * Z.e1b[r]);
        float y2a = fmaf(-kL, dlb - da, ak * Z.e2a[r]);
        const float y2b = fmaf(-kL, da - db, ak * Z.e2b[r]);
        if (r == 0 && !c.top_var) y1a = y1b = 0.0f;  // image boundary: not variables
        if (!c.left_var) y2a = 0.0f;
        if (mom) {
            P.e1a[r] = fmaf(bk, y1a, P.e1a[r]);
            P.e1b[r] = fmaf(bk, y1b, P.e1b[r]);
            P.e2a[r] = fmaf(bk, y2a, P.e2a[r]);
            P.e2b[r] = fmaf(bk, y2b, P.e2b[r]);
            Z.e1a[r] = -beta * y1a;
            Z.e1b[r] = -beta * y1b;
            Z.e2a[r] = -beta * y2a;
            Z.e2b[r] = -beta * y2b;
        } else {
            P.e1a[r] += y1a;
            P.e1b[r] += y1b;
            P.e2a[r] += y2a;
            P.e2b[r] += y2b;
            Z.e1a[r] = Z.e1b[r] = Z.e2a[r] = Z.e2b[r] = 0.0f;
        }
        if (r == kR - 1) {  // bottom boundary edges (strip 15)
            const bool v = c.last && c.bot_var;
            const float yba = v ? fmaf(-kL, da, ak * Z.ba) : 0.0f;
            const float ybb = v ? fmaf(-kL, db, ak * Z.bb) : 0.0f;
            if (mom) {
                P.ba = fmaf(bk, yba, P.ba);
                P.bb = fmaf(bk, ybb, P.bb);
                Z.ba = -beta * yba;
                Z.bb = -beta * ybb;
            } else {
                P.ba += yba;
                P.bb += ybb;
                Z.ba = Z.bb = 0.0f;
            }
        }
        if (c.lane == 63) L.dR[c.il0 + r] = db;  // div zbar of the last column
        pin4(P.e1a[r], P.e1b[r], P.e2a[r], P.e2b[r]);
        pin4(Z.e1a[r], Z.e1b[r], Z.e2a[r], Z.e2b[r]);
        dua = da;
        dub = db;
    }
    if (c.lane < kR) {  // right boundary edges
        const float yr = c.right_var ? fmaf(-kL, L.dR[row], ak * RZ[row]) : 0.0f;
        if (mom) {
            RP[row] = fmaf(bk, yr, RP[row]);
            RZ[row] = -beta * yr;
        } else {
            RP[row] += yr;
            RZ[row] = 0.0f;
        }
    }
}

// reverse steps k = K .. 1 (the slots swap roles every step)
template <int K, int QD = 4, int k = K>
__device__ __forceinline__ void bwd_steps(const BwdCtx &c, BwdLds &L, Slot &Z, Slot &P, const float *beta,
                                          const float4 *rec, long long rec_step, double &acc_q)
{
    if constexpr (k >= 1) {
        bwd_step<(k >= 3), QD>(c, L, Z, P, (K - k) & 1, k >= 3 ? beta[k] : 0.0f, rec + (k - 1) * rec_step, acc_q);
        bwd_steps<K, QD, k - 1>(c, L, P, Z, beta, rec, rec_step, acc_q);
    }
}

}  // namespace

// p + byte offset off, the offset zero-extended: with p uniform the access takes the scalar base
// and one 32-bit VGPR offset, instead of a 64-bit address per row
template <class T>
__device__ __forceinline__ T *at_b(T *p, unsigned off)
{
    return (T *)((char *)p + off);
}
template <class T>
__device__ __forceinline__ const T *at_b(const T *p, unsigned off)
{
    return (const T *)((const char *)p + off);
}

// Where the epilogue of a reverse outer step puts pbar^n: the per-step kernel stores it, and
// phatbar on the interface copies, to HBM; the persistent kernel writes it over S in LDS as S is
// consumed (S1, S2 on the thread's own entries, Sb, the right column in rx[0]) and stages phatbar
// of the interface copies for the transposed multiplier update (ih: [side][edge], sides as in
// exchange.h).  nxa, nxb (persistent kernel, strips 0..14): S on the top edges of the next strip's
// first row, read before the barrier that precedes the epilogue (that strip overwrites them).
struct EpiOut {
    float *pb1, *pb2, *hb1, *hb2;
    float *ih;
    float nxa, nxb;
};

// The epilogue of the reverse of one outer step, from xbar_0 in A (right column in rx[rxs]) and S:
// pbar^n = xbar_0 + phatbar with phatbar = S / (L tau) (0 on the image boundary), fbar -= div S / L,
// and the step's alpha derivative besides sum_k <zbar_k, q_k>, returned:
// dA/tau <phat, S> - dA <f, div S> (phat from p~^n, t copies + tau lambda^(n+1), s copies - tau lambda^(n+1)).
template <bool KEEP>
__device__ __forceinline__ double bwd_epilogue(const BwdCtx &c, BwdLds &L, Slot &A, int rxs, const SubTile &tl,
                                               const ImgDev &im, const float *x1, const float *x2, const float *lam,
                                               const float *f_tile, float *gf_tile, EpiOut o, long long P1,
                                               long long P2, float tau, float itau)
{
    // (the persistent kernel: the column passes through opaque() here, so that the addresses formed
    // from it are formed in the epilogue and not kept from the top of the outer step)
    const int H = im.H, W = im.W, s = c.s, lane = c.lane, ja = KEEP ? opaque(c.ja) : c.ja, il0 = c.il0;
    const bool top_bnd = tl.ra == 0, bot_bnd = tl.ra + kFusedMax == H, right_bnd = tl.ca + kFusedMax == W;
    const float invL = im.invL, hL = invL * itau;
    const double dA = im.dA;
    double sp = 0.0, fs = 0.0;  // <phat, S>, <f, div S>
    // the row addresses of pbar are formed again here (kept from the prologue they would stay live
    // through the steps, in scratch); phatbar is needed on the interface copies only (the interface
    // transpose reads nothing else), so it is written there alone
    if constexpr (!KEEP) asm volatile("" : "+s"(o.pb1), "+s"(o.pb2));
    const bool top_if = tl.r > 0, left_if = tl.c > 0;
    // the persistent kernel keeps slot A through the epilogue: there the row accesses take the
    // row's (uniform) base and the thread's byte offset along it, one register for all rows
    const unsigned jb = (unsigned)ja * 4u;
    auto row_at = [&](auto *row) { return KEEP ? at_b(row, jb) : row + ja; };
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        if constexpr (KEEP) __builtin_amdgcn_sched_barrier(0);  // one row's loads at a time
        const int il = il0 + r;
        const long long gi = tl.ra + il;
        float s1a, s1b, s2a, s2b;
        lds_ld2(&L.S1[il][ja], s1a, s1b);
        lds_ld2(&L.S2[il][ja], s2a, s2b);
        // anchors phat of the owned edges (t copies +tau lambda)
        float x1a, x1b, x2a, x2b;
        ld2(row_at(x1 + (long long)il * P1), x1a, x1b);
        ld2(row_at(x2 + (long long)il * P2), x2a, x2b);
        if (il == 0 && tl.r > 0) {
            const float *lr = row_at(lam + (long long)(tl.r - 1) * W + tl.ca);
            x1a = fmaf(tau, lr[0], x1a);
            x1b = fmaf(tau, lr[1], x1b);
        }
        if (ja == 0 && tl.c > 0) x2a = fmaf(tau, lam[im.nlh + (long long)(tl.c - 1) * H + gi], x2a);
        sp += (double)x1a * s1a + (double)x1b * s1b + (double)x2a * s2a + (double)x2b * s2b;
        // the row's edges
        const bool tv = !(il == 0 && top_bnd);
        const float h1a = tv ? hL * s1a : 0.0f, h1b = tv ? hL * s1b : 0.0f;
        const float h2a = c.left_var ? hL * s2a : 0.0f, h2b = hL * s2b;
        const float n1a = tv ? A.e1a[r] + h1a : 0.0f, n1b = tv ? A.e1b[r] + h1b : 0.0f;
        const float n2a = c.left_var ? A.e2a[r] + h2a : 0.0f, n2b = A.e2b[r] + h2b;
        if constexpr (KEEP) {
            if (il == 0 && top_if) {
                o.ih[ja] = h1a;
                o.ih[ja + 1] = h1b;
            }
            if (ja == 0 && left_if) o.ih[2 * kFusedMax + il] = h2a;
        } else {
            if (il == 0 && top_if) st2(o.hb1 + ja, h1a, h1b);
            if (ja == 0 && left_if) o.hb2[(long long)il * P2] = h2a;
            st2(o.pb1 + (long long)il * P1 + ja, n1a, n1b);
            st2(o.pb2 + (long long)il * P2 + ja, n2a, n2b);
        }
        // div S of the row's pixels (bottom edge: next row, or the bottom boundary row)
        float sba, sbb;
        if (KEEP && r == kR - 1 && !c.last) {
            sba = o.nxa;
            sbb = o.nxb;
        } else if (il < kFusedMax - 1) {
            lds_ld2(&L.S1[il + 1][ja], sba, sbb);
        } else {
            lds_ld2(&L.Sb[ja], sba, sbb);
        }
        const float sra = s2b;
        const float srb = ja + 2 < kFusedMax ? L.S2[il][ja + 2] : L.Sr[il];
        const float dsa = div4(s1a, sba, s2a, sra), dsb = div4(s1b, sbb, s2b, srb);
        float fa, fb, ga, gb;
        float *gp = row_at(gf_tile + (long long)il * W);
        ld2(row_at(f_tile + (long long)il * W), fa, fb);
        ld2(gp, ga, gb);
        st2(gp, fmaf(-invL, dsa, ga), fmaf(-invL, dsb, gb));
        fs += (double)fa * dsa + (double)fb * dsb;
        if constexpr (KEEP) {
            // over the row's S, after every read of it: the lane to the left reads S2 of column ja
            // (srb above) in the same instruction stream, the thread itself reads S1 of this row as
            // the previous row's bottom edges
            lds_st2(&L.S1[il][ja], n1a, n1b);
            lds_st2(&L.S2[il][ja], n2a, n2b);
        }
    }
    if (c.last) {  // bottom boundary edges: s copies -tau lambda
        float sa, sb;
        lds_ld2(&L.Sb[ja], sa, sb);
        float xa, xb;
        ld2(x1 + (long long)kFusedMax * P1 + ja, xa, xb);
        if (!bot_bnd) {
            const float *lb = lam + (long long)tl.r * W + tl.ca;
            xa = fmaf(-tau, lb[ja], xa);
            xb = fmaf(-tau, lb[ja + 1], xb);
        }
        sp += (double)xa * sa + (double)xb * sb;
        const float ha = bot_bnd ? 0.0f : hL * sa, hbv = bot_bnd ? 0.0f : hL * sb;
        const float na = bot_bnd ? 0.0f : A.ba + ha, nb = bot_bnd ? 0.0f : A.bb + hbv;
        if constexpr (KEEP) {
            lds_st2(&L.Sb[ja], na, nb);  // strip 15 alone reads Sb (above, and the row sweep's last row)
            if (!bot_bnd) {
                o.ih[kFusedMax + ja] = ha;
                o.ih[kFusedMax + ja + 1] = hbv;
            }
        } else {
            if (!bot_bnd) st2(o.hb1 + (long long)kFusedMax * P1 + ja, ha, hbv);
            st2(o.pb1 + (long long)kFusedMax * P1 + ja, na, nb);
        }
    }
    if (lane < kR) {  // right boundary edges: s copies -tau lambda
        const int il = il0 + lane;
        const float sr = L.Sr[il];
        float xr = x2[(long long)il * P2 + kFusedMax];
        if (!right_bnd) xr = fmaf(-tau, lam[im.nlh + (long long)tl.c * H + tl.ra + il], xr);
        sp += (double)xr * sr;
        const float hr = right_bnd ? 0.0f : hL * sr;
        const float nr = right_bnd ? 0.0f : L.rx[rxs][il] + hr;
        if constexpr (KEEP) {
            // this lane alone reads and writes these entries in the epilogue
            L.rx[0][il] = nr;
            L.rx[1][il] = 0.0f;
            if (!right_bnd) o.ih[3 * kFusedMax + il] = hr;
        } else {
            if (!right_bnd) o.hb2[(long long)il * P2 + kFusedMax] = hr;
            o.pb2[(long long)il * P2 + kFusedMax] = nr;
        }
    }
    (void)s;
    return dA * (double)itau * sp - dA * fs;
}

template <int KF>
__global__ __launch_bounds__(1024) void k_fused_bwd(FusedBwdArgs a)
{
    __shared__ BwdLds L;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const SubTile tl = a.subs[t];
    const ImgDev im = a.imgs[tl.img];
    BwdCtx c;
    c.s = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    c.lane = threadIdx.x & 63;
    c.ja = 2 * c.lane;
    c.il0 = kR * c.s;
    c.last = c.s == kWaves - 1;
    const int H = im.H, W = im.W, s = c.s, lane = c.lane, ja = c.ja, il0 = c.il0;
    const bool top_bnd = tl.ra == 0, bot_bnd = tl.ra + kFusedMax == H;
    const bool left_bnd = tl.ca == 0, right_bnd = tl.ca + kFusedMax == W;
    c.top_var = !(top_bnd && s == 0);
    c.left_var = !(left_bnd && lane == 0);
    c.bot_var = !bot_bnd;
    c.right_var = !right_bnd;
    c.ak = im.a_keep;
    c.kL = im.kL;
    const long long P1 = im.pitch1, P2 = im.pitch2;
    const long long row1 = (long long)tl.ra + tl.r;
    const long long col2 = (long long)tl.ca + tl.c;
    float *pb1 = a.pb1 + im.p1 + row1 * P1 + tl.ca, *pb2 = a.pb2 + im.p2 + (long long)tl.ra * P2 + col2;
    float *hb1 = a.hb1 + im.p1 + row1 * P1 + tl.ca, *hb2 = a.hb2 + im.p2 + (long long)tl.ra * P2 + col2;
    const float *x1 = a.x0_1 + im.p1 + row1 * P1 + tl.ca, *x2 = a.x0_2 + im.p2 + (long long)tl.ra * P2 + col2;
    const float *f_tile = a.f + im.px + (long long)tl.ra * W + tl.ca;
    float *gf_tile = a.gf + im.px + (long long)tl.ra * W + tl.ca;

    // ---- xbar_K = pbar^(n+1) into slot A (right column in LDS), S = 0, slot B = 0
    Slot A, B;
    A.ba = A.bb = 0.0f;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int il = il0 + r;
        ld2(pb1 + (long long)il * P1 + ja, A.e1a[r], A.e1b[r]);
        ld2(pb2 + (long long)il * P2 + ja, A.e2a[r], A.e2b[r]);
        lds_st2(&L.S1[il][ja], 0.0f, 0.0f);
        lds_st2(&L.S2[il][ja], 0.0f, 0.0f);
        B.e1a[r] = B.e1b[r] = B.e2a[r] = B.e2b[r] = 0.0f;
    }
    B.ba = B.bb = 0.0f;
    if (c.last) ld2(pb1 + (long long)kFusedMax * P1 + ja, A.ba, A.bb);
    if (s == 0) lds_st2(&L.Sb[ja], 0.0f, 0.0f);
    if (lane < kR) {
        L.rx[0][il0 + lane] = pb2[(long long)(il0 + lane) * P2 + kFusedMax];
        L.rx[1][il0 + lane] = 0.0f;
        L.Sr[il0 + lane] = 0.0f;
    }
    __syncthreads();

    // ---- the K reverse steps; xbar_0 ends in A (right column in rx[K & 1])
    double acc_q = 0.0;  // sum_k <zbar_k, q_k>
    const long long rec_step = (long long)gridDim.x * kRecGroups * kRecThreads;
    const float4 *rec = a.rec + (long long)t * kRecGroups * kRecThreads;  // uniform: this subdomain's record
    bwd_steps<KF>(c, L, A, B, a.beta, rec, rec_step, acc_q);
    if constexpr (KF & 1) copy_slot(A, B);
    __syncthreads();

    // ---- outputs and the alpha derivative
    double acc = acc_q;
    acc += bwd_epilogue<false>(c, L, A, KF & 1, tl, im, x1, x2, a.lam + im.lam, f_tile, gf_tile,
                               EpiOut{pb1, pb2, hb1, hb2, nullptr, 0.0f, 0.0f}, P1, P2, a.tau, a.inv_tau);
    // fixed-order reduction over the workgroup
    acc = wave_sum_d(acc);
    if (lane == 0) L.red[s] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < kWaves; ++w) tot += L.red[w];
        a.galpha[t] += tot;
    }
}

// ---- persistent reverse: every outer step of a range in one cooperative launch

// this thread's lane, formed from nothing (an asm statement, so it is formed here and not kept
// in a register from an earlier use)
__device__ __forceinline__ int fresh_lane()
{
    int x;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(x));
    return x;
}

// record groups the persistent reverse holds at once (its loop keeps slot A live through the
// epilogue and the exchange)
constexpr int kPersistBwdQD = 2;

struct PersistBwdLds {
    BwdLds b;
    float lam0[xchg::kSides][kFusedMax];  // lambdabar (first component) of the tile's interface multipliers
    float lamo[xchg::kSides][kFusedMax];  // lambdabar of the tile's own copy (s sides: second, t sides: third)
    int ok;                               // every wait of the current step completed
    double g;                             // this subdomain's alphabar partial sums (thread 0)
};
static_assert(sizeof(PersistBwdLds) <= 160 * 1024, "the persistent reverse's LDS exceeds a workgroup's 160 KB");

// The reverse of outer steps q = n_steps - 1 .. 0 of a range on subdomain t, one workgroup per
// subdomain for the whole range.  Between outer steps pbar lives in LDS, over S (S1, S2 and Sb; the
// right column in rx[0]): the epilogue writes it there as it consumes S, the transposed multiplier
// update adds to the interface copies there, and the next outer step takes it into slot A and
// clears S.  The interface copies take the operations of the interface-transpose kernel, so the
// result is bitwise that of the per-step launches: each tile publishes phatbar of its own copies,
// reads its neighbour's through the exchange words of exchange.h (step counter
// m = n_steps - 1 - q), and both tiles of an interface edge compute lambdabar's update from the
// two values.  Three workgroup barriers per outer step besides the steps' own: after the steps,
// after the epilogue, after the exchange.
template <int KF>
__global__ __launch_bounds__(1024) void k_persist_bwd(PersistBwdArgs a)
{
    __shared__ PersistBwdLds PL;
    BwdLds &L = PL.b;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const SubTile tl = a.b.subs[t];
    const ImgDev im = a.b.imgs[tl.img];
    BwdCtx c;
    c.s = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    c.lane = threadIdx.x & 63;
    c.ja = 2 * c.lane;
    c.il0 = kR * c.s;
    c.last = c.s == kWaves - 1;
    const int H = im.H, W = im.W, s = c.s, lane = c.lane, ja = c.ja, il0 = c.il0;
    const bool top_bnd = tl.ra == 0, bot_bnd = tl.ra + kFusedMax == H;
    const bool left_bnd = tl.ca == 0, right_bnd = tl.ca + kFusedMax == W;
    c.top_var = !(top_bnd && s == 0);
    c.left_var = !(left_bnd && lane == 0);
    c.bot_var = !bot_bnd;
    c.right_var = !right_bnd;
    c.ak = im.a_keep;
    c.kL = im.kL;
    const long long P1 = im.pitch1, P2 = im.pitch2;
    const long long row1 = (long long)tl.ra + tl.r;
    const long long col2 = (long long)tl.ca + tl.c;
    const long long o1 = im.p1 + row1 * P1 + tl.ca, o2 = im.p2 + (long long)tl.ra * P2 + col2;
    const float *f_tile = a.b.f + im.px + (long long)tl.ra * W + tl.ca;
    float *gf_tile = a.b.gf + im.px + (long long)tl.ra * W + tl.ca;
    const long long nlam = im.nlam;
    // side work: waves 0..7, side = wave / 2 (wave-uniform), edge si = 64 (wave % 2) + lane
    const int side = s >> 1;
    const bool side_lane = s < 2 * xchg::kSides && xchg::side_exists(im, tl, side);
    const bool side_s = side == 1 || side == 3;  // s copies: bottom and right sides
    const long long side_base = side_lane ? xchg::side_edge(im, tl, side, 0) : 0;
    float *lamb = a.lamb + im.lam + side_base;
    // phatbar of the interface copies, staged in the parity-1 zbar rows (written by the second
    // reverse step alone, after the first step's barriers)
    float *ih = &L.zt[1][0][0];

    // ---- pbar at the end of the range into LDS (over S), lambdabar
    {
        const float *pb1 = a.b.pb1 + o1, *pb2 = a.b.pb2 + o2;
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int il = il0 + r;
            float x, y;
            ld2(pb1 + (long long)il * P1 + ja, x, y);
            lds_st2(&L.S1[il][ja], x, y);
            ld2(pb2 + (long long)il * P2 + ja, x, y);
            lds_st2(&L.S2[il][ja], x, y);
        }
        if (c.last) {
            float x, y;
            ld2(pb1 + (long long)kFusedMax * P1 + ja, x, y);
            lds_st2(&L.Sb[ja], x, y);
        }
        if (lane < kR) {
            L.rx[0][il0 + lane] = pb2[(long long)(il0 + lane) * P2 + kFusedMax];
            L.rx[1][il0 + lane] = 0.0f;
        }
    }
    if (side_lane) {
        const int si = (s & 1) * 64 + lane;
        PL.lam0[side][si] = lamb[si];
        PL.lamo[side][si] = lamb[(side_s ? nlam : 2 * nlam) + si];
    }
    if (threadIdx.x == 0) {
        PL.ok = 1;
        PL.g = a.b.galpha[t];
    }
    const long long rec_step = (long long)gridDim.x * kRecGroups * kRecThreads;
    __syncthreads();

    for (int m = 0; m < a.n_steps; ++m) {
        const int q = a.n_steps - 1 - m;
        // the thread's lane and column are formed again in each outer step, so that the addresses
        // formed from them are not kept through the loop
        BwdCtx ci = c;
        ci.lane = fresh_lane();
        ci.ja = 2 * ci.lane;
        // ---- xbar_K = pbar^(q+1) from LDS into slot A, S = 0 (each thread its own entries)
        Slot A, B;
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int il = il0 + r;
            lds_ld2(&L.S1[il][ci.ja], A.e1a[r], A.e1b[r]);
            lds_ld2(&L.S2[il][ci.ja], A.e2a[r], A.e2b[r]);
            lds_st2(&L.S1[il][ci.ja], 0.0f, 0.0f);
            lds_st2(&L.S2[il][ci.ja], 0.0f, 0.0f);
            B.e1a[r] = B.e1b[r] = B.e2a[r] = B.e2b[r] = 0.0f;
        }
        A.ba = A.bb = B.ba = B.bb = 0.0f;
        if (c.last) {
            lds_ld2(&L.Sb[ci.ja], A.ba, A.bb);
            lds_st2(&L.Sb[ci.ja], 0.0f, 0.0f);
        }
        if (ci.lane < kR) L.Sr[il0 + ci.lane] = 0.0f;
        // ---- the K reverse steps of outer step q; xbar_0 ends in A (right column in rx[K & 1])
        double acc = 0.0;
        const float4 *rec = a.rec + (long long)q * a.rec_outer + (long long)t * kRecGroups * kRecThreads;
        bwd_steps<KF, kPersistBwdQD>(ci, L, A, B, a.b.beta, rec, rec_step, acc);
        if constexpr (KF & 1) copy_slot(A, B);
        float nxa = 0.0f, nxb = 0.0f;  // S on the next strip's first-row top edges (final since the last step's first barrier)
        if (!c.last) lds_ld2(&L.S1[il0 + kR][ci.ja], nxa, nxb);
        __syncthreads();

        // ---- pbar^q = xbar_0 + phatbar over S, fbar, the alpha derivative; phatbar of the interface copies staged
        const float *st = a.st + (long long)q * a.st_stride;
        const float *lam = a.st + (long long)(q + 1) * a.st_stride + a.lam_off + im.lam;
        acc += bwd_epilogue<true>(ci, L, A, KF & 1, tl, im, st + o1, st + a.p2_off + o2, lam, f_tile, gf_tile,
                                  EpiOut{nullptr, nullptr, nullptr, nullptr, ih, nxa, nxb}, P1, P2, a.b.tau,
                                  a.b.inv_tau);
        acc = wave_sum_d(acc);
        if (ci.lane == 0) L.red[s] = acc;
        __syncthreads();

        if (threadIdx.x == 0) {  // fixed-order reduction over the workgroup, added step by step
            double tot = 0.0;
            for (int w = 0; w < kWaves; ++w) tot += L.red[w];
            PL.g += tot;
        }
        // ---- the transposed multiplier update on the interface copies (pbar in LDS)
        if (side_lane) {
            const int si = (s & 1) * 64 + ci.lane;
            unsigned long long *xw = a.xch + (long long)(m & 1) * a.xch_stride + im.lam + side_base + si;
            const float hown = ih[side * kFusedMax + si];
            xchg::publish(xw + (side_s ? 0 : nlam), hown, m);
            float hoth = 0.0f;
            if (xchg::fetch(xw + (side_s ? nlam : 0), m, hoth, a.spin_limit)) {
                const float hs = side_s ? hown : hoth, ht = side_s ? hoth : hown;
                float l0 = PL.lam0[side][si], lo = PL.lamo[side][si], ds, dt;
                iface_bwd(hs, ht, a.b.tau, a.sigma, l0, side_s ? lo : 0.0f, side_s ? 0.0f : lo, ds, dt);
                float &v = side == 0 ? L.S1[0][si] : side == 1 ? L.Sb[si] : side == 2 ? L.S2[si][0] : L.rx[0][si];
                v = v + (side_s ? ds : dt);
                PL.lam0[side][si] = l0;
                PL.lamo[side][si] = side_s ? -a.sigma * l0 : a.sigma * l0;
            } else {
                PL.ok = 0;
                atomicOr(a.err, 1);
            }
        }
        __syncthreads();
        if (!PL.ok) break;  // a neighbour stopped publishing: leave (the host reports the error)
    }

    // ---- pbar at the start of the range (in LDS), lambdabar, alphabar
    {
        float *pb1 = a.b.pb1 + o1, *pb2 = a.b.pb2 + o2;
        asm volatile("" : "+s"(pb1), "+s"(pb2));
        const int jo = opaque(ja);
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int il = il0 + r;
            float x, y;
            lds_ld2(&L.S1[il][jo], x, y);
            st2(pb1 + (long long)il * P1 + jo, x, y);
            lds_ld2(&L.S2[il][jo], x, y);
            st2(pb2 + (long long)il * P2 + jo, x, y);
        }
        if (c.last) {
            float x, y;
            lds_ld2(&L.Sb[jo], x, y);
            st2(pb1 + (long long)kFusedMax * P1 + jo, x, y);
        }
        if (lane < kR) pb2[(long long)(il0 + lane) * P2 + kFusedMax] = L.rx[0][il0 + lane];
    }
    if (side_lane) {
        const int si = (s & 1) * 64 + lane;
        if (side_s) {
            lamb[si] = PL.lam0[side][si];
            lamb[nlam + si] = PL.lamo[side][si];
        } else {
            lamb[2 * nlam + si] = PL.lamo[side][si];
        }
    }
    if (threadIdx.x == 0) a.b.galpha[t] = PL.g;
    (void)left_bnd;
    (void)right_bnd;
}

namespace {

using BwdKernel = void (*)(FusedBwdArgs);

template <int... Ks>
struct BwdTable {
    static BwdKernel get(int K)
    {
        BwdKernel k = nullptr;
        ((K == Ks ? (k = k_fused_bwd<Ks>, 0) : 0), ...);
        return k;
    }
};
using Bwd = BwdTable<1, 2, 3, 4, 5, 6, 7, 8, 10>;

}  // namespace

bool fused_bwd_supported(int K) { return Bwd::get(K) != nullptr; }

namespace {

using PersistBwdKernel = void (*)(PersistBwdArgs);

template <int... Ks>
struct PersistBwdTable {
    static PersistBwdKernel get(int K)
    {
        PersistBwdKernel k = nullptr;
        ((K == Ks ? (k = k_persist_bwd<Ks>, 0) : 0), ...);
        return k;
    }
};
using PersistBwd = PersistBwdTable<1, 2, 3, 4, 5, 6, 7, 8, 10>;

}  // namespace

int persist_bwd_capacity(int device, int K)
{
    const PersistBwdKernel k = PersistBwd::get(K);
    int per_cu = 0, cus = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 1024, 0) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    return per_cu * cus;
}

hipError_t launch_persist_bwd(const PersistBwdArgs &a, int nsub, hipStream_t s)
{
    if (nsub <= 0 || a.n_steps <= 0) return hipSuccess;
    const PersistBwdKernel k = PersistBwd::get(a.b.n_inner);
    if (!k) return hipErrorInvalidValue;
    PersistBwdArgs arg = a;
    void *args[] = {&arg};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k), dim3(nsub), dim3(1024), args, 0, s);
}

hipError_t launch_fused_bwd(const FusedBwdArgs &a, int nsub, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (nsub <= 0) return hipSuccess;
    const BwdKernel k = Bwd::get(a.n_inner);
    if (!k) return hipErrorInvalidValue;
    if (e0)
        hipExtLaunchKernelGGL(k, dim3(nsub), dim3(1024), 0, s, e0, e1, 0, a);
    else
        hipLaunchKernelGGL(k, dim3(nsub), dim3(1024), 0, s, a);
    return hipGetLastError();
}

}  // namespace dtv
