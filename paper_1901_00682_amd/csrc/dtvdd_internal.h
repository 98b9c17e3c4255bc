// Internal declarations shared by the host runtime and the HIP kernels of
// libdtvdd.so.  Layout conventions are those documented in include/dtvdd.h.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dtv {

// Per-image descriptor as the kernels see it (lives in the workspace).
struct ImgDev {
    int H, W, ny, nx;
    long long px;        // offset of the H*W pixel block (f, u, mask, grads)
    long long p1, p2;    // offsets of P1 / P2 in the edge arrays
    int pitch1, pitch2;  // row pitches (floats) of P1 / P2
    long long lam;       // offset of the 3*n_lam lambda-state block
    int nlh, nlam;       // horizontal-interface dofs, all interface dofs
    long long rinfo;     // offset of H row-info words in the info array
    long long cinfo;     // offset of W column-info words
    long long rcut;      // offset of ny+1 row cuts in the info array
    long long ccut;      // offset of nx+1 column cuts
    float alpha, inv_alpha;
    float invL;          // FISTA step 1/L, L = 8/alpha + 1/tau
    float a_keep;        // FISTA: 1 - 1/(L tau), the weight of y in the update
    float kL;            // FISTA: 1/(alpha L), the weight of the divergence difference
    float pad0;
    double dA, dB;       // adjoint: d(1/L)/dalpha = 8/(alpha L)^2, d(1/(alpha L))/dalpha = -1/(tau (alpha L)^2)
};

// Row / column info word: subdomain index << 2 | first << 0 | last << 1.
__host__ __device__ inline int info_sub(int w) { return w >> 2; }
__host__ __device__ inline bool info_first(int w) { return (w & 1) != 0; }
__host__ __device__ inline bool info_last(int w) { return (w & 2) != 0; }

// Work item of the streaming kernels: one wave handles columns
// [j0 - 1, j0 + 62] (lane 0 is a halo column) and rows [i0, i0 + R).
struct StreamTile {
    int img, i0, j0, pad;
};

// Work item of the fused kernels: one subdomain.
struct SubTile {
    int img, r, c;       // image, subdomain row / column
    int ra, ca, h, w;    // pixel origin and extent
    int pad;
};

constexpr int kStreamCols = 63;   // output columns per wave
constexpr int kRowChoices = 4;    // rows per strip of the streaming kernels: 4, 8, 16 or 32
constexpr int kRecGroups = 9;     // float4 groups per thread in a step record of the fused kernel (fused_common.h)
constexpr int kRecThreads = 1024; // threads of a fused workgroup
constexpr size_t kSegRecordBytes = size_t(4) << 30;  // reverse mode: most bytes of step records kept at once
inline int row_index(int R) { return R <= 4 ? 0 : R <= 8 ? 1 : R <= 16 ? 2 : 3; }
constexpr int kFusedMax = 128;    // largest subdomain side handled by the fused kernel
constexpr int kMaxFusedInner = 64;  // largest n_inner of the fused kernel
constexpr int kMaxAdaptiveInner = 100000;  // largest cap on the local steps with adaptive stopping
constexpr unsigned kSpinLimitDefault = 1u << 21;  // persistent schedules: polls of one exchange word (~0.1 s)

// FISTA step of the streaming schedule.  The local gradient step
//   z = y - (1/L) [div_s^*(f + div_s y / alpha) + (y - phat)/tau]
// is evaluated as  z = a_keep y + c' - kL (d_before - d_after)  with
// d = div_s y per pixel and the per-edge constant
//   c' = (phat / tau - (f_before - f_after)) / L,
// which the first step of every outer iteration computes (from p~^n, lambda
// and f) and stores; later steps read it.  Same formulas as the fused kernel.
enum FistaMode { kFistaFirst = 0, kFistaPlain = 1, kFistaMomentum = 2 };

struct FistaStepArgs {
    const ImgDev *imgs;
    const StreamTile *tiles;
    int ntiles;
    const int *info;
    const float *xa1, *xa2;   // x_{k-1} (first step: x_0 = p~^n)
    const float *xb1, *xb2;   // x_{k-2} (momentum steps only)
    const float *lam;         // lambda state (first step)
    const float *f;           // image (first step)
    float *c1, *c2;           // c' (written by the first step, read by the others)
    float *out1, *out2;       // x_k
    float *z1, *z2;           // optional: z_k before the projection (recorded for the reverse pass)
    float beta;               // momentum coefficient of this step
    float tau;                // outer tau (anchor p~ -/+ tau lambda)
    float inv_tau;
};

// Reverse of one FISTA step over every subdomain (reverse mode of the
// unrolled solve).  With zbar = xbar_k * 1{|z_k| < 1}:
//   ybar = a_keep zbar - kL div_s^*(div_s zbar)   (the linear part of the step
//          is self-adjoint, so this is the forward stencil applied to zbar),
//   xbar_{k-1} += (1 + beta) ybar,  xbar_{k-2} -= beta ybar,
//   phatbar += zbar / (L tau),  fbar -= div_s zbar / L,
//   alphabar += -dA (<div zbar, f> + <zbar, y - phat>/tau) - dB <div zbar, div y>.
struct FistaBwdArgs {
    const ImgDev *imgs;
    const StreamTile *tiles;
    int ntiles;
    const int *info;
    const float *z1, *z2;      // z_k
    const float *xa1, *xa2;    // x_{k-1}
    const float *xb1, *xb2;    // x_{k-2} (momentum steps)
    const float *base1, *base2;  // p~^n
    const float *lam;          // lambda state holding lambda^{n+1}
    const float *f;
    const float *gx1, *gx2;    // xbar_k
    float *ga1, *ga2;          // xbar_{k-1} (accumulated)
    float *gb1, *gb2;          // xbar_{k-2} (accumulated, momentum steps)
    float *gh1, *gh2;          // phatbar (accumulated)
    float *gf;                 // fbar (accumulated)
    double *galpha;            // per-tile partial sums of alphabar (accumulated)
    float beta;                // beta_{k-1}
    float tau, inv_tau;
};

struct FusedArgs {
    const ImgDev *imgs;
    const SubTile *subs;
    const float *base1, *base2;  // p~^n
    const float *lam;            // lambda state of step n (lambda^n, p_s^(n-1), p_t^(n-1))
    float *lam_out;              // fused kernel: lambda state of step n + 1 (not aliasing lam)
    float sigma;
    float4 *rec;                 // reverse mode: the step records of full tiles (fused_common.h), or null
    const float *f;
    float *out1, *out2;          // p~^(n+1)
    float tau, inv_tau;
    int n_inner;
    float beta[kMaxFusedInner + 1];  // beta[k], k = 1..n_inner
    // adaptive inner stopping (tol2 > 0): up to n_inner steps per subdomain, momentum table
    // beta_dev[k] in device memory, per-subdomain [total steps, most steps in one outer step]
    double tol2;
    const float *beta_dev;
    int *counts;
    // launches of many rounds of full tiles: delaying blocks ahead of the tiles and their
    // delay in ticks of the 100 MHz constant clock (0: none; fused.hip)
    int stagger_blocks, stagger_ticks;
};

// Fused local primal-dual solves on full 128 x 128 subdomains (fused_cp2.hip).
// Step k + 1 (k = 0 .. n_inner - 1) uses tau_k = tk[k], sigma_k = sk[k], the
// extrapolation theta_k = th[k] of its result, and the weights c_keep = ck[k],
// c_anchor = ca[k] of the dual update.
struct FusedCp2Args {
    const ImgDev *imgs;
    const SubTile *subs;       // the subdomains (full, or framed in the fused kernel)
    float *p1, *p2;            // p~^n in (the persistent kernel: also p~^(n+1) out, in place)
    float *out1, *out2;        // fused kernel: p~^(n+1) out (not p1, p2: the tiles read each other's copies)
    const float *lam;          // fused kernel: lambda state before the multiplier update;
                               // persistent kernel: lambda state in
    float *lam_out;            // fused kernel: lambda state after the update (not lam)
    float sigma;               // multiplier step
    const float *f;
    const uint8_t *mask;       // NULL: every pixel observed
    float *u;                  // u in and out
    float tau;
    int fidelity;              // 0 L2, 1 L1, 2 convex Chan-Vese
    float cv_c1, cv_c2;
    int n_inner;
    int frames;                // fused kernel: some subdomains are framed (smaller than 128 x 128,
                               // their short sides on the image boundary)
    float tk[kMaxFusedInner], sk[kMaxFusedInner], th[kMaxFusedInner], ck[kMaxFusedInner], ca[kMaxFusedInner];
    // adaptive inner stopping (tol2 > 0): up to n_inner steps per subdomain with the step scalars
    // of step k + 1 in device memory, tab[5 k .. 5 k + 4] = tk, sk, th, ck, ca (k < n_inner), and
    // per-subdomain [total steps, most steps in one outer step] in counts
    double tol2;
    const float *tab;
    int *counts;
};

// Persistent primal-dual schedule (persist_cp2.hip): every outer step in one cooperative launch,
// p~, u and lambda updated in place; xch, err as in PersistArgs.
struct PersistCp2Args {
    FusedCp2Args ca;
    float *lam_out;
    unsigned long long *xch;
    long long xch_stride;
    int *err;
    int n_outer;
    float sigma;
    unsigned spin_limit;
};

struct Cp2StepArgs {
    const ImgDev *imgs;
    const StreamTile *tiles;
    int ntiles;
    const int *info;
    const float *xa1, *xa2;   // x_{k-1} (the current p)
    const float *xb1, *xb2;   // x_{k-2} (for the extrapolation; theta_prev = 0 on the first step)
    const float *base1, *base2;
    const float *lam;
    const float *f;
    const uint8_t *mask;      // NULL: all observed
    const float *u_in;
    float *u_out;
    float *out1, *out2;
    float theta_prev;         // extrapolation weight of xbar = x + theta_prev (x - x_prev)
    float sk;                 // sigma_k
    float tk;                 // tau_k
    float tau;                // outer tau
    float c_keep, c_anchor;   // tau/(tau+tau_k), tau_k/(tau+tau_k) (1 and 0 without the proximal term)
    int fidelity;             // 0 L2, 1 L1, 2 convex Chan-Vese
    float cv_c1, cv_c2;       // Chan-Vese intensities
};

// Kernel launchers (kernels.hip).
hipError_t launch_lambda(const ImgDev *imgs, int nimg, int max_nlam, const int *info, const float *p1,
                         const float *p2, float *lam, float sigma, hipStream_t s);
// e0 / e1: optional events stamped at the kernel's start and end (launch timing)
hipError_t launch_fista_step(const FistaStepArgs &a, int mode, int rows, hipStream_t s, hipEvent_t e0 = nullptr,
                             hipEvent_t e1 = nullptr);
hipError_t launch_cp2_step(const Cp2StepArgs &a, bool extrapolate, int rows, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);
hipError_t launch_fused_cp2(const FusedCp2Args &a, int nsub, hipStream_t s, hipEvent_t e0 = nullptr,
                            hipEvent_t e1 = nullptr);
hipError_t launch_persist_cp2(const PersistCp2Args &a, int nsub, hipStream_t s);
int persist_cp2_capacity(int device);
hipError_t launch_u_from_p(const ImgDev *imgs, int nimg, int maxH, int maxW, const int *info, const float *p1,
                           const float *p2, const float *f, float *u, hipStream_t s);
// zero `bytes` bytes (a multiple of 4) at p with a fill kernel
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_zero_boundary(const ImgDev *imgs, int nimg, int maxH, int maxW, float *p1, float *p2,
                                hipStream_t s);
// FP64 diagnostics: per image 6 partial sums reduced into out[img*6 + q]:
// q = 0 fidelity sum, 1 TV, 2 <f, div p_avg> (Chan-Vese: sum of min(0, alpha g - div p_avg)),
// 3 |div p_avg|^2, 4 |B p|^2, 5 non-finite count.
hipError_t launch_diag(const ImgDev *imgs, int nimg, int maxH, int maxW, const int *info, const float *p1,
                       const float *p2, const float *f, const float *u, const uint8_t *mask, int fidelity,
                       double cv_c1, double cv_c2,
                       double *partials, int nblk_per_img, double *out, hipStream_t s);
int diag_blocks_per_image(int maxH, int maxW);
// Persistent schedule: every outer step in one cooperative launch (persist.hip).
// The subdomains of the launch are at most 128 x 128 and resident on the device at once.
// frames: 0 every one is a full 128 x 128 tile, 1 the smaller ones have their short sides on the
// image boundary, 2 any smaller ones (run in a 128 x 128 frame with masks).
struct PersistArgs {
    FusedArgs fa;          // base = p~^0 (read), out = p~^N (written; may alias base), lam = lambda state in
    float *lam_out;        // lambda state out (may alias fa.lam)
    unsigned long long *xch;  // exchange words of the extrapolated copies: 2 slots of xch_stride, zero at launch
    long long xch_stride;     // >= length of the lambda state
    int *err;                 // set to 1 when a wait for a neighbour times out, 0 at launch
    int n_outer;
    float sigma;
    unsigned spin_limit;      // polls of one exchange word before a wait gives up
};
bool persist_supported(int device);
int persist_capacity(int device);  // workgroups of the persistent kernel resident at once
hipError_t launch_persist_fista(const PersistArgs &a, int nsub, int frames, hipStream_t s);

// Reverse mode of one outer step on full 128 x 128 subdomains (fused_bwd.hip),
// from the step records of the fused kernel.
struct FusedBwdArgs {
    const ImgDev *imgs;
    const SubTile *subs;
    const float4 *rec;           // the forward's step records (all subdomains, all steps)
    const float *x0_1, *x0_2;    // p~^n
    const float *lam;            // lambda state holding lambda^(n+1)
    const float *f;
    float *pb1, *pb2;            // in: pbar^(n+1); out: xbar_0 + phatbar (0 on the image boundary)
    float *hb1, *hb2;            // out: phatbar
    float *gf;                   // fbar (accumulated)
    double *galpha;              // per-subdomain partial sums of alphabar (accumulated)
    float tau, inv_tau;
    int n_inner;
    float beta[kMaxFusedInner + 1];
};
bool fused_bwd_supported(int K);
hipError_t launch_fused_bwd(const FusedBwdArgs &a, int nsub, hipStream_t s, hipEvent_t e0 = nullptr,
                            hipEvent_t e1 = nullptr);

// whether the fused kernel can record its steps for this inner count (full tiles only)
bool fused_record_supported(int K);
// workgroups of the full-tile fused kernel resident on the device at once
int fused_capacity(int device);
// subs[0, nfull) are 128 x 128 tiles (specialised kernel), subs[nfull, nfull + nframed) framed
// tiles (smaller, their short sides on the image boundary: the specialised kernel in a 128 x 128
// frame), the rest any other tiles of at most 128 x 128 (the specialised kernel in a frame, with
// masks; the general kernel with adaptive stopping or recording)
hipError_t launch_fused_fista(const FusedArgs &a, int nsub, int nfull, int nframed, hipStream_t s,
                              hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// reverse-mode kernels (kernels_bwd.hip)
hipError_t launch_fista_bwd_step(const FistaBwdArgs &a, bool momentum, int rows, hipStream_t s);
// u = f + div p / alpha reversed: fbar = ubar, pbar = div^*(ubar / alpha),
// galpha[tile] += -<ubar, div p> / alpha^2
hipError_t launch_bwd_final_u(const ImgDev *imgs, const StreamTile *tiles, int ntiles, int rows, const int *info,
                              const float *p1, const float *p2, const float *ubar, float *fbar, float *pb1,
                              float *pb2, double *galpha, hipStream_t s);
// pbar = xbar_0 + phatbar (all edges)
hipError_t launch_axpy_edges(const float *x, const float *y, float *out, long long n, hipStream_t s);
// per interface dof: lt = lamb - tau (hb_s - hb_t); pbar_s += prevb_s + 2 sigma lt;
// pbar_t += prevb_t - 2 sigma lt; prevb_s = -sigma lt; prevb_t = sigma lt; lamb = lt
hipError_t launch_bwd_interface(const ImgDev *imgs, int nimg, int max_nlam, const int *info, const float *hb1,
                                const float *hb2, float *pb1, float *pb2, float *lamb, float tau, float sigma,
                                hipStream_t s);
// dl/dalpha per image from the per-tile partial sums (fixed order)
hipError_t launch_alpha_reduce2(const StreamTile *tiles, int ntiles, const double *galpha, const SubTile *subs,
                                int nsub, const double *gsub, int nimg, float *out, hipStream_t s);
hipError_t launch_alpha_reduce(const StreamTile *tiles, int ntiles, int nimg, const double *galpha, float *out,
                               hipStream_t s);


}  // namespace dtv
