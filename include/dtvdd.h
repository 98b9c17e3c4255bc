/*
 * dtvdd.h -- C-ABI of libdtvdd.so, the MI355X (gfx950) solver for the
 * primal-dual nonoverlapping domain decomposition of dual total-variation
 * problems (C.-O. Lee and J. Park, arXiv 1901.00682).
 *
 * The problem (Sec. 3, eq. model): min_u  alpha F(u) + TV(u) on an H x W image,
 * TV the anisotropic discrete total variation of the lowest-order
 * Raviart-Thomas dual (Sec. 2.3, eq. dTV), F one of
 *     L2:  F(u) = 1/2 sum_m (u - f)^2     (ROF denoising / L2 inpainting)
 *     L1:  F(u) = sum_m |u - f|           (TV-L1 denoising / L1 inpainting)
 * where the optional mask m (1 = observed pixel, 0 = pixel of the inpainting
 * set D) removes pixels from the fidelity term (Sec. 3, inpainting models).
 *
 * The method is Algorithm 1 (Sec. 4): the dual problem is torn along the
 * interfaces of an ny x nx grid of rectangular subdomains (Sec. 2.4), the
 * continuity of the normal flux is enforced with Lagrange multipliers lambda
 * (eq. DD), and the saddle problem is solved by an outer Chambolle-Pock
 * iteration whose primal step is a set of independent local problems, one
 * per subdomain (eq. DD_local), each solved approximately by n_inner steps of
 *     FISTA on the local dual (ROF without mask), or
 *     the accelerated primal-dual method of Chambolle-Pock (Sec. 5, any F).
 *
 * Data (all device buffers are owned by the caller; the library never
 * allocates or frees them):
 *   f, u, mask:  H x W row-major per image, images concatenated (px_off).
 *   p1, p2:      the torn dual variable p~ in the "torn layout":
 *       P1 has H+ny rows of p1_pitch floats (W used).  Subdomain row r,
 *          covering pixel rows [a, b), stores its horizontal edges
 *          (edge above pixel row a .. edge below pixel row b-1) in P1 rows
 *          a+r .. b+r.  Entry = normal flux in the +row direction.
 *       P2 has H rows of p2_pitch floats (W+nx used).  Subdomain column c,
 *          covering pixel columns [a, b), stores its vertical edges in P2
 *          columns a+c .. b+c.  Entry = normal flux in the +column direction.
 *       Interface edges thus appear twice (one copy per side); edges on the
 *       image boundary (P1 rows 0 and H+ny-1, P2 columns 0 and W+nx-1) are
 *       not unknowns (H_0(div)) and hold 0.
 *   lambda:      per image 3*n_lam floats: the multipliers lambda
 *       [n_lam_h horizontal-interface dofs, (r-1)*W + j for the interface
 *        between subdomain rows r-1 and r;  then n_lam_v vertical, (c-1)*H + i],
 *       then the side-s copies and the side-t copies of p~ at the previous
 *       outer step (same ordering), which Algorithm 1 needs for its
 *       extrapolation 2 p~^n - p~^(n-1).  Side s is the upper / left
 *       subdomain (lower row-major index); (B p~)_e = p~_s,e - p~_t,e.
 *
 * Error convention: every call returns DTV_OK (0) or a negative code; the
 * message of the last failing call on the calling thread is returned by
 * dtv_last_error().  Arguments are validated before anything is enqueued,
 * so a failing call leaves every output untouched.  Calls are stream-ordered
 * on the given stream (a hipStream_t, NULL = default stream).  The host waits
 * only where a call says so: dtv_dd_bind_workspace (synchronous uploads),
 * dtv_dd_solve with diagnostics (h_stats, gap_tol), with time_kernels, or
 * on the autotuner's first solve of a shape (DTV_SCHED_AUTO), and the calls
 * that return device results to the host (dtv_dd_diagnostics, dtv_dd_status,
 * dtv_dd_inner_counts with inner_tol).  A plan is not thread-safe; distinct
 * plans are independent.
 */
#ifndef DTVDD_H
#define DTVDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define DTV_OK 0
#define DTV_EINVAL (-1)      /* bad shape, cuts, alpha, step sizes, null pointer, unsupported combination */
#define DTV_ENOWS (-2)       /* no workspace bound, or the bound one is too small */
#define DTV_EHIP (-3)        /* a HIP runtime call failed (its message is in dtv_last_error) */
#define DTV_ESTATE (-4)      /* backward without a forward that saved its checkpoints */
#define DTV_ENONFINITE (-5)  /* the FP64 diagnostics saw NaN or Inf (outputs are still written) */

/* fidelity (Sec. 3) */
#define DTV_L2 0
#define DTV_L1 1
#define DTV_CV 2             /* convex Chan-Vese segmentation, eq. (CCV): F(u) = <u, g> + the
                                indicator of 0 <= u <= 1, g = (f - c1)^2 - (f - c2)^2 (c1, c2 =
                                cv_c1, cv_c2); prox_{a F}(z) = projection of z - a g onto [0, 1];
                                CP2 only, no mask */

/* local solver */
#define DTV_INNER_FISTA 0    /* projected FISTA on the local dual; L2 without mask only */
#define DTV_INNER_CP2 1      /* accelerated primal-dual (Sec. 5); any fidelity, mask allowed */

/* kernel schedule of the local solves (numerically identical results) */
#define DTV_SCHED_AUTO 0     /* pick by measurement: the first solve of a plan whose shape the
                                process has not seen runs its first outer steps in short timed
                                chunks, one per candidate (schedule x streaming rows; the
                                persistent launch at two chunk lengths, to separate its fixed
                                cost from its cost per step), keeps the one that would finish
                                the remaining steps first and caches it per shape (the
                                schedules round identically, so the result does not depend on
                                the choice); with too few outer steps, or with time_kernels, a
                                fixed rule picks: persistent, else fused, else streaming */
#define DTV_SCHED_STREAM 1   /* launches of up to steps_per_launch inner steps over all
                                subdomains, any size (rows swept, each step one row behind
                                the step before it) */
#define DTV_SCHED_FUSED 2    /* one workgroup per subdomain runs all inner steps on chip
                                (FISTA: subdomains up to 128 x 128; CP2: 128 x 128, or smaller
                                with the short sides on the image boundary) */
#define DTV_SCHED_PERSIST 3  /* one cooperative launch runs every outer step; the iterates stay
                                on chip between outer steps (no diagnostics; with
                                save_for_backward one launch per checkpoint segment, the
                                state saved between them).  FISTA with a fixed inner count: every
                                subdomain at most 128 x 128 (smaller ones run in a 128 x 128
                                frame); each image's subdomains resident on the device at
                                once, the images run in groups of launches.  CP2: every
                                subdomain 128 x 128, or smaller with its short sides on the
                                image boundary.  CP2 and inner_tol run every subdomain in one
                                launch, all resident at once */

typedef struct dtv_dd_plan dtv_dd_plan; /* opaque, owned by the library */

/* One image and its subdomain grid (Sec. 2.4; cuts need not be equal, any
   strictly increasing cut vector is accepted). */
typedef struct {
    int32_t H, W;              /* rows, columns; >= 1 */
    int32_t ny, nx;            /* subdomain rows / columns; 1 <= ny <= H, 1 <= nx <= W */
    const int32_t *row_cuts;   /* host array of ny+1 strictly increasing values, [0] = 0,
                                  [ny] = H; NULL: floor(k H / ny) */
    const int32_t *col_cuts;   /* host array of nx+1 values likewise; NULL: floor(k W / nx) */
    double alpha;              /* fidelity weight, > 0 (eq. model) */
} dtv_image_desc;

/* Solver settings.  Outer step sizes of Algorithm 1 and the local-solver
   parameters of Sec. 5 (defaults used by the paper: tau = 50, tau sigma = 1/2,
   tau0 = 10, tau0 sigma0 = 1/8, gamma = 1/(8 tau)). */
typedef struct {
    int32_t fidelity;          /* DTV_L2, DTV_L1 or DTV_CV */
    int32_t inner;             /* DTV_INNER_FISTA or DTV_INNER_CP2 */
    int32_t has_mask;          /* 1: d_mask is given */
    double tau, sigma;         /* > 0, tau * sigma <= 1/2 (|B|^2 = 2, Prop. B_norm) */
    double tau0, sigma0;       /* CP2: > 0, 8 tau0 sigma0 <= 1 (|div_s|^2 <= 8) */
    double gamma;              /* CP2: 0 <= gamma <= 1/tau (G_s^* is 1/tau-uniformly convex) */
    int32_t n_outer, n_inner;  /* iteration counts; n_outer >= 0, n_inner >= 1 */
    int32_t diag_every;        /* 0: none; k > 0: FP64 diagnostics every k outer steps and after the last */
    double gap_tol;            /* > 0 (single L2 or CV image without mask, diag_every > 0): stop at the
                                  first diagnostic step with gap <= gap_tol * |J| */
    int32_t warm_start;        /* 0: start from p~ = 0, lambda = 0, u = f; 1: continue from the
                                  state held in d_p1, d_p2, d_lambda (and d_u for CP2) */
    int32_t save_for_backward; /* 1: keep outer-step checkpoints for dtv_dd_backward (FISTA only) */
    int32_t ckpt_every;        /* outer steps between checkpoints, >= 1 */
    int32_t schedule;          /* DTV_SCHED_* */
    int32_t time_kernels;      /* 1: time every launch of the inner-step kernel with HIP events
                                  (read back with dtv_dd_kernel_time) */
    int32_t rows;              /* rows per wave strip of the streaming kernels: 4, 8, 16 or 32;
                                  0: chosen by the autotuner (16 until measured) */
    int32_t no_graphs;         /* 1: enqueue every outer step eagerly; 0: replay the outer steps of
                                  the per-step schedules from a captured hipGraph (when no
                                  per-step host work is asked for: diagnostics, checkpoints,
                                  kernel timing) */
    double cv_c1, cv_c2;       /* DTV_CV: the two region intensities of eq. (CCV); finite */
    int32_t full_problem;      /* 1: the undecomposed problem (Sec. 5 compares against it): every
                                  image is one subdomain (ny = nx = 1) and the local problem has no
                                  proximal term (the limit 1/tau -> 0, so tau and sigma play no
                                  part), i.e. the local solver is the plain method on the whole
                                  dual problem -- FISTA on the dual ROF problem, or the
                                  primal-dual method of Chambolle and Pock with tau0, sigma0 and
                                  gamma >= 0; each outer step restarts it from the current
                                  iterate (n_outer = 1: n_inner plain iterations); no
                                  save_for_backward */
    int32_t spin_limit;        /* persistent schedules: polls of one exchange word before a
                                  tile gives up on a neighbour and its launch ends early
                                  (dtv_dd_status then returns DTV_EHIP); 0: the default (2^21,
                                  about 0.1 s) */
    double inner_tol;          /* > 0: adaptive local solves (Sec. 5.1 stops them by relative change):
                                  each subdomain stops its local steps (FISTA or primal-dual) in
                                  an outer step after the first step k with |p_k - p_(k-1)|_2 <
                                  inner_tol |p_k|_2 over its own edge dofs (or p_k = p_(k-1)), at
                                  most n_inner (the cap, <= 100000) steps; the norms are summed in
                                  FP64; the primal-dual state is then (p_k, u_k).  The fused or
                                  the persistent schedule (or auto, which picks between them)
                                  only: every subdomain at most 128 x 128 (FISTA), or 128 x 128
                                  or smaller with its short sides on the image boundary (CP2);
                                  no save_for_backward.  0: fixed n_inner steps */
    int32_t steps_per_launch;  /* streaming schedule (both local solvers): the most local steps one
                                  launch runs, 1 .. 5 (0: the library's default, 5).  The n_inner
                                  steps of an outer step are cut into the fewest launches of at
                                  most that many steps, as evenly as possible (5 steps at 3 per
                                  launch: 3 + 2); the intermediate iterates of a launch stay in
                                  registers.  Every value gives the same result bitwise.  Ignored
                                  by the other schedules; the reverse pass's recomputation runs one
                                  step per launch */
    int32_t keep_records;      /* 1 (with save_for_backward, the fused or auto schedule and the
                                  on-chip reverse: every subdomain 128 x 128, n_inner 1 .. 8 or 10):
                                  the forward solve runs the recording fused kernel at every outer
                                  step and keeps the state before each outer step and that step's
                                  records (9 n_inner bytes per pixel), so that dtv_dd_backward runs
                                  the reverse steps alone, with no recomputation; ckpt_every is then
                                  not used.  The workspace grows to about n_outer (9 n_inner + 8)
                                  bytes per pixel.  0: checkpoints every ckpt_every outer steps,
                                  recomputed by the backward pass */
    int32_t reverse_schedule;  /* the reverse steps of dtv_dd_backward on the on-chip reverse (every
                                  subdomain 128 x 128): DTV_SCHED_AUTO = one cooperative launch per
                                  range of outer steps whose records are all kept (a checkpoint
                                  segment's when they fit 4 GiB, the whole solve's with keep_records)
                                  when every subdomain is resident at once, pbar kept on chip and
                                  the interface transpose done point to point between the tiles,
                                  else as DTV_SCHED_FUSED; DTV_SCHED_FUSED = one launch per outer
                                  step and an interface-transpose launch; DTV_SCHED_PERSIST = the
                                  cooperative launches or DTV_EINVAL at setup.  Every choice gives
                                  the same result bitwise.  A wait that gives up (spin_limit) is
                                  reported by dtv_dd_status */
} dtv_dd_params;

/* Where image `image` lives in the concatenated buffers (element offsets). */
typedef struct {
    int64_t px_off;            /* f, u, mask, grad_f, grad_u: H*W block at this offset */
    int64_t p1_off;            /* P1 block at this offset in d_p1 */
    int64_t p2_off;            /* P2 block at this offset in d_p2 */
    int64_t lam_off;           /* 3*n_lam lambda-state block at this offset in d_lambda */
    int32_t H, W, ny, nx;
    int32_t p1_rows, p1_pitch; /* H+ny rows, row pitch in floats (>= W) */
    int32_t p2_cols, p2_pitch; /* W+nx used columns, row pitch in floats */
    int32_t n_lam_h, n_lam_v;  /* (ny-1)*W and (nx-1)*H */
} dtv_layout;

/* Validate the problem and build a plan.  imgs: n_images >= 1 descriptors.
   Batched solves (n_images > 1) take every solver, fidelity and mask the
   single-image solve takes; gap_tol needs a single image. */
int dtv_dd_setup(const dtv_image_desc *imgs, int32_t n_images, const dtv_dd_params *prm, dtv_dd_plan **out);

/* Layout of one image (image in [0, n_images)); image = -1 reports totals:
   px_off = total pixels, p1_off / p2_off = floats of d_p1 / d_p2,
   lam_off = floats of d_lambda. */
int dtv_dd_layout(const dtv_dd_plan *plan, int32_t image, dtv_layout *out);

/* Device workspace the solver needs (bytes), and binding of a caller-owned
   allocation of at least that size (256-byte aligned).  Binding uploads the
   plan's metadata with a synchronous copy. */
int dtv_dd_workspace_bytes(const dtv_dd_plan *plan, size_t *bytes);
int dtv_dd_bind_workspace(dtv_dd_plan *plan, void *d_ws, size_t bytes);

/* Run n_outer steps of Algorithm 1 (Sec. 4):
     lambda <- lambda + sigma B(2 p~^n - p~^(n-1));  phat = p~^n - tau B^* lambda;
     every subdomain: n_inner local steps on eq. (DD_local), warm-started;
     u assembled from the local primal variables (for FISTA u = f + div p~ / alpha).
   d_f: input image(s); d_mask: NULL unless has_mask; d_u, d_p1, d_p2,
   d_lambda: outputs (and inputs when warm_start = 1).
   h_stats: NULL, or host room for n_images * (n_outer / diag_every + 1) rows of
   5 doubles [outer step, J(u), D(p_avg), gap = J - D, |B p~|_2], image-major;
   *n_rows (may be NULL) receives the number of rows per image.  J(u) =
   alpha F(u) + TV(u) (for DTV_CV, F(u) = <u, g> without the indicator: the
   prox keeps u in [0, 1]); D(p) = -(alpha F)^*(div p): -<f, div p> -
   |div p|^2/(2 alpha) for L2, sum over pixels of min(0, alpha g - div p) for
   DTV_CV, NaN (and so the gap) for L1 and for masked problems.  Returns
   DTV_ENONFINITE if a diagnostic is not finite.  Without diagnostics,
   time_kernels or a first autotuned solve the call only enqueues work; the
   persistent schedule's wait status is read with dtv_dd_status.
   Workspace: the bound one (dtv_dd_bind_workspace), DTV_ENOWS without. */
int dtv_dd_solve(dtv_dd_plan *plan, const float *d_f, const uint8_t *d_mask, float *d_u, float *d_p1,
                 float *d_p2, float *d_lambda, double *h_stats, int32_t *n_rows, void *stream);

/* Outcome of the last solve's (or, after dtv_dd_backward, the last backward pass's) persistent
   launches: a persistent schedule lets a subdomain wait a
   bounded number of polls (spin_limit) for each neighbour's interface copies; a wait that gives up
   sets an error word in the workspace that solve used, and the launch ends early.  The solve itself
   does not wait for its launches, so it cannot see that word; this call copies it to the host
   (stream-ordered on `stream`, returns after it arrives) and returns DTV_EHIP if any wait gave up,
   DTV_OK otherwise (also when the last solve ran no persistent launch).  After
   dtv_dd_solve_noalloc, call it before another plan's dtv_dd_solve_noalloc on the same device. */
int dtv_dd_status(dtv_dd_plan *plan, void *stream);

/* FP64 diagnostics of a given state (same quantities as a row of h_stats,
   without the step count): h_out receives 4 doubles per image. */
int dtv_dd_diagnostics(dtv_dd_plan *plan, const float *d_f, const uint8_t *d_mask, const float *d_u,
                       const float *d_p1, const float *d_p2, double *h_out, void *stream);

/* Reverse mode of the unrolled solve (FISTA, save_for_backward = 1): given
   dl/du, writes dl/df (H*W per image) and dl/dalpha (one float per image).
   The last dtv_dd_solve of this plan must have saved its checkpoints; d_f
   must hold the same data as in that solve. */
int dtv_dd_backward(dtv_dd_plan *plan, const float *d_f, const float *d_grad_u, float *d_grad_f,
                    float *d_grad_alpha, void *stream);

/* Average duration (ms) of the inner-step kernel launches timed in the last
   solve with time_kernels = 1, their count, the kernel's name and its
   algorithmic HBM bytes per launch (the bytes model of the chosen schedule). */
int dtv_dd_kernel_time(const dtv_dd_plan *plan, double *avg_ms, int64_t *launches, const char **name,
                       double *bytes_per_launch);

/* Average duration (ms) of the reverse mode's kernel launches timed in the last dtv_dd_backward
   of a plan with time_kernels = 1 and the fused reverse (every subdomain 128 x 128): which = 0
   the on-chip reverse steps (k_fused_bwd, one launch per outer step), which = 1 the recording
   forward (one launch per outer step; none with keep_records, where the forward solve records);
   their count, the kernel's name and its algorithmic HBM bytes per launch.  Zeros when nothing
   was timed. */
int dtv_dd_backward_kernel_time(const dtv_dd_plan *plan, int32_t which, double *avg_ms, int64_t *launches,
                                const char **name, double *bytes_per_launch);

/* The schedule the plan will use (DTV_SCHED_STREAM, DTV_SCHED_FUSED or DTV_SCHED_PERSIST). */
int dtv_dd_schedule(const dtv_dd_plan *plan, int32_t *schedule);

/* The schedule and streaming rows the plan uses and where they came from:
   source 0 = the fixed rule (nothing measured yet), 1 = measured by this
   plan's first solve, 2 = taken from the process-wide cache of an earlier
   plan with the same shape, 3 = set explicitly in dtv_dd_params. */
int dtv_dd_choice(const dtv_dd_plan *plan, int32_t *schedule, int32_t *rows, int32_t *source);

/* Local steps of every subdomain in the last solve: h_counts receives 2
   int32 per subdomain, [total over the outer steps, most in one outer step],
   image-major and row-major over each image's subdomain grid (n_outer *
   n_inner and n_inner without inner_tol; zeros before the first solve).
   With inner_tol it reads them from the device: stream-ordered on `stream`,
   returns after they arrive. */
int dtv_dd_inner_counts(dtv_dd_plan *plan, int32_t *h_counts, void *stream);

/* For callers that cannot allocate device memory: code under HIP graph capture, tight serving
   loops, harnesses that forbid allocation.  dtv_dd_solve with the library's own device scratch
   array (DTV_SCRATCH_BYTES bytes, one per device, held until the process ends) as the
   workspace instead of a bound one; the caller still passes every input and output buffer.
   Makes no device or pinned-host allocation and creates no stream, event or graph: the outer
   steps are enqueued eagerly with the plan's current schedule (explicit, cached, or the fixed
   rule: the autotuner does not run), and the host does not wait (read the persistent schedule's
   wait status with dtv_dd_status).
   Requirements: the plan's workspace size (dtv_dd_workspace_bytes) at most DTV_SCRATCH_BYTES
   (a plan set up with schedule = DTV_SCHED_PERSIST needs no rotation buffers, so a 2048 x 2048
   image with 16 x 16 subdomains needs about 3.5 MB), else DTV_ENOWS; diag_every = 0, gap_tol = 0,
   save_for_backward = 0 and time_kernels = 0, else DTV_EINVAL.
   The array is shared by every call on a device and keeps the last call's contents: the first
   call of a plan on a device (and the first after another plan's call there) uploads the plan's
   metadata into it with stream-ordered copies from host memory and clears the buffers that must
   start at zero with a fill kernel; later calls of the same plan go straight to the kernels (a
   caller capturing the call into a graph makes one uncaptured call first).  Calls that overlap
   on one device (other streams, other threads, other plans) race on the array. */
#define DTV_SCRATCH_BYTES (32u << 20)
int dtv_dd_solve_noalloc(dtv_dd_plan *plan, const float *d_f, const uint8_t *d_mask, float *d_u, float *d_p1,
                         float *d_p2, float *d_lambda, void *stream);

void dtv_dd_destroy(dtv_dd_plan *plan);

/* Message of the last failing call on this thread ("" if none). */
const char *dtv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DTVDD_H */
