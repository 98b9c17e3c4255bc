// Host runtime and C-ABI of libdtvdd.so: plan building and validation, the
// torn HBM layout, workspace binding, and the outer loop of Algorithm 1
// (Lee & Park, arXiv 1901.00682, Sec. 4) driving the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dtvdd.h"
#include "bwd.h"
#include "cp2_multi.h"
#include "fista_multi.h"
#include "dtvdd_internal.h"

using namespace dtv;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return DTV_EHIP;
}

#define HIP_TRY(call, what)                        \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int pitch_of(int n) { return (int)align_up((size_t)n, 64); }

// steps per launch of the streaming primal-dual schedule when the parameters leave it open (the
// most a launch runs: n_inner = 5 in one launch, 10 in two)
constexpr int kDefaultStepsPerLaunch = kMaxMultiSteps;

// The local steps of one streaming primal-dual outer step cut into launches of at most spl steps,
// as evenly as the launch count allows, longer launches first (K = 5: spl 2 -> 2 2 1, spl 3 or 4
// -> 3 2, spl 5 -> 5).
std::vector<int> cp2_launch_steps(int K, int spl)
{
    std::vector<int> v;
    if (spl <= 1) {
        v.assign(K, 1);
        return v;
    }
    const int n = (K + spl - 1) / spl;
    for (int i = 0; i < n; ++i) v.push_back(K / n + (i < K % n ? 1 : 0));
    return v;
}

// One launch of that sequence: steps k0 .. k0 + steps - 1, reading x_{k0-1} from edge buffer ia and
// x_{k0-2} from ib, writing x_{k0+steps-2} to ic (steps >= 2) and x_{k0+steps-1} to id.
struct Cp2Launch {
    int k0, steps, ia, ib, ic, id;
};

// The launches of one outer step over nb edge buffers (4 with one-step launches, 5 otherwise) from
// x_0 in buffer base: each writes to the lowest buffers that hold neither x_0 (the anchors) nor
// what it reads.  One-step launches put x_k in the (k - 1) % 3-th buffer other than the base.
std::vector<Cp2Launch> cp2_stream_plan(int K, int spl, int base, int nb)
{
    std::vector<Cp2Launch> v;
    int a = base, b = base, k = 1;
    for (int S : cp2_launch_steps(K, spl)) {
        int fr[2] = {-1, -1}, q = 0;
        for (int x = 0; x < nb && q < 2; ++x)
            if (x != base && x != a && x != b) fr[q++] = x;
        const Cp2Launch l{k, S, a, b, S >= 2 ? fr[0] : -1, S >= 2 ? fr[1] : fr[0]};
        v.push_back(l);
        b = S >= 2 ? l.ic : a;
        a = l.id;
        k += S;
    }
    return v;
}

// The launches of one streaming FISTA outer step (lengths as cp2_launch_steps) over the x buffers
// 0, 1, 2 and 4 (buffer 3 holds c'): each writes to the lowest of them that holds none of its
// inputs.  x_0 is read only by the first launch, which forms c' from it, so its buffer is free
// afterwards; the last launch writes x_K alone (the next outer step restarts from it, without
// momentum), the others also x_{k+S-2} (ic; -1 where it is not written).
std::vector<Cp2Launch> fista_stream_plan(int K, int spl, int base)
{
    static const int X[4] = {0, 1, 2, 4};
    std::vector<Cp2Launch> v;
    const std::vector<int> steps = cp2_launch_steps(K, spl);
    int a = base, b = base, k = 1;
    for (size_t n = 0; n < steps.size(); ++n) {
        const int S = steps[n];
        const bool prev = S >= 2 && n + 1 < steps.size();
        int fr[2] = {-1, -1}, q = 0;
        for (int x : X)
            if (q < 2 && x != a && x != b) fr[q++] = x;
        const Cp2Launch l{k, S, a, b, prev ? fr[0] : -1, prev ? fr[1] : fr[0]};
        v.push_back(l);
        b = S >= 2 ? l.ic : a;
        a = l.id;
        k += S;
    }
    return v;
}

struct ImgHost {
    int H, W, ny, nx;
    double alpha;
    std::vector<int> rcut, ccut;
    dtv_layout L;
};

}  // namespace

namespace {

// a schedule and the rows per strip of the streaming kernels
struct Choice {
    int schedule, rows;
};

// what a captured hipGraph of outer steps was recorded with
struct GraphKey {
    int schedule = -1, rows = 0, base = 0;
    bool u_alt = false;
    int period = 0;
    const void *f = nullptr, *mask = nullptr, *u = nullptr, *p1 = nullptr, *p2 = nullptr, *lam = nullptr,
               *ws = nullptr;
    bool operator==(const GraphKey &o) const
    {
        return schedule == o.schedule && rows == o.rows && base == o.base && u_alt == o.u_alt && period == o.period &&
               f == o.f && mask == o.mask && u == o.u && p1 == o.p1 && p2 == o.p2 && lam == o.lam && ws == o.ws;
    }
};

// autotuner results of this process, by shape key
std::mutex g_tune_mu;
std::map<std::string, Choice> g_tune_cache;

std::atomic<uint64_t> g_plan_ids{0};

}  // namespace

struct dtv_dd_plan {
    dtv_dd_params prm;
    std::vector<ImgHost> imgs;
    int n = 0;
    int maxH = 0, maxW = 0, max_nlam = 0;
    int64_t tot_px = 0, tot_p1 = 0, tot_p2 = 0, tot_lam = 0;
    int schedule = DTV_SCHED_STREAM;
    int rows = 16;  // rows per wave strip of the streaming kernels
    double inv_tau = 0.0;  // 1/tau of the local proximal term (0 for the undecomposed problem)

    // metadata uploaded to the workspace at bind time
    std::vector<ImgDev> h_imgs;
    std::vector<int> h_info;
    std::vector<StreamTile> h_tiles[kRowChoices];  // streaming work lists, strips of 4 << ri rows
    // the same for the multi-step primal-dual kernel, by steps per launch S = 2 .. kMaxMultiSteps
    // (strips of multi_cols(S) columns); only for the S the plan's launches use
    std::vector<StreamTile> h_mtiles[kMaxMultiSteps - 1][kRowChoices];
    std::vector<SubTile> h_subs;
    std::vector<float> h_beta;  // adaptive stopping: the FISTA momentum table (beta[k], k = 0 .. n_inner)
    std::vector<float> h_cp2tab;  // adaptive stopping: the primal-dual step scalars (FusedCp2Args::tab)
    int n_full = 0;         // h_subs[0, n_full) are 128 x 128
    int n_framed = 0;       // h_subs[n_full, n_full + n_framed): framed (fused.hip), the rest any other
    // persistent FISTA schedule: the subdomains grouped by image into launches that fit on the device
    // at once (p_subs: the groups one after the other, each image's subdomains in grid order)
    std::vector<SubTile> p_subs;
    std::vector<int> p_group;  // first subdomain of each group in p_subs, then p_subs.size()
    // schedule choice: the fixed rule until measured (or cached, or explicit)
    bool tuned = false;
    int choice_source = 0;  // 0 rule, 1 measured, 2 cached, 3 explicit
    std::string key;        // shape key of the autotuner cache
    // hipGraph of one cycle of outer steps of a per-step schedule
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    GraphKey gkey;
    bool fused_ok = false;  // every subdomain fits the fused kernel
    int stagger_blocks = 0, stagger_ticks = 0;  // fused FISTA over many rounds of full tiles (fused.hip)
    bool persist_ok = false;  // the persistent schedule applies (full tiles, all resident, no per-step host work)

    uint64_t uid = 0;          // process-wide plan id (the scratch array records whose metadata it holds)
    char *run_ws = nullptr;    // workspace of the last solve: the bound one, or the scratch array
    bool ran_persist = false;  // the last solve ran the persistent schedule (its error word is in run_ws)
    size_t buf_bytes = 0;      // bytes of each rotation buffer (0: the plan runs only the persistent schedule)
    int spl = 1;               // the streaming primal-dual schedule runs up to spl local steps per launch

    // workspace layout (byte offsets)
    size_t off_imgs = 0, off_info = 0, off_tiles[kRowChoices] = {0, 0, 0, 0}, off_mtiles[kMaxMultiSteps - 1][kRowChoices] = {},
           off_subs = 0, off_psubs = 0, off_buf[4] = {0, 0, 0, 0},
           off_u2 = 0,
           off_part = 0, off_dout = 0, off_xch = 0, off_sync = 0, off_lamw = 0, ws_bytes = 0;
    int diag_nblk = 0;
    char *ws = nullptr;
    double *h_diag = nullptr;  // pinned host mirror of the diagnostics sums

    // reverse mode: outer-step checkpoints and the work buffers of the adjoint
    int nseg = 0;             // checkpoint slots ckpt(0..nseg-1) hold the state before steps 0, C, 2C, ...
    size_t state_floats = 0;  // one state: P1, P2, then the lambda state
    size_t off_ckpt = 0, off_seg = 0, off_xrec = 0, off_zrec = 0, off_lam1 = 0, off_xb = 0, off_hb = 0, off_pb = 0,
           off_lb = 0, off_galpha = 0, off_frec = 0, off_gsub = 0;
    bool fbwd = false;        // reverse mode with the fused kernels (every subdomain 128 x 128)
    bool pbwd = false;        // and the persistent reverse (one cooperative launch per range of outer steps)
    size_t off_bxch = 0;      // its exchange words
    bool seg_rec = false;     // fused reverse: the step records of a whole checkpoint segment are kept
    size_t rec_step = 0;      // bytes of one outer step's records
    bool adaptive = false;    // inner_tol > 0: the fused kernel stops each local solve by the relative-change rule
    size_t off_beta = 0, off_counts = 0;  // adaptive: momentum table, per-subdomain step counts
    size_t off_cp2tab = 0;                // adaptive primal-dual: the step scalars
    int last_outer = 0;       // outer steps run by the last solve
    bool solved = false;      // a solve has run
    bool saved = false;       // the last solve saved its checkpoints
    int saved_outer = 0;      // outer steps of that solve

    // timing of the inner-step kernel
    std::vector<hipEvent_t> events;
    double t_ms = 0.0;
    int64_t t_count = 0;
    // timing of the reverse mode's kernels (time_kernels): [0] the on-chip reverse steps,
    // [1] the recording forward; events in pairs, start and stop of each launch
    std::vector<hipEvent_t> bwd_events[2];
    double tb_ms[2] = {0.0, 0.0};
    int64_t tb_count[2] = {0, 0};

    ~dtv_dd_plan()
    {
        // a replay of the plan's graph may still be in flight on the caller's stream
        if (gexec) (void)hipDeviceSynchronize();
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (auto &v : bwd_events)
            for (hipEvent_t e : v) (void)hipEventDestroy(e);
        if (h_diag) (void)hipHostFree(h_diag);
    }

    const ImgDev *d_imgs() const { return (const ImgDev *)(ws + off_imgs); }
    const SubTile *d_subs() const { return (const SubTile *)(ws + off_subs); }
    const SubTile *d_psubs() const { return (const SubTile *)(ws + off_psubs); }
    const int *d_info() const { return (const int *)(ws + off_info); }
    const StreamTile *d_tiles(int R) const { return (const StreamTile *)(ws + off_tiles[row_index(R)]); }
    int ntiles(int R) const { return (int)h_tiles[row_index(R)].size(); }
    const StreamTile *d_mtiles(int S, int R) const { return (const StreamTile *)(ws + off_mtiles[S - 2][row_index(R)]); }
    int nmtiles(int S, int R) const { return (int)h_mtiles[S - 2][row_index(R)].size(); }
    // rotation buffer k: three always (FISTA: x in two, c' in the third), a fourth for the
    // multi-step primal-dual launches
    size_t buf_size(int k) const { return k < 3 || spl > 1 ? buf_bytes : 0; }
    float *buf1(int k) const { return (float *)(ws + off_buf[k]); }
    float *buf2(int k) const { return (float *)(ws + off_buf[k]) + tot_p1; }
    float *u2() const { return (float *)(ws + off_u2); }
    double *partials() const { return (double *)(ws + off_part); }
    size_t edges() const { return (size_t)(tot_p1 + tot_p2); }
    float *ckpt(int k) const { return (float *)(ws + off_ckpt) + (size_t)k * state_floats; }
    float *seg(int k) const { return (float *)(ws + off_seg) + (size_t)k * state_floats; }
    float *xrec(int k) const { return (float *)(ws + off_xrec) + (size_t)k * edges(); }
    float *zrec(int k) const { return (float *)(ws + off_zrec) + (size_t)k * edges(); }
    float *lam1() const { return (float *)(ws + off_lam1); }
    float *xb(int k) const { return (float *)(ws + off_xb) + (size_t)k * edges(); }
    float *hb() const { return (float *)(ws + off_hb); }
    float *pb() const { return (float *)(ws + off_pb); }
    float *lb() const { return (float *)(ws + off_lb); }
    double *galpha() const { return (double *)(ws + off_galpha); }
    // step records of the fused forward: outer step q of the segment (q = 0 without seg_rec)
    float4 *frec(int q = 0) const { return (float4 *)(ws + off_frec + (size_t)q * rec_step); }
    double *gsub() const { return (double *)(ws + off_gsub); }     // per-subdomain alpha partial sums
    unsigned long long *bxch() const { return (unsigned long long *)(ws + off_bxch); }
    double *dout() const { return (double *)(ws + off_dout); }
    unsigned long long *xch() const { return (unsigned long long *)(ws + off_xch); }
    float *lamw() const { return (float *)(ws + off_lamw); }  // second lambda state (fused schedule)
    unsigned *sync_words() const { return (unsigned *)(ws + off_sync); }  // error flag of the persistent kernel
    float *beta_tab() const { return (float *)(ws + off_beta); }
    const float *cp2_tab() const { return (const float *)(ws + off_cp2tab); }
    int *counts() const { return (int *)(ws + off_counts); }
    const int *run_counts() const { return (const int *)(run_ws + off_counts); }
    const unsigned *run_sync_words() const { return (const unsigned *)(run_ws + off_sync); }
};

// ---------------------------------------------------------------------------
// validation and plan building

static int check_cuts(const int32_t *given, int parts, int n, std::vector<int> &out, const char *what)
{
    out.resize(parts + 1);
    if (!given) {
        for (int k = 0; k <= parts; ++k) out[k] = (int)(((int64_t)k * n) / parts);
    } else {
        for (int k = 0; k <= parts; ++k) out[k] = given[k];
    }
    if (out[0] != 0 || out[parts] != n) return fail(DTV_EINVAL, std::string(what) + " cuts must start at 0 and end at the size");
    for (int k = 0; k < parts; ++k)
        if (out[k + 1] <= out[k]) return fail(DTV_EINVAL, std::string(what) + " cuts must be strictly increasing");
    return DTV_OK;
}

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

static std::vector<float> fista_betas(int K);

// Step sizes of the local accelerated primal-dual method (Chambolle-Pock Alg. 2, Sec. 5): step
// k + 1 uses tau_k = tk[k], sigma_k = sk[k] and the extrapolation theta_k = th[k], with
// theta_k = 1/sqrt(1 + 2 gamma tau_k), tau_(k+1) = theta_k tau_k, sigma_(k+1) = sigma_k / theta_k,
// reset to (tau0, sigma0) every outer step; computed in double precision.
static void cp2_steps(const dtv_dd_params &P, int K, std::vector<double> &tk, std::vector<double> &sk,
                      std::vector<double> &th)
{
    tk.assign(K + 1, 0.0);
    sk.assign(K + 1, 0.0);
    th.assign(K + 1, 0.0);
    double a = P.tau0, b = P.sigma0;
    for (int it = 0; it < K; ++it) {
        tk[it] = a;
        sk[it] = b;
        th[it] = 1.0 / std::sqrt(1.0 + 2.0 * P.gamma * a);
        a *= th[it];
        b /= th[it];
    }
}

// the weights of the local dual update: tau / (tau + tau_k) on x - tau_k div^* u and
// tau_k / (tau + tau_k) on the anchor (1 and 0 without the proximal term)
static float cp2_keep(const dtv_dd_params &P, double tk) { return P.full_problem ? 1.0f : (float)(P.tau / (P.tau + tk)); }
static float cp2_anchor(const dtv_dd_params &P, double tk) { return P.full_problem ? 0.0f : (float)(tk / (P.tau + tk)); }

static bool any_of_sched(int requested, int sched) { return requested == DTV_SCHED_AUTO || requested == sched; }

// How the full-tile step runs a subdomain: 0 a full 128 x 128 tile; 1 a framed tile (smaller, each
// short side on the image boundary); 2 any other tile of at most 128 x 128 (framed, with masks);
// 3 larger than 128 in either direction (the streaming kernels only)
static int frame_kind(const dtv_dd_plan *pl, const SubTile &st)
{
    if (st.h > kFusedMax || st.w > kFusedMax) return 3;
    if (st.h == kFusedMax && st.w == kFusedMax) return 0;
    const ImgHost &h = pl->imgs[st.img];
    return (st.h == kFusedMax || st.r == h.ny - 1) && (st.w == kFusedMax || st.c == h.nx - 1) ? 1 : 2;
}

// The autotuner's candidates: the schedules the plan admits (persistent, fused,
// streaming) times the streaming rows (4, 8, 16, 32), restricted by explicit
// choices in the parameters.
static std::vector<Choice> candidates(const dtv_dd_plan *pl)
{
    const dtv_dd_params &p = pl->prm;
    std::vector<Choice> c;
    if (pl->adaptive) {  // the stopping rule lives in the fused and persistent kernels
        if ((any_of_sched(p.schedule, DTV_SCHED_PERSIST)) && pl->persist_ok) c.push_back({DTV_SCHED_PERSIST, pl->rows});
        if (any_of_sched(p.schedule, DTV_SCHED_FUSED)) c.push_back({DTV_SCHED_FUSED, pl->rows});
        return c;
    }
    if (p.keep_records) {  // only the fused kernel records its steps
        c.push_back({DTV_SCHED_FUSED, pl->rows});
        return c;
    }
    const bool any = p.schedule == DTV_SCHED_AUTO;
    if ((any || p.schedule == DTV_SCHED_PERSIST) && pl->persist_ok) c.push_back({DTV_SCHED_PERSIST, pl->rows});
    if ((any || p.schedule == DTV_SCHED_FUSED) && pl->fused_ok) c.push_back({DTV_SCHED_FUSED, pl->rows});
    if (any || p.schedule == DTV_SCHED_STREAM) {
        if (p.rows)
            c.push_back({DTV_SCHED_STREAM, p.rows});
        else
            for (int R : {4, 8, 16, 32}) c.push_back({DTV_SCHED_STREAM, R});
    }
    return c;
}

// key of the autotuner cache: device, solver, inner count and every image's sizes and cuts
static std::string shape_key(const dtv_dd_plan *pl)
{
    const dtv_dd_params &p = pl->prm;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::string k = "dev" + std::to_string(dev) + ":" + std::to_string(p.inner) + ":" + std::to_string(p.fidelity) +
                    ":" + std::to_string(p.has_mask) + ":" + std::to_string(p.n_inner) + ":" +
                    std::to_string(p.schedule) + ":" + std::to_string(p.rows) + ":" +
                    std::to_string(pl->adaptive ? 1 : 0) + ":" + std::to_string(p.full_problem);
    for (const ImgHost &h : pl->imgs) {
        k += "|" + std::to_string(h.H) + "x" + std::to_string(h.W) + ":";
        for (int v : h.rcut) k += std::to_string(v) + ",";
        k += ":";
        for (int v : h.ccut) k += std::to_string(v) + ",";
    }
    return k;
}

extern "C" int dtv_dd_setup(const dtv_image_desc *imgs, int32_t n_images, const dtv_dd_params *prm,
                            dtv_dd_plan **out)
{
    if (!imgs || !prm || !out) return fail(DTV_EINVAL, "null argument");
    if (n_images < 1) return fail(DTV_EINVAL, "n_images must be >= 1");
    const dtv_dd_params &p = *prm;
    if (p.fidelity != DTV_L2 && p.fidelity != DTV_L1 && p.fidelity != DTV_CV)
        return fail(DTV_EINVAL, "fidelity must be DTV_L2, DTV_L1 or DTV_CV");
    if (p.inner != DTV_INNER_FISTA && p.inner != DTV_INNER_CP2) return fail(DTV_EINVAL, "unknown inner solver");
    if (p.inner == DTV_INNER_FISTA && (p.fidelity != DTV_L2 || p.has_mask))
        return fail(DTV_EINVAL, "FISTA local solver needs the L2 fidelity without mask (use CP2)");
    if (p.fidelity == DTV_CV && p.has_mask) return fail(DTV_EINVAL, "the Chan-Vese fidelity takes no mask");
    if (p.fidelity == DTV_CV && (!std::isfinite(p.cv_c1) || !std::isfinite(p.cv_c2)))
        return fail(DTV_EINVAL, "cv_c1 and cv_c2 must be finite");
    if (p.full_problem != 0 && p.full_problem != 1) return fail(DTV_EINVAL, "full_problem must be 0 or 1");
    const bool full = p.full_problem != 0;
    if (!full) {
        if (!finite_pos(p.tau) || !finite_pos(p.sigma)) return fail(DTV_EINVAL, "tau and sigma must be positive");
        if (p.tau * p.sigma > 0.5 * (1.0 + 1e-12)) return fail(DTV_EINVAL, "tau * sigma must be <= 1/2");
    }
    if (p.inner == DTV_INNER_CP2) {
        if (!finite_pos(p.tau0) || !finite_pos(p.sigma0)) return fail(DTV_EINVAL, "tau0 and sigma0 must be positive");
        if (8.0 * p.tau0 * p.sigma0 > 1.0 + 1e-12) return fail(DTV_EINVAL, "8 tau0 sigma0 must be <= 1");
        if (!(p.gamma >= 0.0) || !std::isfinite(p.gamma)) return fail(DTV_EINVAL, "gamma must be finite and >= 0");
        if (!full && p.gamma > 1.0 / p.tau * (1.0 + 1e-12)) return fail(DTV_EINVAL, "gamma must lie in [0, 1/tau]");
    }
    if (full && p.save_for_backward) return fail(DTV_EINVAL, "full_problem takes no save_for_backward");
    if (!(p.inner_tol >= 0.0) || !std::isfinite(p.inner_tol)) return fail(DTV_EINVAL, "inner_tol must be finite and >= 0");
    if (p.inner_tol > 0.0 && (p.save_for_backward || p.schedule == DTV_SCHED_STREAM))
        return fail(DTV_EINVAL, "inner_tol needs the fused or persistent schedule (or auto) and no save_for_backward");
    if (p.inner_tol > 0.0 && p.n_inner > kMaxAdaptiveInner)
        return fail(DTV_EINVAL, "inner_tol: n_inner (the cap) must be <= 100000");
    if (full)
        for (int b = 0; b < n_images; ++b)
            if (imgs[b].ny != 1 || imgs[b].nx != 1) return fail(DTV_EINVAL, "full_problem needs ny = nx = 1");
    if (p.n_outer < 0 || p.n_inner < 1) return fail(DTV_EINVAL, "n_outer must be >= 0 and n_inner >= 1");
    if (p.diag_every < 0) return fail(DTV_EINVAL, "diag_every must be >= 0");
    if (p.gap_tol < 0.0 || !std::isfinite(p.gap_tol)) return fail(DTV_EINVAL, "gap_tol must be finite and >= 0");
    if (p.gap_tol > 0.0 && (n_images != 1 || p.fidelity == DTV_L1 || p.has_mask || p.diag_every <= 0))
        return fail(DTV_EINVAL, "gap_tol needs one L2 or Chan-Vese image without mask and diag_every > 0");
    if (p.save_for_backward && (p.inner != DTV_INNER_FISTA || p.ckpt_every < 1))
        return fail(DTV_EINVAL, "save_for_backward needs FISTA and ckpt_every >= 1");
    if (p.save_for_backward && p.gap_tol > 0.0) return fail(DTV_EINVAL, "save_for_backward needs fixed iteration counts");
    if (p.schedule < DTV_SCHED_AUTO || p.schedule > DTV_SCHED_PERSIST) return fail(DTV_EINVAL, "unknown schedule");
    if (p.rows != 0 && p.rows != 4 && p.rows != 8 && p.rows != 16 && p.rows != 32)
        return fail(DTV_EINVAL, "rows must be 0, 4, 8, 16 or 32");
    if (p.no_graphs != 0 && p.no_graphs != 1) return fail(DTV_EINVAL, "no_graphs must be 0 or 1");
    if (p.spin_limit < 0) return fail(DTV_EINVAL, "spin_limit must be >= 0");
    if (p.steps_per_launch < 0 || p.steps_per_launch > kMaxMultiSteps)
        return fail(DTV_EINVAL, "steps_per_launch must be between 0 and 5");
    if (p.keep_records != 0 && p.keep_records != 1) return fail(DTV_EINVAL, "keep_records must be 0 or 1");
    if (p.keep_records && !p.save_for_backward) return fail(DTV_EINVAL, "keep_records needs save_for_backward");
    if (p.keep_records && p.schedule != DTV_SCHED_AUTO && p.schedule != DTV_SCHED_FUSED)
        return fail(DTV_EINVAL, "keep_records runs the fused schedule (auto or fused)");
    if (p.reverse_schedule != DTV_SCHED_AUTO && p.reverse_schedule != DTV_SCHED_FUSED &&
        p.reverse_schedule != DTV_SCHED_PERSIST)
        return fail(DTV_EINVAL, "reverse_schedule must be auto, fused or persistent");

    dtv_dd_plan *pl = new dtv_dd_plan();
    pl->uid = ++g_plan_ids;
    pl->prm = p;
    pl->n = n_images;
    pl->imgs.resize(n_images);
    int64_t px = 0, o1 = 0, o2 = 0, ol = 0;
    for (int b = 0; b < n_images; ++b) {
        const dtv_image_desc &d = imgs[b];
        ImgHost &h = pl->imgs[b];
        if (d.H < 1 || d.W < 1) { delete pl; return fail(DTV_EINVAL, "image sizes must be >= 1"); }
        if (d.ny < 1 || d.ny > d.H || d.nx < 1 || d.nx > d.W) {
            delete pl;
            return fail(DTV_EINVAL, "subdomain grid must satisfy 1 <= ny <= H and 1 <= nx <= W");
        }
        if (!finite_pos(d.alpha)) { delete pl; return fail(DTV_EINVAL, "alpha must be positive"); }
        if ((int64_t)(d.H + d.ny) * pitch_of(d.W) >= (1LL << 40)) { delete pl; return fail(DTV_EINVAL, "image too large"); }
        int rc = check_cuts(d.row_cuts, d.ny, d.H, h.rcut, "row");
        if (rc == DTV_OK) rc = check_cuts(d.col_cuts, d.nx, d.W, h.ccut, "column");
        if (rc != DTV_OK) { delete pl; return rc; }
        h.H = d.H; h.W = d.W; h.ny = d.ny; h.nx = d.nx; h.alpha = d.alpha;
        dtv_layout &L = h.L;
        L.H = d.H; L.W = d.W; L.ny = d.ny; L.nx = d.nx;
        L.p1_rows = d.H + d.ny;
        L.p1_pitch = pitch_of(d.W);
        L.p2_cols = d.W + d.nx;
        L.p2_pitch = pitch_of(d.W + d.nx);
        L.n_lam_h = (d.ny - 1) * d.W;
        L.n_lam_v = (d.nx - 1) * d.H;
        L.px_off = px;
        L.p1_off = o1;
        L.p2_off = o2;
        L.lam_off = ol;
        px += (int64_t)d.H * d.W;
        o1 += align_up((size_t)L.p1_rows * L.p1_pitch, 64);
        o2 += align_up((size_t)d.H * L.p2_pitch, 64);
        ol += align_up((size_t)3 * (L.n_lam_h + L.n_lam_v), 64);
        pl->maxH = std::max(pl->maxH, d.H);
        pl->maxW = std::max(pl->maxW, d.W);
        pl->max_nlam = std::max(pl->max_nlam, L.n_lam_h + L.n_lam_v);
    }
    pl->tot_px = px;
    pl->tot_p1 = o1;
    pl->tot_p2 = o2;
    pl->tot_lam = ol;

    // device metadata: image descriptors, info words, cuts, work lists
    // 1/tau of the local proximal term; 0 for the undecomposed problem
    pl->inv_tau = full ? 0.0 : 1.0 / p.tau;
    for (int b = 0; b < n_images; ++b) {
        const ImgHost &h = pl->imgs[b];
        ImgDev g{};
        g.H = h.H; g.W = h.W; g.ny = h.ny; g.nx = h.nx;
        g.px = h.L.px_off; g.p1 = h.L.p1_off; g.p2 = h.L.p2_off;
        g.pitch1 = h.L.p1_pitch; g.pitch2 = h.L.p2_pitch;
        g.lam = h.L.lam_off;
        g.nlh = h.L.n_lam_h; g.nlam = h.L.n_lam_h + h.L.n_lam_v;
        g.rinfo = (long long)pl->h_info.size();
        for (int r = 0; r < h.ny; ++r)
            for (int i = h.rcut[r]; i < h.rcut[r + 1]; ++i)
                pl->h_info.push_back((r << 2) | (i == h.rcut[r] ? 1 : 0) | (i == h.rcut[r + 1] - 1 ? 2 : 0));
        g.cinfo = (long long)pl->h_info.size();
        for (int c = 0; c < h.nx; ++c)
            for (int j = h.ccut[c]; j < h.ccut[c + 1]; ++j)
                pl->h_info.push_back((c << 2) | (j == h.ccut[c] ? 1 : 0) | (j == h.ccut[c + 1] - 1 ? 2 : 0));
        g.rcut = (long long)pl->h_info.size();
        for (int v : h.rcut) pl->h_info.push_back(v);
        g.ccut = (long long)pl->h_info.size();
        for (int v : h.ccut) pl->h_info.push_back(v);
        const double L = 8.0 / h.alpha + pl->inv_tau;
        g.alpha = (float)h.alpha;
        g.inv_alpha = (float)(1.0 / h.alpha);
        g.invL = (float)(1.0 / L);
        g.a_keep = full ? 1.0f : (float)(1.0 - 1.0 / (L * p.tau));
        g.kL = (float)(1.0 / (h.alpha * L));
        g.dA = 8.0 / ((h.alpha * L) * (h.alpha * L));
        g.dB = -pl->inv_tau / ((h.alpha * L) * (h.alpha * L));
        pl->h_imgs.push_back(g);
        for (int ri = 0; ri < kRowChoices; ++ri)
            for (int i0 = 0; i0 < h.H; i0 += 4 << ri)
                for (int j0 = 0; j0 < h.W; j0 += kStreamCols) pl->h_tiles[ri].push_back(StreamTile{b, i0, j0, 0});
        for (int r = 0; r < h.ny; ++r)
            for (int c = 0; c < h.nx; ++c)
                pl->h_subs.push_back(SubTile{b, r, c, h.rcut[r], h.ccut[c], h.rcut[r + 1] - h.rcut[r],
                                             h.ccut[c + 1] - h.ccut[c], 0});
    }
    // full 128 x 128 subdomains first, then framed ones (smaller, with each short side on the image
    // boundary), then the rest: the fused schedule runs all three with the specialised full-tile
    // step (frame_kind)
    auto is_full = [&](const SubTile &st) { return frame_kind(pl, st) == 0; };
    auto is_framed = [&](const SubTile &st) { return frame_kind(pl, st) == 1; };
    std::stable_partition(pl->h_subs.begin(), pl->h_subs.end(),
                          [&](const SubTile &st) { return is_full(st) || is_framed(st); });
    std::stable_partition(pl->h_subs.begin(), pl->h_subs.end(), is_full);
    for (const SubTile &st : pl->h_subs) {
        pl->n_full += is_full(st);
        pl->n_framed += is_framed(st);
    }
    pl->adaptive = p.inner_tol > 0.0;
    if (pl->adaptive && p.inner == DTV_INNER_FISTA) pl->h_beta = fista_betas(p.n_inner);
    if (pl->adaptive && p.inner == DTV_INNER_CP2) {
        std::vector<double> tk, sk, th;
        cp2_steps(p, p.n_inner, tk, sk, th);
        for (int it = 0; it < p.n_inner; ++it) {
            const float v[5] = {(float)tk[it], (float)sk[it], (float)th[it], cp2_keep(p, tk[it]), cp2_anchor(p, tk[it])};
            pl->h_cp2tab.insert(pl->h_cp2tab.end(), v, v + 5);
        }
    }
    if (p.inner == DTV_INNER_FISTA) {
        pl->fused_ok = p.n_inner <= kMaxFusedInner || pl->adaptive;
        for (const SubTile &st : pl->h_subs)
            if (st.h > kFusedMax || st.w > kFusedMax) pl->fused_ok = false;
    } else {  // the fused primal-dual kernel takes 128 x 128 subdomains and framed ones
        pl->fused_ok = (p.n_inner <= kMaxFusedInner || pl->adaptive) && !pl->h_subs.empty() &&
                       pl->n_full + pl->n_framed == (int)pl->h_subs.size();
    }
    if (pl->adaptive && !pl->fused_ok) {
        delete pl;
        return fail(DTV_EINVAL, "inner_tol needs the fused schedule's subdomains: at most 128 x 128 (FISTA), or "
                                "128 x 128 or smaller with their short sides on the image boundary (CP2)");
    }
    if (p.inner == DTV_INNER_FISTA && pl->fused_ok && !pl->adaptive && pl->n_full == (int)pl->h_subs.size()) {
        // more full tiles than four rounds of the device: delay half the CUs by about the on-chip part
        // of a tile (c' and the steps: 1 us + 2.2 us per step, in 10 ns ticks; the best of a sweep of
        // 5 to 15 us at 8192 x 8192 with 5 steps)
        int dev = 0;
        const int cap = hipGetDevice(&dev) == hipSuccess ? fused_capacity(dev) : 0;
        if (cap > 0 && pl->n_full >= 4 * cap) {
            pl->stagger_blocks = (cap / 2) & ~7;
            pl->stagger_ticks = 100 + 220 * std::min(p.n_inner, kMaxFusedInner);
        }
    }
    if (p.schedule == DTV_SCHED_FUSED && !pl->fused_ok) {
        delete pl;
        return fail(DTV_EINVAL, "the fused schedule needs n_inner <= 64 and subdomains of at most 128 x 128 (FISTA) "
                                "or of 128 x 128, smaller only with their short sides on the image boundary (CP2)");
    }
    {
        // persistent: full subdomains (fixed-count FISTA: any of at most 128 x 128; the primal-dual
        // kernel: also framed ones), no per-step host work; the primal-dual kernel and adaptive
        // stopping take every subdomain in one launch,
        // fixed-count FISTA runs the images in groups of launches, each group resident on the
        // device at once
        const int nsub = (int)pl->h_subs.size();
        const bool fista = p.inner == DTV_INNER_FISTA;
        const bool one_launch = !fista || pl->adaptive;
        pl->persist_ok = pl->fused_ok && nsub > 0 && p.diag_every == 0 &&
                         (fista || pl->n_full + pl->n_framed == nsub);
        int dev = 0;
        if (pl->persist_ok && hipGetDevice(&dev) == hipSuccess && persist_supported(dev)) {
            const int cap = fista ? persist_capacity(dev) : persist_cp2_capacity(dev);
            if (one_launch) {
                pl->persist_ok = nsub <= cap;
                if (pl->persist_ok) {
                    pl->p_subs = pl->h_subs;
                    pl->p_group = {0, nsub};
                }
            } else {
                pl->p_group = {0};
                int in_group = 0;
                for (int b = 0; b < n_images && pl->persist_ok; ++b) {
                    const int nt = pl->imgs[b].ny * pl->imgs[b].nx;
                    if (nt > cap) pl->persist_ok = false;
                    if (in_group + nt > cap) {
                        pl->p_group.push_back((int)pl->p_subs.size());
                        in_group = 0;
                    }
                    for (const SubTile &st : pl->h_subs)
                        if (st.img == b) pl->p_subs.push_back(st);
                    in_group += nt;
                }
                pl->p_group.push_back((int)pl->p_subs.size());
            }
        } else {
            pl->persist_ok = false;
        }
        if (!pl->persist_ok) {
            pl->p_subs.clear();
            pl->p_group.clear();
        }
    }
    if (p.schedule == DTV_SCHED_PERSIST && !pl->persist_ok) {
        delete pl;
        return fail(DTV_EINVAL, "the persistent schedule needs n_inner <= 64 (or inner_tol), every subdomain 128 x "
                                "128 (fixed-count FISTA: or smaller with its short sides on the image boundary), "
                                "each image's subdomains resident on the device at once (primal-dual or inner_tol: "
                                "all of them) and diag_every = 0");
    }

    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1), 256);
        return o;
    };
    pl->off_imgs = take(sizeof(ImgDev) * pl->h_imgs.size());
    pl->off_info = take(sizeof(int) * pl->h_info.size());
    for (int ri = 0; ri < kRowChoices; ++ri) pl->off_tiles[ri] = take(sizeof(StreamTile) * pl->h_tiles[ri].size());
    pl->off_subs = take(sizeof(SubTile) * pl->h_subs.size());
    pl->off_psubs = take(sizeof(SubTile) * std::max<size_t>(1, pl->p_subs.size()));
    // the persistent schedule updates p~, u and lambda in place: a plan that runs only that schedule
    // needs no rotation buffers, no second u and no second lambda state
    // (a plan that keeps checkpoints recomputes its outer steps with the other kernels in reverse mode)
    const bool persist_only = p.schedule == DTV_SCHED_PERSIST && !p.save_for_backward;
    pl->buf_bytes = persist_only ? 0 : sizeof(float) * (size_t)(pl->tot_p1 + pl->tot_p2);
    pl->spl = !persist_only && p.n_inner >= 2
                  ? std::min(p.steps_per_launch == 0 ? kDefaultStepsPerLaunch : p.steps_per_launch, p.n_inner)
                  : 1;
    // the multi-step kernel addresses a row by 32-bit byte offsets (at most 4 (W + nx) along a row
    // and 4 nx H in the vertical multipliers); an image beyond that runs one step per launch, which
    // gives the same result
    for (const ImgHost &h : pl->imgs)
        if (4.0 * std::max((double)h.W + h.nx, (double)h.nx * h.H) >= 2147483648.0) pl->spl = 1;
    if (pl->spl > 1) {
        // work lists of the multi-step launches an outer step makes
        for (int S : cp2_launch_steps(p.n_inner, pl->spl)) {
            if (S < 2 || !pl->h_mtiles[S - 2][0].empty()) continue;
            for (int b = 0; b < n_images; ++b) {
                const ImgHost &h = pl->imgs[b];
                for (int ri = 0; ri < kRowChoices; ++ri)
                    for (int i0 = 0; i0 < h.H; i0 += 4 << ri)
                        for (int j0 = 0; j0 < h.W; j0 += multi_cols(S))
                            pl->h_mtiles[S - 2][ri].push_back(StreamTile{b, i0, j0, 0});
            }
        }
    }
    for (int S = 2; S <= kMaxMultiSteps; ++S)
        for (int ri = 0; ri < kRowChoices; ++ri)
            pl->off_mtiles[S - 2][ri] = take(sizeof(StreamTile) * pl->h_mtiles[S - 2][ri].size());
    for (int k = 0; k < 4; ++k) pl->off_buf[k] = take(pl->buf_size(k));
    pl->off_u2 = take(p.inner == DTV_INNER_CP2 && !persist_only ? sizeof(float) * (size_t)pl->tot_px : 0);
    pl->diag_nblk = diag_blocks_per_image(pl->maxH, pl->maxW);
    pl->off_part = take(sizeof(double) * 6 * (size_t)pl->diag_nblk * n_images);
    pl->off_dout = take(sizeof(double) * 6 * (size_t)n_images);
    pl->off_xch = take(pl->persist_ok ? sizeof(unsigned long long) * 2 * (size_t)pl->tot_lam : 0);
    pl->off_sync = take(2 * sizeof(unsigned));
    pl->off_lamw = take(persist_only ? 0 : sizeof(float) * (size_t)pl->tot_lam);
    pl->off_beta = take(sizeof(float) * pl->h_beta.size());
    pl->off_counts = take(pl->adaptive ? sizeof(int) * 2 * pl->h_subs.size() : 0);
    pl->off_cp2tab = take(sizeof(float) * pl->h_cp2tab.size());
    if (p.save_for_backward) {
        const size_t E = (size_t)(pl->tot_p1 + pl->tot_p2);
        pl->state_floats = E + (size_t)pl->tot_lam;
        // with keep_records the state before every outer step is a checkpoint (and no segment is
        // recomputed)
        const int C = p.keep_records ? 1 : p.ckpt_every;
        pl->nseg = (p.n_outer + C - 1) / C;
        const int segmax = std::min(C, std::max(p.n_outer, 1));
        pl->off_ckpt = take(sizeof(float) * pl->state_floats * (size_t)(pl->nseg + 1));
        // a segment's states before each of its steps and after its last one
        pl->off_seg = take(p.keep_records ? 0 : sizeof(float) * pl->state_floats * (size_t)(segmax + 1));
        const size_t nsub = pl->h_subs.size();
        pl->fbwd = pl->fused_ok && pl->n_full == (int)nsub && fused_record_supported(p.n_inner) &&
                   fused_bwd_supported(p.n_inner);
        if (p.keep_records && !pl->fbwd) {
            delete pl;
            return fail(DTV_EINVAL, "keep_records needs the on-chip reverse: every subdomain 128 x 128 and n_inner "
                                    "1 .. 8 or 10");
        }
        if (p.keep_records) {
            // the records of every outer step, written by the forward solve
            pl->rec_step = sizeof(float4) * (size_t)p.n_inner * nsub * kRecGroups * kRecThreads;
            pl->off_frec = take(pl->rec_step * (size_t)std::max(p.n_outer, 1));
            pl->off_gsub = take(sizeof(double) * nsub);
        } else if (pl->fbwd) {
            // the records of a whole segment when they fit the budget (the segment's states are then
            // recomputed by the recording launches themselves), else of one outer step
            pl->rec_step = sizeof(float4) * (size_t)p.n_inner * nsub * kRecGroups * kRecThreads;
            pl->seg_rec = (size_t)segmax * pl->rec_step <= kSegRecordBytes;
            pl->off_frec = take(pl->rec_step * (size_t)(pl->seg_rec ? segmax : 1));
            pl->off_gsub = take(sizeof(double) * nsub);
        } else {
            pl->off_xrec = take(sizeof(float) * E * (size_t)p.n_inner);
            pl->off_zrec = take(sizeof(float) * E * (size_t)p.n_inner);
        }
        // the persistent reverse takes the ranges whose records are all kept (a checkpoint segment's,
        // or the whole solve's with keep_records) when every subdomain is resident at once
        if (pl->fbwd && (p.keep_records || pl->seg_rec) && p.reverse_schedule != DTV_SCHED_FUSED) {
            int dev = 0;
            pl->pbwd = hipGetDevice(&dev) == hipSuccess && persist_supported(dev) &&
                       (int)nsub <= persist_bwd_capacity(dev, p.n_inner);
        }
        if (p.reverse_schedule == DTV_SCHED_PERSIST && !pl->pbwd) {
            delete pl;
            return fail(DTV_EINVAL, "reverse_schedule persistent needs the on-chip reverse with the records of a "
                                    "range kept (every subdomain 128 x 128, all resident at once)");
        }
        pl->off_bxch = take(pl->pbwd ? sizeof(unsigned long long) * 2 * (size_t)pl->tot_lam : 0);
        pl->off_lam1 = take(sizeof(float) * (size_t)pl->tot_lam);
        pl->off_xb = take(sizeof(float) * E * 3);
        pl->off_hb = take(sizeof(float) * E);
        pl->off_pb = take(sizeof(float) * E);
        pl->off_lb = take(sizeof(float) * (size_t)pl->tot_lam);
        pl->off_galpha = take(sizeof(double) * pl->h_tiles[0].size());  // the longest list (4-row strips)
    }
    pl->ws_bytes = off;
    if (p.schedule != DTV_SCHED_AUTO)
        pl->schedule = p.schedule;
    else if (p.keep_records)  // only the fused kernel records its steps
        pl->schedule = DTV_SCHED_FUSED;
    else
        pl->schedule = pl->persist_ok ? DTV_SCHED_PERSIST : pl->fused_ok ? DTV_SCHED_FUSED : DTV_SCHED_STREAM;
    pl->rows = p.rows ? p.rows : 16;
    // explicit choices are final; otherwise an earlier plan of the same shape may have measured one
    if (candidates(pl).size() <= 1) {
        pl->tuned = true;
        pl->choice_source = p.schedule != DTV_SCHED_AUTO || p.rows != 0 ? 3 : 0;
    } else {
        pl->key = shape_key(pl);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(pl->key);
        // a cached choice is taken only where this plan admits it (the key covers what decides that)
        bool admitted = false;
        if (it != g_tune_cache.end())
            for (const Choice &ch : candidates(pl))
                if (ch.schedule == it->second.schedule && (ch.schedule != DTV_SCHED_STREAM || ch.rows == it->second.rows ||
                                                           p.rows == 0))
                    admitted = true;
        if (it != g_tune_cache.end() && admitted) {
            pl->schedule = it->second.schedule;
            pl->rows = it->second.rows;
            pl->tuned = true;
            pl->choice_source = 2;
        }
    }
    *out = pl;
    g_err.clear();
    return DTV_OK;
}

extern "C" int dtv_dd_layout(const dtv_dd_plan *pl, int32_t image, dtv_layout *out)
{
    if (!pl || !out) return fail(DTV_EINVAL, "null argument");
    if (image == -1) {
        dtv_layout L{};
        L.px_off = pl->tot_px;
        L.p1_off = pl->tot_p1;
        L.p2_off = pl->tot_p2;
        L.lam_off = pl->tot_lam;
        *out = L;
        return DTV_OK;
    }
    if (image < 0 || image >= pl->n) return fail(DTV_EINVAL, "image index out of range");
    *out = pl->imgs[image].L;
    return DTV_OK;
}

extern "C" int dtv_dd_workspace_bytes(const dtv_dd_plan *pl, size_t *bytes)
{
    if (!pl || !bytes) return fail(DTV_EINVAL, "null argument");
    *bytes = pl->ws_bytes;
    return DTV_OK;
}

static std::vector<float> fista_betas(int K);

extern "C" int dtv_dd_bind_workspace(dtv_dd_plan *pl, void *d_ws, size_t bytes)
{
    if (!pl || !d_ws) return fail(DTV_EINVAL, "null argument");
    if (bytes < pl->ws_bytes) return fail(DTV_ENOWS, "workspace too small");
    if (((uintptr_t)d_ws & 255) != 0) return fail(DTV_EINVAL, "workspace must be 256-byte aligned");
    char *ws = (char *)d_ws;
    HIP_TRY(hipMemcpy(ws + pl->off_imgs, pl->h_imgs.data(), sizeof(ImgDev) * pl->h_imgs.size(), hipMemcpyHostToDevice),
            "upload image descriptors");
    HIP_TRY(hipMemcpy(ws + pl->off_info, pl->h_info.data(), sizeof(int) * pl->h_info.size(), hipMemcpyHostToDevice),
            "upload info words");
    if (!pl->h_beta.empty())
        HIP_TRY(hipMemcpy(ws + pl->off_beta, pl->h_beta.data(), sizeof(float) * pl->h_beta.size(), hipMemcpyHostToDevice),
                "upload momentum table");
    if (!pl->h_cp2tab.empty())
        HIP_TRY(hipMemcpy(ws + pl->off_cp2tab, pl->h_cp2tab.data(), sizeof(float) * pl->h_cp2tab.size(),
                          hipMemcpyHostToDevice),
                "upload primal-dual step table");
    for (int ri = 0; ri < kRowChoices; ++ri)
        HIP_TRY(hipMemcpy(ws + pl->off_tiles[ri], pl->h_tiles[ri].data(), sizeof(StreamTile) * pl->h_tiles[ri].size(),
                          hipMemcpyHostToDevice),
                "upload work list");
    for (int S = 2; S <= kMaxMultiSteps; ++S)
        for (int ri = 0; ri < kRowChoices; ++ri)
            if (!pl->h_mtiles[S - 2][ri].empty())
                HIP_TRY(hipMemcpy(ws + pl->off_mtiles[S - 2][ri], pl->h_mtiles[S - 2][ri].data(),
                                  sizeof(StreamTile) * pl->h_mtiles[S - 2][ri].size(), hipMemcpyHostToDevice),
                        "upload work list");
    HIP_TRY(hipMemcpy(ws + pl->off_subs, pl->h_subs.data(), sizeof(SubTile) * pl->h_subs.size(), hipMemcpyHostToDevice),
            "upload subdomain list");
    if (!pl->p_subs.empty())
        HIP_TRY(hipMemcpy(ws + pl->off_psubs, pl->p_subs.data(), sizeof(SubTile) * pl->p_subs.size(),
                          hipMemcpyHostToDevice),
                "upload subdomain groups");
    // rotation buffers start at zero so that their boundary (non-dof) edges are 0
    for (int k = 0; k < 4; ++k)
        if (pl->buf_size(k)) HIP_TRY(hipMemset(ws + pl->off_buf[k], 0, pl->buf_size(k)), "clear buffers");
    // reverse-mode buffers: the step kernels write dof edges only, so the
    // boundary entries of every edge buffer must start (and stay) at zero
    if (pl->prm.save_for_backward)
        HIP_TRY(hipMemset(ws + pl->off_ckpt, 0, pl->ws_bytes - pl->off_ckpt), "clear reverse-mode buffers");
    if (!pl->h_diag) HIP_TRY(hipHostMalloc((void **)&pl->h_diag, sizeof(double) * 6 * pl->n), "pinned diag buffer");
    pl->ws = ws;
    return DTV_OK;
}

extern "C" int dtv_dd_schedule(const dtv_dd_plan *pl, int32_t *schedule)
{
    if (!pl || !schedule) return fail(DTV_EINVAL, "null argument");
    *schedule = pl->schedule;
    return DTV_OK;
}

// ---------------------------------------------------------------------------
// diagnostics

static int run_diag(dtv_dd_plan *pl, const float *f, const uint8_t *mask, const float *u, const float *p1,
                    const float *p2, hipStream_t s, double *rows /* n x 4 */, bool *nonfinite)
{
    HIP_TRY(launch_diag(pl->d_imgs(), pl->n, pl->maxH, pl->maxW, pl->d_info(), p1, p2, f, u, mask,
                        pl->prm.fidelity, pl->prm.cv_c1, pl->prm.cv_c2, pl->partials(), pl->diag_nblk, pl->dout(), s),
            "diagnostics kernels");
    HIP_TRY(hipMemcpyAsync(pl->h_diag, pl->dout(), sizeof(double) * 6 * pl->n, hipMemcpyDeviceToHost, s),
            "diagnostics copy");
    HIP_TRY(hipStreamSynchronize(s), "diagnostics sync");
    const bool dual_ok = pl->prm.fidelity != DTV_L1 && !pl->prm.has_mask;
    const bool cv = pl->prm.fidelity == DTV_CV;
    *nonfinite = false;
    for (int b = 0; b < pl->n; ++b) {
        const double *q = pl->h_diag + 6 * b;
        const double alpha = pl->imgs[b].alpha;
        const double J = alpha * q[0] + q[1];
        const double D = !dual_ok ? NAN : (cv ? q[2] : -q[2] - q[3] / (2.0 * alpha));
        rows[4 * b + 0] = J;
        rows[4 * b + 1] = D;
        rows[4 * b + 2] = J - D;
        rows[4 * b + 3] = std::sqrt(q[4]);
        if (q[5] != 0.0 || !std::isfinite(J) || !std::isfinite(q[4])) *nonfinite = true;
    }
    return DTV_OK;
}

extern "C" int dtv_dd_diagnostics(dtv_dd_plan *pl, const float *d_f, const uint8_t *d_mask, const float *d_u,
                                  const float *d_p1, const float *d_p2, double *h_out, void *stream)
{
    if (!pl || !d_f || !d_u || !d_p1 || !d_p2 || !h_out) return fail(DTV_EINVAL, "null argument");
    if (pl->prm.has_mask && !d_mask) return fail(DTV_EINVAL, "mask expected");
    if (!pl->ws) return fail(DTV_ENOWS, "no workspace bound");
    bool nf = false;
    int rc = run_diag(pl, d_f, pl->prm.has_mask ? d_mask : nullptr, d_u, d_p1, d_p2, (hipStream_t)stream, h_out, &nf);
    if (rc != DTV_OK) return rc;
    return nf ? fail(DTV_ENONFINITE, "non-finite value in the diagnostics") : DTV_OK;
}

// ---------------------------------------------------------------------------
// solve

namespace {

struct EdgeBuf {
    float *p1, *p2;
};

// inner-step timing: start / stop events stamped by each launch of the
// dominant kernel
struct Timer {
    dtv_dd_plan *pl;
    hipStream_t s;
    size_t used = 0;
    bool on;
    hipEvent_t e0 = nullptr, e1 = nullptr;  // events for the next launch (null when off)
    int begin()
    {
        e0 = e1 = nullptr;
        if (!on) return DTV_OK;
        while (pl->events.size() < used + 2) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e), "event create");
            pl->events.push_back(e);
        }
        e0 = pl->events[used];
        e1 = pl->events[used + 1];
        return DTV_OK;
    }
    int end()
    {
        if (on) used += 2;
        return DTV_OK;
    }
    int collect()
    {
        if (!on) return DTV_OK;
        HIP_TRY(hipStreamSynchronize(s), "timing sync");
        double tot = 0.0;
        for (size_t k = 0; k < used; k += 2) {
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, pl->events[k], pl->events[k + 1]), "event elapsed");
            tot += ms;
        }
        pl->t_ms = used ? tot / (double)(used / 2) : 0.0;
        pl->t_count = (int64_t)(used / 2);
        return DTV_OK;
    }
};

}  // namespace

static std::vector<float> fista_betas(int K);

// next rotation state of the edge buffers after one outer step (see outer_step)
static int next_base(int sched, bool cp2, int K, int base, int spl)
{
    if (sched == DTV_SCHED_PERSIST) return base;
    if (sched == DTV_SCHED_FUSED) return base == 0 ? 1 : 0;  // the fused kernels read one buffer and write the other
    if (!cp2) {
        if (spl > 1) return fista_stream_plan(K, spl, base).back().id;
        int rot[3] = {base, 0, 0}, q = 1;
        for (int k = 0; k < 3; ++k)
            if (k != base) rot[q++] = k;
        return rot[K % 3];
    }
    // primal-dual: the buffer the last launch of the outer step writes x_K to (cp2_stream_plan)
    return cp2_stream_plan(K, spl, base, spl > 1 ? 5 : 4).back().id;
}

// launches of one streaming primal-dual outer step (each swaps the two u buffers)
static int cp2_launches(int K, int spl) { return (int)cp2_launch_steps(K, spl).size(); }

// Arguments every solve entry point checks before anything is enqueued.
static int check_solve_args(const dtv_dd_plan *pl, const float *d_f, const uint8_t *d_mask, const float *d_u,
                            const float *d_p1, const float *d_p2, const float *d_lambda)
{
    if (!pl || !d_f || !d_u || !d_p1 || !d_p2) return fail(DTV_EINVAL, "null argument");
    if (!d_lambda && pl->tot_lam > 0) return fail(DTV_EINVAL, "null argument (lambda)");
    if (pl->prm.has_mask && !d_mask) return fail(DTV_EINVAL, "mask expected (has_mask = 1)");
    return DTV_OK;
}

// The solve, on the workspace pl->ws.  noalloc: the outer steps are enqueued eagerly (no graph is
// captured), the autotuner does not run (the plan's current choice is used) and nothing waits on
// the host; the caller has checked that no per-step host work (diagnostics, checkpoints, kernel
// timing) is asked for.
static int solve_impl(dtv_dd_plan *pl, const float *d_f, const uint8_t *d_mask, float *d_u, float *d_p1,
                      float *d_p2, float *d_lambda, double *h_stats, int32_t *n_rows, void *stream, bool noalloc)
{
    const dtv_dd_params &P = pl->prm;
    hipStream_t s = (hipStream_t)stream;
    pl->run_ws = pl->ws;
    pl->ran_persist = false;
    const uint8_t *mask = P.has_mask ? d_mask : nullptr;
    const bool cp2 = P.inner == DTV_INNER_CP2;
    const int K = P.n_inner;

    if (!P.warm_start) {
        HIP_TRY(launch_fill_zero(d_p1, sizeof(float) * (size_t)pl->tot_p1, s), "clear p1");
        HIP_TRY(launch_fill_zero(d_p2, sizeof(float) * (size_t)pl->tot_p2, s), "clear p2");
        if (pl->tot_lam > 0) HIP_TRY(launch_fill_zero(d_lambda, sizeof(float) * (size_t)pl->tot_lam, s), "clear lambda");
        if (cp2) HIP_TRY(hipMemcpyAsync(d_u, d_f, sizeof(float) * (size_t)pl->tot_px, hipMemcpyDeviceToDevice, s), "u = f");
    }
    HIP_TRY(launch_zero_boundary(pl->d_imgs(), pl->n, pl->maxH, pl->maxW, d_p1, d_p2, s), "zero boundary");

    // step parameters, computed in double precision on the host
    const std::vector<float> beta = fista_betas(K);  // FISTA momentum of step k (1-based); 0 for k = 1, 2
    std::vector<double> tk, sk, th;
    cp2_steps(P, K, tk, sk, th);

    // edge buffers: 0 = the caller's p~, 1..3 = workspace
    EdgeBuf bufs[5] = {{d_p1, d_p2}, {pl->buf1(0), pl->buf2(0)}, {pl->buf1(1), pl->buf2(1)}, {pl->buf1(2), pl->buf2(2)},
                       {pl->buf1(3), pl->buf2(3)}};
    int base = 0;
    float *u_cur = d_u;       // CP2: current u buffer (d_u or the workspace copy)
    float *lam_cur = d_lambda;  // current lambda state (the fused schedule alternates with the workspace copy)
    auto lam_other = [&]() { return lam_cur == d_lambda ? pl->lamw() : d_lambda; };
    Timer tm{pl, s, 0, P.time_kernels != 0};
    const int rows_cap = P.diag_every > 0 ? P.n_outer / P.diag_every + 1 : 0;
    int nrow = 0;
    bool nonfinite = false, stop = false;
    std::vector<double> drow(4 * pl->n);

    FusedArgs fa{};
    fa.imgs = pl->d_imgs();
    fa.subs = pl->d_subs();
    fa.f = d_f;
    fa.sigma = (float)P.sigma;
    fa.tau = (float)P.tau;
    fa.inv_tau = (float)pl->inv_tau;
    fa.n_inner = std::min(K, kMaxFusedInner);
    fa.stagger_blocks = pl->stagger_blocks;
    fa.stagger_ticks = pl->stagger_ticks;
    for (int k = 1; k <= fa.n_inner; ++k) fa.beta[k] = beta[k];
    if (pl->adaptive) {
        fa.n_inner = K;
        fa.tol2 = P.inner_tol * P.inner_tol;
        fa.beta_dev = pl->beta_tab();
        fa.counts = pl->counts();
        HIP_TRY(launch_fill_zero(pl->counts(), sizeof(int) * 2 * pl->h_subs.size(), s), "clear step counts");
    }
    int stop_at = P.n_outer;

    auto emit_stats = [&](int step, const float *u, const EdgeBuf &b) -> int {
        bool nf = false;
        int rc = run_diag(pl, d_f, mask, u, b.p1, b.p2, s, drow.data(), &nf);
        if (rc != DTV_OK) return rc;
        nonfinite = nonfinite || nf;
        if (h_stats && nrow < rows_cap)
            for (int img = 0; img < pl->n; ++img) {
                double *r = h_stats + 5 * ((size_t)img * rows_cap + nrow);
                r[0] = step;
                for (int q = 0; q < 4; ++q) r[1 + q] = drow[4 * img + q];
            }
        nrow++;
        return DTV_OK;
    };

    auto save_state = [&](int slot, const EdgeBuf &b) -> int {
        float *dst = pl->ckpt(slot);
        HIP_TRY(hipMemcpyAsync(dst, b.p1, sizeof(float) * (size_t)pl->tot_p1, hipMemcpyDeviceToDevice, s), "checkpoint");
        HIP_TRY(hipMemcpyAsync(dst + pl->tot_p1, b.p2, sizeof(float) * (size_t)pl->tot_p2, hipMemcpyDeviceToDevice, s),
                "checkpoint");
        if (pl->tot_lam > 0)
            HIP_TRY(hipMemcpyAsync(dst + pl->edges(), lam_cur, sizeof(float) * (size_t)pl->tot_lam,
                                   hipMemcpyDeviceToDevice, s),
                    "checkpoint");
        return DTV_OK;
    };
    // arguments of the fused and persistent primal-dual kernels (state pointers: the current buffers)
    auto cp2_args = [&]() {
        FusedCp2Args ca{};
        ca.imgs = pl->d_imgs();
        ca.subs = pl->d_subs();
        ca.p1 = bufs[base].p1;
        ca.p2 = bufs[base].p2;
        ca.out1 = ca.p1;  // in place (the persistent kernel); the fused step sets its own outputs
        ca.out2 = ca.p2;
        ca.lam = lam_cur;
        ca.sigma = (float)P.sigma;
        ca.f = d_f;
        ca.mask = mask;
        ca.u = u_cur;
        ca.tau = (float)P.tau;
        ca.fidelity = P.fidelity;
        ca.cv_c1 = (float)P.cv_c1;
        ca.cv_c2 = (float)P.cv_c2;
        ca.n_inner = std::min(K, kMaxFusedInner);
        for (int it = 0; it < ca.n_inner; ++it) {
            ca.tk[it] = (float)tk[it];
            ca.sk[it] = (float)sk[it];
            ca.th[it] = (float)th[it];
            ca.ck[it] = cp2_keep(P, tk[it]);
            ca.ca[it] = cp2_anchor(P, tk[it]);
        }
        if (pl->adaptive) {  // the cap may exceed the argument tables: the scalars come from the workspace
            ca.n_inner = K;
            ca.tol2 = P.inner_tol * P.inner_tol;
            ca.tab = pl->cp2_tab();
            ca.counts = pl->counts();
        }
        return ca;
    };
    pl->saved = false;
    const bool host_work = P.diag_every > 0 || P.save_for_backward || P.time_kernels;

    // One outer step n (a1 + a2 + a3) of a per-step schedule, enqueued on q.
    // With host work: the checkpoint before it, the diagnostics after it.
    auto outer_step = [&](int n, int sched, int rows, hipStream_t q, bool with_host) -> int {
        if (with_host && P.save_for_backward && n % P.ckpt_every == 0) {
            int rc = save_state(n / P.ckpt_every, bufs[base]);
            if (rc != DTV_OK) return rc;
        }
        // (a1) multipliers from the extrapolated interface jump: inside the fused kernels, else a launch
        if (sched != DTV_SCHED_FUSED)
            HIP_TRY(launch_lambda(pl->d_imgs(), pl->n, pl->max_nlam, pl->d_info(), bufs[base].p1, bufs[base].p2,
                                  lam_cur, (float)P.sigma, q),
                    "lambda update");
        // (a2)+(a3) local solves; the anchor phat is formed on the fly from p~^n and lambda
        if (sched == DTV_SCHED_FUSED && cp2) {
            const int out = next_base(sched, cp2, K, base, pl->spl);
            FusedCp2Args ca = cp2_args();
            ca.out1 = bufs[out].p1;
            ca.out2 = bufs[out].p2;
            ca.lam_out = lam_other();
            ca.frames = pl->n_full < (int)pl->h_subs.size();
            int rc = with_host ? tm.begin() : DTV_OK;
            if (rc != DTV_OK) return rc;
            HIP_TRY(launch_fused_cp2(ca, (int)pl->h_subs.size(), q, with_host ? tm.e0 : nullptr,
                                     with_host ? tm.e1 : nullptr),
                    "fused CP2");
            rc = with_host ? tm.end() : DTV_OK;
            if (rc != DTV_OK) return rc;
            base = out;
            lam_cur = lam_other();
        } else if (sched == DTV_SCHED_FUSED) {
            const int out = next_base(sched, cp2, K, base, pl->spl);
            fa.base1 = bufs[base].p1; fa.base2 = bufs[base].p2;
            fa.out1 = bufs[out].p1; fa.out2 = bufs[out].p2;
            fa.lam = lam_cur;
            fa.lam_out = lam_other();
            int rc = with_host ? tm.begin() : DTV_OK;
            if (rc != DTV_OK) return rc;
            HIP_TRY(launch_fused_fista(fa, (int)pl->h_subs.size(), pl->n_full, pl->n_framed, q,
                                       with_host ? tm.e0 : nullptr,
                                       with_host ? tm.e1 : nullptr),
                    "fused FISTA");
            rc = with_host ? tm.end() : DTV_OK;
            if (rc != DTV_OK) return rc;
            base = out;
            lam_cur = lam_other();
        } else if (!cp2 && pl->spl > 1) {
            // launches of up to pl->spl steps (fista_stream_plan); c' in workspace buffer 3, formed
            // by the first launch and stored when launches follow it
            const std::vector<Cp2Launch> plan = fista_stream_plan(K, pl->spl, base);
            for (const Cp2Launch &l : plan) {
                const int mode = l.k0 == 1 ? kFistaFirst : (l.k0 == 2 ? kFistaPlain : kFistaMomentum);
                int rc = with_host ? tm.begin() : DTV_OK;
                if (rc != DTV_OK) return rc;
                if (l.steps >= 2) {  // steps k0 .. k0 + steps - 1 in one launch
                    FistaMultiArgs a{};
                    a.imgs = pl->d_imgs(); a.tiles = pl->d_mtiles(l.steps, rows); a.ntiles = pl->nmtiles(l.steps, rows);
                    a.info = pl->d_info();
                    a.xa1 = bufs[l.ia].p1; a.xa2 = bufs[l.ia].p2; a.xb1 = bufs[l.ib].p1; a.xb2 = bufs[l.ib].p2;
                    a.lam = lam_cur; a.f = d_f;
                    a.c1 = bufs[3].p1; a.c2 = bufs[3].p2;
                    const int ik = l.ic >= 0 ? l.ic : l.id;  // (not written when ic < 0)
                    a.outk1 = bufs[ik].p1; a.outk2 = bufs[ik].p2;
                    a.outn1 = bufs[l.id].p1; a.outn2 = bufs[l.id].p2;
                    for (int L = 0; L < l.steps; ++L) a.beta[L] = beta[l.k0 + L];
                    a.tau = (float)P.tau; a.inv_tau = (float)pl->inv_tau;
                    a.store_c = l.k0 == 1 && plan.size() > 1;
                    a.store_prev = l.ic >= 0;
                    HIP_TRY(launch_fista_multi(a, mode, rows, l.steps, q, with_host ? tm.e0 : nullptr,
                                               with_host ? tm.e1 : nullptr),
                            "FISTA multi-step launch");
                } else {
                    FistaStepArgs a{};
                    a.imgs = pl->d_imgs(); a.tiles = pl->d_tiles(rows); a.ntiles = pl->ntiles(rows); a.info = pl->d_info();
                    a.xa1 = bufs[l.ia].p1; a.xa2 = bufs[l.ia].p2; a.xb1 = bufs[l.ib].p1; a.xb2 = bufs[l.ib].p2;
                    a.lam = lam_cur; a.f = d_f;
                    a.c1 = bufs[3].p1; a.c2 = bufs[3].p2;
                    a.out1 = bufs[l.id].p1; a.out2 = bufs[l.id].p2;
                    a.beta = beta[l.k0]; a.tau = (float)P.tau; a.inv_tau = (float)pl->inv_tau;
                    HIP_TRY(launch_fista_step(a, mode, rows, q, with_host ? tm.e0 : nullptr, with_host ? tm.e1 : nullptr),
                            "FISTA step");
                }
                rc = with_host ? tm.end() : DTV_OK;
                if (rc != DTV_OK) return rc;
            }
            base = plan.back().id;
        } else if (!cp2) {
            // x_k lives in rot[k % 3]; c' in workspace buffer 3
            int rot[3] = {base, 0, 0}, r = 1;
            for (int k = 0; k < 3; ++k)
                if (k != base) rot[r++] = k;
            for (int k = 1; k <= K; ++k) {
                const int ia = rot[(k - 1) % 3], ib = rot[(k + 1) % 3], io = rot[k % 3];
                FistaStepArgs a{};
                a.imgs = pl->d_imgs(); a.tiles = pl->d_tiles(rows); a.ntiles = pl->ntiles(rows); a.info = pl->d_info();
                a.xa1 = bufs[ia].p1; a.xa2 = bufs[ia].p2; a.xb1 = bufs[ib].p1; a.xb2 = bufs[ib].p2;
                a.lam = lam_cur; a.f = d_f;
                a.c1 = bufs[3].p1; a.c2 = bufs[3].p2;
                a.out1 = bufs[io].p1; a.out2 = bufs[io].p2;
                a.beta = beta[k]; a.tau = (float)P.tau; a.inv_tau = (float)pl->inv_tau;
                const int mode = k == 1 ? kFistaFirst : (k == 2 ? kFistaPlain : kFistaMomentum);
                int rc = with_host ? tm.begin() : DTV_OK;
                if (rc != DTV_OK) return rc;
                HIP_TRY(launch_fista_step(a, mode, rows, q, with_host ? tm.e0 : nullptr, with_host ? tm.e1 : nullptr),
                        "FISTA step");
                rc = with_host ? tm.end() : DTV_OK;
                if (rc != DTV_OK) return rc;
            }
            base = rot[K % 3];
        } else {
            // launches of up to pl->spl steps (cp2_stream_plan); each reads x_(k-1) and x_(k-2) and
            // writes its last two iterates (one-step launches: x_k) to buffers other than those and the base
            const std::vector<Cp2Launch> plan = cp2_stream_plan(K, pl->spl, base, pl->spl > 1 ? 5 : 4);
            for (const Cp2Launch &l : plan) {
                const int it = l.k0 - 1;
                float *u_next = u_cur == d_u ? pl->u2() : d_u;
                int rc = with_host ? tm.begin() : DTV_OK;
                if (rc != DTV_OK) return rc;
                if (l.steps >= 2) {  // steps k0 .. k0 + steps - 1 in one launch
                    Cp2MultiArgs a{};
                    a.imgs = pl->d_imgs(); a.tiles = pl->d_mtiles(l.steps, rows); a.ntiles = pl->nmtiles(l.steps, rows);
                    a.info = pl->d_info();
                    a.xa1 = bufs[l.ia].p1; a.xa2 = bufs[l.ia].p2; a.xb1 = bufs[l.ib].p1; a.xb2 = bufs[l.ib].p2;
                    a.base1 = bufs[base].p1; a.base2 = bufs[base].p2; a.lam = lam_cur; a.f = d_f; a.mask = mask;
                    a.u_in = u_cur; a.u_out = u_next;
                    a.outk1 = bufs[l.ic].p1; a.outk2 = bufs[l.ic].p2;
                    a.outn1 = bufs[l.id].p1; a.outn2 = bufs[l.id].p2;
                    for (int L = 0; L < l.steps; ++L) {  // level L runs step k0 + L (index it + L)
                        a.theta[L] = it + L >= 1 ? (float)th[it + L - 1] : 0.0f;
                        a.sk[L] = (float)sk[it + L];
                        a.tk[L] = (float)tk[it + L];
                        a.ck[L] = cp2_keep(P, tk[it + L]);
                        a.ca[L] = cp2_anchor(P, tk[it + L]);
                    }
                    a.tau = (float)P.tau;
                    a.fidelity = P.fidelity;
                    a.cv_c1 = (float)P.cv_c1;
                    a.cv_c2 = (float)P.cv_c2;
                    a.store_prev = &l != &plan.back();  // the next outer step starts without extrapolation
                    HIP_TRY(launch_cp2_multi(a, it >= 1, rows, l.steps, q, with_host ? tm.e0 : nullptr,
                                             with_host ? tm.e1 : nullptr),
                            "CP2 multi-step launch");
                } else {
                    Cp2StepArgs a{};
                    a.imgs = pl->d_imgs(); a.tiles = pl->d_tiles(rows); a.ntiles = pl->ntiles(rows); a.info = pl->d_info();
                    a.xa1 = bufs[l.ia].p1; a.xa2 = bufs[l.ia].p2; a.xb1 = bufs[l.ib].p1; a.xb2 = bufs[l.ib].p2;
                    a.base1 = bufs[base].p1; a.base2 = bufs[base].p2; a.lam = lam_cur; a.f = d_f; a.mask = mask;
                    a.u_in = u_cur; a.u_out = u_next;
                    a.out1 = bufs[l.id].p1; a.out2 = bufs[l.id].p2;
                    a.theta_prev = it >= 1 ? (float)th[it - 1] : 0.0f;
                    a.sk = (float)sk[it]; a.tk = (float)tk[it]; a.tau = (float)P.tau;
                    a.c_keep = cp2_keep(P, tk[it]);
                    a.c_anchor = cp2_anchor(P, tk[it]);
                    a.fidelity = P.fidelity;
                    a.cv_c1 = (float)P.cv_c1;
                    a.cv_c2 = (float)P.cv_c2;
                    HIP_TRY(launch_cp2_step(a, it >= 1, rows, q, with_host ? tm.e0 : nullptr, with_host ? tm.e1 : nullptr),
                            "CP2 step");
                }
                rc = with_host ? tm.end() : DTV_OK;
                if (rc != DTV_OK) return rc;
                u_cur = u_next;
            }
            base = plan.back().id;
        }
        const bool last = n == P.n_outer - 1;
        if (with_host && P.diag_every > 0 && ((n + 1) % P.diag_every == 0 || last)) {
            const float *u = u_cur;
            if (!cp2) {
                HIP_TRY(launch_u_from_p(pl->d_imgs(), pl->n, pl->maxH, pl->maxW, pl->d_info(), bufs[base].p1,
                                        bufs[base].p2, d_f, d_u, s),
                        "u recovery");
                u = d_u;
            }
            int rc = emit_stats(n + 1, u, bufs[base]);
            if (rc != DTV_OK) return rc;
            if (P.gap_tol > 0.0 && drow[2] <= P.gap_tol * std::fabs(drow[0])) {
                stop = true;
                stop_at = n + 1;
            }
        }
        return DTV_OK;
    };

    // outer steps [n0, n0 + count) in one persistent launch; p~ and lambda updated in place
    const unsigned spin_limit = P.spin_limit > 0 ? (unsigned)P.spin_limit : kSpinLimitDefault;
    auto run_persist = [&](int count) -> int {
        unsigned *sync = pl->sync_words();
        HIP_TRY(launch_fill_zero(sync, 2 * sizeof(unsigned), s), "clear error flag");
        HIP_TRY(launch_fill_zero(pl->xch(), sizeof(unsigned long long) * 2 * (size_t)pl->tot_lam, s), "clear exchange");
        int rc = tm.begin();
        if (rc != DTV_OK) return rc;
        if (tm.e0) HIP_TRY(hipEventRecord(tm.e0, s), "event");
        if (cp2) {
            PersistCp2Args pc{};
            pc.ca = cp2_args();
            pc.lam_out = lam_cur;
            pc.xch = pl->xch();
            pc.xch_stride = pl->tot_lam;
            pc.err = (int *)sync;
            pc.n_outer = count;
            pc.sigma = (float)P.sigma;
            pc.spin_limit = spin_limit;
            pc.ca.frames = pl->n_full < (int)pl->h_subs.size();
            HIP_TRY(launch_persist_cp2(pc, (int)pl->h_subs.size(), s), "persistent primal-dual");
        } else {
            PersistArgs pa{};
            pa.fa = fa;
            pa.fa.base1 = pa.fa.out1 = bufs[base].p1;
            pa.fa.base2 = pa.fa.out2 = bufs[base].p2;
            pa.fa.lam = lam_cur;
            pa.lam_out = lam_cur;
            pa.xch = pl->xch();
            pa.xch_stride = pl->tot_lam;
            pa.err = (int *)sync;
            pa.n_outer = count;
            pa.sigma = (float)P.sigma;
            pa.spin_limit = spin_limit;
            // one cooperative launch per group of images; the groups share nothing
            for (size_t g = 0; g + 1 < pl->p_group.size(); ++g) {
                int frames = 0;  // the most general kind of subdomain in the group (frame_kind)
                for (int i = pl->p_group[g]; i < pl->p_group[g + 1]; ++i)
                    frames = std::max(frames, frame_kind(pl, pl->p_subs[i]));
                pa.fa.subs = pl->d_psubs() + pl->p_group[g];
                HIP_TRY(launch_persist_fista(pa, pl->p_group[g + 1] - pl->p_group[g], frames, s), "persistent FISTA");
            }
        }
        if (tm.e1) HIP_TRY(hipEventRecord(tm.e1, s), "event");
        rc = tm.end();
        if (rc != DTV_OK) return rc;
        // a wait that gave up leaves its flag in the workspace; dtv_dd_status reads it
        pl->ran_persist = true;
        return DTV_OK;
    };

    // keep_records: outer steps [n0, n1) with the recording fused kernel.  Step n reads its state
    // (p~^n and the lambda state) from checkpoint slot n and writes the next one to slot n + 1, its
    // records to frec(n); the state after step n1 - 1 is then copied to the current buffers.
    auto run_recorded = [&](int n0, int n1) -> int {
        const size_t E = pl->edges();
        if (n0 == 0) {
            int rc = save_state(0, bufs[base]);
            if (rc != DTV_OK) return rc;
        }
        for (int n = n0; n < n1; ++n) {
            float *st = pl->ckpt(n), *nx = pl->ckpt(n + 1);
            FusedArgs ra = fa;
            ra.base1 = st;
            ra.base2 = st + pl->tot_p1;
            ra.lam = st + E;
            ra.out1 = nx;
            ra.out2 = nx + pl->tot_p1;
            ra.lam_out = nx + E;
            ra.rec = pl->frec(n);
            int rc = tm.begin();
            if (rc != DTV_OK) return rc;
            HIP_TRY(launch_fused_fista(ra, (int)pl->h_subs.size(), pl->n_full, pl->n_framed, s, tm.e0, tm.e1),
                    "fused FISTA (recording)");
            rc = tm.end();
            if (rc != DTV_OK) return rc;
            if (P.diag_every > 0 && ((n + 1) % P.diag_every == 0 || n == P.n_outer - 1)) {
                HIP_TRY(launch_u_from_p(pl->d_imgs(), pl->n, pl->maxH, pl->maxW, pl->d_info(), nx, nx + pl->tot_p1,
                                        d_f, d_u, s),
                        "u recovery");
                rc = emit_stats(n + 1, d_u, EdgeBuf{nx, nx + pl->tot_p1});
                if (rc != DTV_OK) return rc;
            }
        }
        const float *fin = pl->ckpt(n1);
        HIP_TRY(hipMemcpyAsync(bufs[base].p1, fin, sizeof(float) * (size_t)pl->tot_p1, hipMemcpyDeviceToDevice, s),
                "state");
        HIP_TRY(hipMemcpyAsync(bufs[base].p2, fin + pl->tot_p1, sizeof(float) * (size_t)pl->tot_p2,
                               hipMemcpyDeviceToDevice, s),
                "state");
        if (pl->tot_lam > 0)
            HIP_TRY(hipMemcpyAsync(lam_cur, fin + E, sizeof(float) * (size_t)pl->tot_lam, hipMemcpyDeviceToDevice, s),
                    "state");
        return DTV_OK;
    };

    // Outer steps [n0, n1) with one schedule.  The per-step schedules replay a
    // captured cycle of outer steps (the rotation of the edge buffers returns
    // to its start after 1, 2 or 3 steps) when there is no host work per step.
    auto run_range = [&](int n0, int n1, int sched, int rows, bool graphs) -> int {
        if (n1 <= n0) return DTV_OK;
        if (P.keep_records) return run_recorded(n0, n1);
        if (sched == DTV_SCHED_PERSIST) {
            if (!P.save_for_backward) return run_persist(n1 - n0);
            // with checkpoints: one launch per segment of ckpt_every outer steps, the state saved before it
            const int C = P.ckpt_every;
            for (int m = n0; m < n1;) {
                const int next = std::min(n1, (m / C + 1) * C);
                int rc = m % C == 0 ? save_state(m / C, bufs[base]) : DTV_OK;
                if (rc == DTV_OK) rc = run_persist(next - m);
                if (rc != DTV_OK) return rc;
                m = next;
            }
            return DTV_OK;
        }
        int n = n0;
        if (graphs && !host_work && !P.no_graphs && n1 - n0 >= 4) {
            // the buffer state (base, which u buffer is current) after each step
            auto state = [&](int b, bool uf, bool lp) { return b * 4 + (uf ? 2 : 0) + (lp ? 1 : 0); };
            std::vector<int> seq;
            int b = base;
            bool uf = u_cur != d_u, lp = lam_cur != d_lambda;
            for (int i = 0; i < 8; ++i) {
                seq.push_back(state(b, uf, lp));
                b = next_base(sched, cp2, K, b, pl->spl);
                if (cp2 && sched != DTV_SCHED_FUSED && (cp2_launches(K, pl->spl) & 1)) uf = !uf;
                if (sched == DTV_SCHED_FUSED) lp = !lp;
            }
            int start = -1, period = 0;
            for (int i = 0; i < 4 && start < 0; ++i)
                for (int j = i + 1; j < 8; ++j)
                    if (seq[j] == seq[i]) {
                        start = i;
                        period = j - i;
                        break;
                    }
            if (start >= 0 && n1 - n0 - start >= 2 * period) {
                for (int i = 0; i < start; ++i, ++n) {
                    int rc = outer_step(n, sched, rows, s, false);
                    if (rc != DTV_OK) return rc;
                }
                const GraphKey key{sched, rows, base, u_cur != d_u, period, d_f, mask, d_u, d_p1, d_p2, lam_cur, pl->ws};
                if (!pl->gexec || !(pl->gkey == key)) {
                    if (pl->gexec) {
                        (void)hipGraphExecDestroy(pl->gexec);
                        pl->gexec = nullptr;
                    }
                    if (!pl->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking), "stream");
                    const int base0 = base;
                    float *u0 = u_cur, *l0 = lam_cur;
                    HIP_TRY(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal), "graph capture");
                    int rc = DTV_OK;
                    for (int i = 0; i < period && rc == DTV_OK; ++i) rc = outer_step(n + i, sched, rows, pl->cap_stream, false);
                    hipGraph_t g = nullptr;
                    const hipError_t ge = hipStreamEndCapture(pl->cap_stream, &g);
                    base = base0;  // the captured cycle returns to the same buffers
                    u_cur = u0;
                    lam_cur = l0;
                    if (rc != DTV_OK) {
                        if (g) (void)hipGraphDestroy(g);
                        return rc;
                    }
                    HIP_TRY(ge, "graph capture");
                    const hipError_t ie = hipGraphInstantiate(&pl->gexec, g, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(g);
                    HIP_TRY(ie, "graph instantiate");
                    pl->gkey = key;
                }
                const int reps = (n1 - n) / period;
                for (int r = 0; r < reps; ++r) HIP_TRY(hipGraphLaunch(pl->gexec, s), "graph launch");
                n += reps * period;
            }
        }
        for (; n < n1 && !stop; ++n) {
            int rc = outer_step(n, sched, rows, s, host_work);
            if (rc != DTV_OK) return rc;
        }
        return DTV_OK;
    };

    int n = 0;
    // ---- autotuner: the first solve of an untuned plan runs its first outer steps in timed chunks.
    // A per-step schedule costs its chunk time per step; the persistent launch has a fixed part (loading
    // and storing every tile) besides its per-step part, so it is timed over chunks of c and 2c steps
    // and priced as fixed + per-step * (the steps left), the way the rest of the solve would run it.
    if (!pl->tuned && !host_work && !noalloc && P.n_outer > 0) {
        const std::vector<Choice> cands = candidates(pl);
        const int nc = (int)cands.size();
        const int chunk = std::min(16, P.n_outer / (2 * (std::max(nc, 1) + 2)) - 1);
        if (nc > 1 && chunk >= 2) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            HIP_TRY(hipEventCreate(&e0), "event create");
            HIP_TRY(hipEventCreate(&e1), "event create");
            int rc = DTV_OK;
            auto time_range = [&](const Choice &ch, int count, double *ms_out) {
                if (hipEventRecord(e0, s) != hipSuccess) rc = fail(DTV_EHIP, "event record");
                if (rc == DTV_OK) rc = run_range(n, n + count, ch.schedule, ch.rows, false);
                if (rc == DTV_OK && hipEventRecord(e1, s) != hipSuccess) rc = fail(DTV_EHIP, "event record");
                float ms = 0.0f;
                if (rc == DTV_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    rc = fail(DTV_EHIP, "autotune timing");
                n += count;
                *ms_out = ms;
            };
            for (int c = 0; c < nc && rc == DTV_OK; ++c) {  // one untimed step each (first use of each kernel)
                rc = run_range(n, n + 1, cands[c].schedule, cands[c].rows, false);
                n += 1;
            }
            std::vector<double> fixed(nc, 0.0), per_step(nc, 0.0);
            for (int c = 0; c < nc && rc == DTV_OK; ++c) {
                double t1 = 0.0, t2 = 0.0;
                time_range(cands[c], chunk, &t1);
                per_step[c] = t1 / chunk;
                if (rc == DTV_OK && cands[c].schedule == DTV_SCHED_PERSIST) {
                    time_range(cands[c], 2 * chunk, &t2);
                    per_step[c] = std::max((t2 - t1) / chunk, 0.25 * t2 / (2 * chunk));
                    fixed[c] = std::max(t1 - per_step[c] * chunk, 0.0);
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            if (rc != DTV_OK) return rc;
            const double left = std::max(P.n_outer - n, 1);
            int bi = 0;
            for (int c = 1; c < nc; ++c)
                if (fixed[c] + per_step[c] * left < fixed[bi] + per_step[bi] * left) bi = c;
            pl->schedule = cands[bi].schedule;
            pl->rows = cands[bi].rows;
            pl->tuned = true;
            pl->choice_source = 1;
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_cache[pl->key] = cands[bi];
        }
    }
    {
        int rc = run_range(n, P.n_outer, pl->schedule, pl->rows, !noalloc);
        if (rc != DTV_OK) return rc;
    }

    if (P.save_for_backward) {
        // (keep_records: the recording steps wrote the last state to slot n_outer = nseg already)
        int rc = P.keep_records && P.n_outer > 0 ? DTV_OK : save_state(pl->nseg, bufs[base]);
        if (rc != DTV_OK) return rc;
        pl->saved = true;
        pl->saved_outer = P.n_outer;
    }
    if (lam_cur != d_lambda && pl->tot_lam > 0)
        HIP_TRY(hipMemcpyAsync(d_lambda, lam_cur, sizeof(float) * (size_t)pl->tot_lam, hipMemcpyDeviceToDevice, s),
                "copy lambda");
    if (base != 0) {
        HIP_TRY(hipMemcpyAsync(d_p1, bufs[base].p1, sizeof(float) * (size_t)pl->tot_p1, hipMemcpyDeviceToDevice, s), "copy p1");
        HIP_TRY(hipMemcpyAsync(d_p2, bufs[base].p2, sizeof(float) * (size_t)pl->tot_p2, hipMemcpyDeviceToDevice, s), "copy p2");
    }
    if (cp2) {
        if (u_cur != d_u)
            HIP_TRY(hipMemcpyAsync(d_u, u_cur, sizeof(float) * (size_t)pl->tot_px, hipMemcpyDeviceToDevice, s), "copy u");
    } else {
        HIP_TRY(launch_u_from_p(pl->d_imgs(), pl->n, pl->maxH, pl->maxW, pl->d_info(), d_p1, d_p2, d_f, d_u, s),
                "u recovery");
    }
    int rc = tm.collect();
    if (rc != DTV_OK) return rc;
    pl->last_outer = stop ? stop_at : P.n_outer;
    pl->solved = true;
    if (n_rows) *n_rows = nrow;
    if (nonfinite) return fail(DTV_ENONFINITE, "non-finite value in the diagnostics");
    return DTV_OK;
}

extern "C" int dtv_dd_solve(dtv_dd_plan *pl, const float *d_f, const uint8_t *d_mask, float *d_u, float *d_p1,
                            float *d_p2, float *d_lambda, double *h_stats, int32_t *n_rows, void *stream)
{
    int rc = check_solve_args(pl, d_f, d_mask, d_u, d_p1, d_p2, d_lambda);
    if (rc != DTV_OK) return rc;
    if (!pl->ws) return fail(DTV_ENOWS, "no workspace bound");
    return solve_impl(pl, d_f, d_mask, d_u, d_p1, d_p2, d_lambda, h_stats, n_rows, stream, false);
}

extern "C" int dtv_dd_status(dtv_dd_plan *pl, void *stream)
{
    if (!pl) return fail(DTV_EINVAL, "null argument");
    if (!pl->ran_persist || !pl->run_ws) return DTV_OK;
    hipStream_t s = (hipStream_t)stream;
    unsigned err = 0;
    HIP_TRY(hipMemcpyAsync(&err, pl->run_sync_words(), sizeof(unsigned), hipMemcpyDeviceToHost, s), "exchange status");
    HIP_TRY(hipStreamSynchronize(s), "exchange status");
    if (err) return fail(DTV_EHIP, "persistent schedule: a wait for a neighbouring subdomain timed out");
    return DTV_OK;
}

extern "C" int dtv_dd_inner_counts(dtv_dd_plan *pl, int32_t *h_counts, void *stream)
{
    if (!pl || !h_counts) return fail(DTV_EINVAL, "null argument");
    const size_t nsub = pl->h_subs.size();
    std::vector<int> dev(2 * nsub, 0);
    if (pl->solved && pl->adaptive) {
        hipStream_t s = (hipStream_t)stream;
        HIP_TRY(hipMemcpyAsync(dev.data(), pl->run_counts(), sizeof(int) * 2 * nsub, hipMemcpyDeviceToHost, s),
                "step counts");
        HIP_TRY(hipStreamSynchronize(s), "step counts");
    } else if (pl->solved) {
        for (size_t t = 0; t < nsub; ++t) {
            dev[2 * t] = pl->last_outer * pl->prm.n_inner;
            dev[2 * t + 1] = pl->last_outer > 0 ? pl->prm.n_inner : 0;
        }
    }
    // the work list holds the full subdomains first: put the counts back in grid order
    std::vector<int64_t> first(pl->n + 1, 0);
    for (int b = 0; b < pl->n; ++b) first[b + 1] = first[b] + (int64_t)pl->imgs[b].ny * pl->imgs[b].nx;
    for (size_t t = 0; t < nsub; ++t) {
        const SubTile &st = pl->h_subs[t];
        const int64_t g = first[st.img] + (int64_t)st.r * pl->imgs[st.img].nx + st.c;
        h_counts[2 * g] = dev[2 * t];
        h_counts[2 * g + 1] = dev[2 * t + 1];
    }
    return DTV_OK;
}

// FISTA momentum coefficients beta[k] of step k (0 for k = 1, 2)
static std::vector<float> fista_betas(int K)
{
    std::vector<float> beta(K + 1, 0.0f);
    std::vector<double> t(K + 2, 1.0);
    for (int m = 1; m <= K; ++m) t[m + 1] = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t[m] * t[m]));
    for (int k = 2; k <= K; ++k) beta[k] = (float)((t[k - 1] - 1.0) / t[k]);
    return beta;
}

// One outer step from a stored state (P1, P2, lambda state) with the
// streaming kernels: the multiplier update into lam1 and the n_inner FISTA
// steps into xrec(0..K-1), recording z_k into zrec when asked.
static int rec_outer(dtv_dd_plan *pl, const float *state, const float *d_f, bool record, const std::vector<float> &beta,
                     hipStream_t s)
{
    const dtv_dd_params &P = pl->prm;
    const float *p1 = state, *p2 = state + pl->tot_p1, *lam = state + pl->edges();
    const int K = P.n_inner, rows = pl->rows;
    if (pl->tot_lam > 0)
        HIP_TRY(hipMemcpyAsync(pl->lam1(), lam, sizeof(float) * (size_t)pl->tot_lam, hipMemcpyDeviceToDevice, s),
                "lambda copy");
    HIP_TRY(launch_lambda(pl->d_imgs(), pl->n, pl->max_nlam, pl->d_info(), p1, p2, pl->lam1(), (float)P.sigma, s),
            "lambda update");
    for (int k = 1; k <= K; ++k) {
        FistaStepArgs a{};
        a.imgs = pl->d_imgs(); a.tiles = pl->d_tiles(rows); a.ntiles = pl->ntiles(rows); a.info = pl->d_info();
        const float *xa = k == 1 ? state : pl->xrec(k - 2);
        const float *xbp = k >= 3 ? pl->xrec(k - 3) : state;
        a.xa1 = xa; a.xa2 = xa + pl->tot_p1;
        a.xb1 = xbp; a.xb2 = xbp + pl->tot_p1;
        a.lam = pl->lam1(); a.f = d_f;
        a.c1 = pl->buf1(2); a.c2 = pl->buf2(2);
        a.out1 = pl->xrec(k - 1); a.out2 = pl->xrec(k - 1) + pl->tot_p1;
        if (record) {
            a.z1 = pl->zrec(k - 1);
            a.z2 = pl->zrec(k - 1) + pl->tot_p1;
        }
        a.beta = beta[k]; a.tau = (float)P.tau; a.inv_tau = (float)pl->inv_tau;
        const int mode = k == 1 ? kFistaFirst : (k == 2 ? kFistaPlain : kFistaMomentum);
        HIP_TRY(launch_fista_step(a, mode, rows, s), "FISTA step (recompute)");
    }
    return DTV_OK;
}

// Reverse mode with the fused kernels (every subdomain 128 x 128): per outer
// step one recording forward launch and one on-chip reverse launch (the n_inner
// reverse steps), then the interface transpose.  pbar holds the adjoint of the
// final p~ (from the u recovery) on entry.
static int backward_fused(dtv_dd_plan *pl, const float *d_f, float *d_grad_f, float *d_grad_alpha,
                          const std::vector<float> &beta, hipStream_t s)
{
    const dtv_dd_params &P = pl->prm;
    const int K = P.n_inner, N = pl->saved_outer, C = P.ckpt_every, nsub = (int)pl->h_subs.size();
    const size_t E = pl->edges();
    HIP_TRY(hipMemsetAsync(pl->gsub(), 0, sizeof(double) * (size_t)nsub, s), "clear");
    FusedArgs fa{};
    fa.imgs = pl->d_imgs();
    fa.subs = pl->d_subs();
    fa.f = d_f;
    fa.sigma = (float)P.sigma;
    fa.tau = (float)P.tau;
    fa.inv_tau = (float)pl->inv_tau;
    fa.n_inner = K;
    for (int k = 1; k <= K; ++k) fa.beta[k] = beta[k];
    FusedBwdArgs ba{};
    ba.imgs = pl->d_imgs();
    ba.subs = pl->d_subs();
    ba.f = d_f;
    ba.pb1 = pl->pb();
    ba.pb2 = pl->pb() + pl->tot_p1;
    ba.hb1 = pl->hb();
    ba.hb2 = pl->hb() + pl->tot_p1;
    ba.gf = d_grad_f;
    ba.galpha = pl->gsub();
    ba.tau = (float)P.tau;
    ba.inv_tau = (float)pl->inv_tau;
    ba.n_inner = K;
    for (int k = 1; k <= K; ++k) ba.beta[k] = beta[k];
    // with time_kernels: a pair of events around every launch of the two kernels of a reverse step
    const bool timed = P.time_kernels != 0;
    size_t used[2] = {0, 0};
    auto events = [&](int which, hipEvent_t *e0, hipEvent_t *e1) -> int {
        *e0 = *e1 = nullptr;
        if (!timed) return DTV_OK;
        std::vector<hipEvent_t> &v = pl->bwd_events[which];
        while (v.size() < used[which] + 2) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e), "event create");
            v.push_back(e);
        }
        *e0 = v[used[which]];
        *e1 = v[used[which] + 1];
        used[which] += 2;
        return DTV_OK;
    };
    // one outer step of the fused forward from a state (p~, lambda state) to p~ out, lambda state out
    auto forward = [&](const float *st, float *p_out, float *lam_out, float4 *rec) -> int {
        fa.base1 = st;
        fa.base2 = st + pl->tot_p1;
        fa.lam = st + E;
        fa.out1 = p_out;
        fa.out2 = p_out + pl->tot_p1;
        fa.lam_out = lam_out;
        fa.rec = rec;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (rec) {
            int rc = events(1, &e0, &e1);
            if (rc != DTV_OK) return rc;
        }
        HIP_TRY(launch_fused_fista(fa, nsub, pl->n_full, pl->n_framed, s, e0, e1),
                rec ? "fused FISTA (recording)" : "fused FISTA");
        return DTV_OK;
    };
    // the reverse of an outer step from its state st, the lambda state after its multiplier update
    // (lam_next) and its records
    auto reverse = [&](const float *st, const float *lam_next, const float4 *rec) -> int {
        ba.x0_1 = st;
        ba.x0_2 = st + pl->tot_p1;
        ba.lam = lam_next;
        ba.rec = rec;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        int rc = events(0, &e0, &e1);
        if (rc != DTV_OK) return rc;
        HIP_TRY(launch_fused_bwd(ba, nsub, s, e0, e1), "fused reverse steps");
        HIP_TRY(launch_bwd_interface(pl->d_imgs(), pl->n, pl->max_nlam, pl->d_info(), pl->hb(), pl->hb() + pl->tot_p1,
                                     pl->pb(), pl->pb() + pl->tot_p1, pl->lb(), (float)P.tau, (float)P.sigma, s),
                "interface reverse");
        return DTV_OK;
    };
    // the persistent reverse of outer steps [0, m) of a range: the state before step q at
    // st0 + q state_floats, its records at rec0 + q rec_step
    const unsigned spin_limit = P.spin_limit > 0 ? (unsigned)P.spin_limit : kSpinLimitDefault;
    if (pl->pbwd) {
        HIP_TRY(launch_fill_zero(pl->sync_words(), 2 * sizeof(unsigned), s), "clear error flag");
        pl->ran_persist = true;
        pl->run_ws = pl->ws;
    }
    auto reverse_range = [&](const float *st0, const float4 *rec0, int m) -> int {
        if (m <= 0) return DTV_OK;
        PersistBwdArgs pa{};
        pa.b = ba;
        pa.st = st0;
        pa.st_stride = (long long)pl->state_floats;
        pa.p2_off = pl->tot_p1;
        pa.lam_off = (long long)E;
        pa.rec = rec0;
        pa.rec_outer = (long long)(pl->rec_step / sizeof(float4));
        pa.n_steps = m;
        pa.sigma = (float)P.sigma;
        pa.lamb = pl->lb();
        pa.xch = pl->bxch();
        pa.xch_stride = pl->tot_lam;
        pa.err = (int *)pl->sync_words();
        pa.spin_limit = spin_limit;
        HIP_TRY(launch_fill_zero(pl->bxch(), sizeof(unsigned long long) * 2 * (size_t)pl->tot_lam, s),
                "clear exchange");
        hipEvent_t e0 = nullptr, e1 = nullptr;
        int rc = events(0, &e0, &e1);
        if (rc != DTV_OK) return rc;
        if (e0) HIP_TRY(hipEventRecord(e0, s), "event");
        HIP_TRY(launch_persist_bwd(pa, nsub, s), "persistent reverse");
        if (e1) HIP_TRY(hipEventRecord(e1, s), "event");
        return DTV_OK;
    };
    // keep_records: the forward solve kept every state and every outer step's records
    if (P.keep_records && pl->pbwd) {
        int rc = reverse_range(pl->ckpt(0), pl->frec(0), N);
        if (rc != DTV_OK) return rc;
    }
    for (int n = P.keep_records && !pl->pbwd ? N - 1 : -1; n >= 0; --n) {
        int rc = reverse(pl->ckpt(n), pl->ckpt(n + 1) + E, pl->frec(n));
        if (rc != DTV_OK) return rc;
    }
    for (int sg = P.keep_records ? -1 : pl->nseg - 1; sg >= 0; --sg) {
        const int n0 = sg * C, n1 = std::min(N, n0 + C), m = n1 - n0;
        HIP_TRY(hipMemcpyAsync(pl->seg(0), pl->ckpt(sg), sizeof(float) * pl->state_floats, hipMemcpyDeviceToDevice, s),
                "restore checkpoint");
        if (pl->seg_rec) {
            // one recording launch per outer step recomputes the segment's states and keeps every record
            for (int q = 0; q < m; ++q) {
                int rc = forward(pl->seg(q), pl->seg(q + 1), pl->seg(q + 1) + E, pl->frec(q));
                if (rc != DTV_OK) return rc;
            }
            if (pl->pbwd) {
                int rc = reverse_range(pl->seg(0), pl->frec(0), m);
                if (rc != DTV_OK) return rc;
                continue;
            }
            for (int q = m - 1; q >= 0; --q) {
                int rc = reverse(pl->seg(q), pl->seg(q + 1) + E, pl->frec(q));
                if (rc != DTV_OK) return rc;
            }
            continue;
        }
        for (int q = 0; q + 1 < m; ++q) {  // the segment's states
            int rc = forward(pl->seg(q), pl->seg(q + 1), pl->seg(q + 1) + E, nullptr);
            if (rc != DTV_OK) return rc;
        }
        for (int q = m - 1; q >= 0; --q) {  // its outer steps in reverse, each recorded again
            int rc = forward(pl->seg(q), pl->buf1(0), pl->lam1(), pl->frec());
            if (rc != DTV_OK) return rc;
            rc = reverse(pl->seg(q), pl->lam1(), pl->frec());
            if (rc != DTV_OK) return rc;
        }
    }
    const int rows = pl->rows;
    HIP_TRY(launch_alpha_reduce2(pl->d_tiles(rows), pl->ntiles(rows), pl->galpha(), pl->d_subs(), nsub, pl->gsub(),
                                 pl->n, d_grad_alpha, s),
            "alpha reduce");
    if (timed) {
        HIP_TRY(hipStreamSynchronize(s), "timing sync");
        for (int w = 0; w < 2; ++w) {
            double tot = 0.0;
            for (size_t k = 0; k < used[w]; k += 2) {
                float ms = 0.0f;
                HIP_TRY(hipEventElapsedTime(&ms, pl->bwd_events[w][k], pl->bwd_events[w][k + 1]), "event elapsed");
                tot += ms;
            }
            pl->tb_count[w] = (int64_t)(used[w] / 2);
            pl->tb_ms[w] = used[w] ? tot / (double)(used[w] / 2) : 0.0;
        }
    }
    return DTV_OK;
}

extern "C" int dtv_dd_backward(dtv_dd_plan *pl, const float *d_f, const float *d_grad_u, float *d_grad_f,
                               float *d_grad_alpha, void *stream)
{
    if (!pl || !d_f || !d_grad_u || !d_grad_f || !d_grad_alpha) return fail(DTV_EINVAL, "null argument");
    if (!pl->prm.save_for_backward || !pl->saved) return fail(DTV_ESTATE, "no forward solve with saved checkpoints");
    if (!pl->ws) return fail(DTV_ENOWS, "no workspace bound");
    hipStream_t s = (hipStream_t)stream;
    const dtv_dd_params &P = pl->prm;
    const int K = P.n_inner, N = pl->saved_outer, C = P.ckpt_every;
    const size_t E = pl->edges();
    const std::vector<float> beta = fista_betas(K);
    const int rows = pl->rows, ntiles = pl->ntiles(rows);

    HIP_TRY(hipMemsetAsync(pl->galpha(), 0, sizeof(double) * (size_t)ntiles, s), "clear");
    HIP_TRY(hipMemsetAsync(pl->pb(), 0, sizeof(float) * E, s), "clear");
    if (pl->tot_lam > 0) HIP_TRY(hipMemsetAsync(pl->lb(), 0, sizeof(float) * (size_t)pl->tot_lam, s), "clear");
    // u = f + div p^N / alpha
    const float *pN = pl->ckpt(pl->nseg);
    HIP_TRY(launch_bwd_final_u(pl->d_imgs(), pl->d_tiles(rows), ntiles, rows, pl->d_info(), pN, pN + pl->tot_p1,
                               d_grad_u, d_grad_f, pl->pb(), pl->pb() + pl->tot_p1, pl->galpha(), s),
            "final u reverse");
    if (pl->fbwd) return backward_fused(pl, d_f, d_grad_f, d_grad_alpha, beta, s);

    for (int sg = pl->nseg - 1; sg >= 0; --sg) {
        const int n0 = sg * C, n1 = std::min(N, n0 + C), m = n1 - n0;
        HIP_TRY(hipMemcpyAsync(pl->seg(0), pl->ckpt(sg), sizeof(float) * pl->state_floats, hipMemcpyDeviceToDevice, s),
                "restore checkpoint");
        // recompute the states of the segment
        for (int q = 0; q + 1 < m; ++q) {
            int rc = rec_outer(pl, pl->seg(q), d_f, false, beta, s);
            if (rc != DTV_OK) return rc;
            HIP_TRY(hipMemcpyAsync(pl->seg(q + 1), pl->xrec(K - 1), sizeof(float) * E, hipMemcpyDeviceToDevice, s),
                    "segment state");
            if (pl->tot_lam > 0)
                HIP_TRY(hipMemcpyAsync(pl->seg(q + 1) + E, pl->lam1(), sizeof(float) * (size_t)pl->tot_lam,
                                       hipMemcpyDeviceToDevice, s),
                        "segment state");
        }
        // reverse the outer steps of the segment
        for (int q = m - 1; q >= 0; --q) {
            const float *st = pl->seg(q);
            int rc = rec_outer(pl, st, d_f, true, beta, s);
            if (rc != DTV_OK) return rc;
            // xbar_K = pbar; xbar_{K-1}, xbar_{K-2} start at 0 (buffers indexed by k mod 3)
            HIP_TRY(hipMemcpyAsync(pl->xb(K % 3), pl->pb(), sizeof(float) * E, hipMemcpyDeviceToDevice, s), "xbar");
            HIP_TRY(hipMemsetAsync(pl->xb((K + 2) % 3), 0, sizeof(float) * E, s), "clear");
            if (K >= 2) HIP_TRY(hipMemsetAsync(pl->xb((K + 1) % 3), 0, sizeof(float) * E, s), "clear");
            HIP_TRY(hipMemsetAsync(pl->hb(), 0, sizeof(float) * E, s), "clear");
            for (int k = K; k >= 1; --k) {
                FistaBwdArgs a{};
                a.imgs = pl->d_imgs(); a.tiles = pl->d_tiles(rows); a.ntiles = ntiles; a.info = pl->d_info();
                a.z1 = pl->zrec(k - 1); a.z2 = pl->zrec(k - 1) + pl->tot_p1;
                const float *xa = k == 1 ? st : pl->xrec(k - 2);
                const float *xbp = k >= 3 ? pl->xrec(k - 3) : st;
                a.xa1 = xa; a.xa2 = xa + pl->tot_p1;
                a.xb1 = xbp; a.xb2 = xbp + pl->tot_p1;
                a.base1 = st; a.base2 = st + pl->tot_p1;
                a.lam = pl->lam1(); a.f = d_f;
                a.gx1 = pl->xb(k % 3); a.gx2 = pl->xb(k % 3) + pl->tot_p1;
                a.ga1 = pl->xb((k + 2) % 3); a.ga2 = pl->xb((k + 2) % 3) + pl->tot_p1;
                a.gb1 = pl->xb((k + 1) % 3); a.gb2 = pl->xb((k + 1) % 3) + pl->tot_p1;
                a.gh1 = pl->hb(); a.gh2 = pl->hb() + pl->tot_p1;
                a.gf = d_grad_f; a.galpha = pl->galpha();
                a.beta = beta[k]; a.tau = (float)P.tau; a.inv_tau = (float)pl->inv_tau;
                HIP_TRY(launch_fista_bwd_step(a, k >= 3, rows, s), "FISTA reverse step");
                // xbar_k is consumed; its buffer becomes xbar_{k-3}
                if (k >= 3) HIP_TRY(hipMemsetAsync(pl->xb(k % 3), 0, sizeof(float) * E, s), "clear");
            }
            // pbar^n = xbar_0 + phatbar, then the interface terms
            HIP_TRY(launch_axpy_edges(pl->xb(0), pl->hb(), pl->pb(), (long long)E, s), "pbar");
            HIP_TRY(launch_bwd_interface(pl->d_imgs(), pl->n, pl->max_nlam, pl->d_info(), pl->hb(),
                                         pl->hb() + pl->tot_p1, pl->pb(), pl->pb() + pl->tot_p1, pl->lb(),
                                         (float)P.tau, (float)P.sigma, s),
                    "interface reverse");
        }
    }
    HIP_TRY(launch_alpha_reduce(pl->d_tiles(rows), ntiles, pl->n, pl->galpha(), d_grad_alpha, s), "alpha reduce");
    return DTV_OK;
}

extern "C" int dtv_dd_kernel_time(const dtv_dd_plan *pl, double *avg_ms, int64_t *launches, const char **name,
                                  double *bytes_per_launch)
{
    if (!pl) return fail(DTV_EINVAL, "null argument");
    if (avg_ms) *avg_ms = pl->t_ms;
    if (launches) *launches = pl->t_count;
    const bool cp2 = pl->prm.inner == DTV_INNER_CP2;
    const bool fused = pl->schedule == DTV_SCHED_FUSED;
    const bool persist = pl->schedule == DTV_SCHED_PERSIST;
    // full and ragged subdomains share one fused FISTA launch unless the solve is adaptive
    const bool mixed = pl->n_full < (int)pl->h_subs.size() && !pl->adaptive;
    if (name)
        *name = persist ? (cp2 ? "k_persist_cp2" : "k_persist_fista")
                : fused ? (cp2 ? "k_fused_cp2"
                               : pl->prm.keep_records ? "k_fused_fista (recording)"
                               : mixed ? "k_fused_fista_mixed"
                               : pl->stagger_blocks > 0 ? "k_fused_fista_staggered"
                                                        : "k_fused_fista")
                        : (cp2 ? (pl->spl > 1 ? "k_cp2_multi" : "k_cp2_step")
                               : (pl->spl > 1 ? "k_fista_multi" : "k_fista_step"));
    if (bytes_per_launch) {
        // Algorithmic HBM bytes of one timed launch (E = edge dofs of the torn
        // p~, N = pixels, 4 bytes each), averaged over the launches of an outer step.
        //   fused: read p~^n and f, write p~^(n+1)                                 4 (2E + N)
        //   fused, recording (keep_records): and write the K step records          4 (2E + N) + 9 K N
        //   fused CP2: read p~^n, u, f (+ mask bytes), write p~^(n+1), u           4 (2E + 3N) + mask
        //   streaming FISTA step 1: read x_0 and f, write c' and x_1                4 (3E + N)
        //   streaming FISTA step 2: read x_1 and c', write x_2                      4 (3E)
        //   streaming FISTA step k >= 3: read x_{k-1}, x_{k-2}, c', write x_k       4 (4E)
        //   CP2 step 1: read x_0, u, f (+ mask bytes), write x_1, u                 4 (2E + 3N) + mask
        //   CP2 step k >= 2: read x_{k-1}, x_{k-2}, anchor base, u, f (+ mask), write 4 (4E + 3N) + mask
        //   CP2 launch of steps k .. k + S - 1 (S >= 2): read x_{k-1}, x_{k-2} (k >= 2), anchor base, u, f
        //     (+ mask), write x_{k+S-1}, u and, unless the launch ends the outer step, x_{k+S-2}:
        //     4 (5E + 3N) + mask (k = 1: 4 (3E + 3N) + mask; all K steps in one launch: 4 (2E + 3N) + mask)
        //   FISTA launch of steps k .. k + S - 1 (S >= 2): read x_{k-1} (k = 1: and f), x_{k-2} (k >= 3),
        //     c' (k >= 2), write x_{k+S-1}, x_{k+S-2} and c' (k = 1) unless the launch ends the outer
        //     step: 4 (2E + N) for all K steps in one launch
        //   (the streaming figures are averages over the launches of an outer step)
        double E = 0.0, N = 0.0;
        for (const ImgHost &h : pl->imgs) {
            E += (double)(h.H + h.ny) * h.W + (double)h.H * (h.W + h.nx);
            N += (double)h.H * h.W;
        }
        const int K = pl->prm.n_inner;
        const double mb = pl->prm.has_mask ? N : 0.0;
        double tot = 0.0;
        double lam = 0.0;  // multipliers
        for (const ImgHost &h : pl->imgs) lam += (double)(h.ny - 1) * h.W + (double)(h.nx - 1) * h.H;
        if (persist) {
            // one launch for the whole solve: read p~^0, f and the lambda state, write p~^N and the
            // lambda state, and per outer step write and read two 8-byte exchange words per multiplier
            // (primal-dual: u read and written once more, mask bytes read once)
            *bytes_per_launch = 4.0 * (2 * E + N + 6 * lam) + 32.0 * lam * pl->prm.n_outer + (cp2 ? 8.0 * N + mb : 0.0);
        } else if (fused && cp2) {
            *bytes_per_launch = 4.0 * (2 * E + 3 * N) + mb;
        } else if (fused && pl->prm.keep_records) {
            // and write the K step records, 9 bytes per pixel each (kRecGroups 16-byte groups per
            // thread of 16 pixels)
            *bytes_per_launch = 4.0 * (2 * E + N) + (double)kRecGroups * K * N;
        } else if (fused) {
            *bytes_per_launch = 4.0 * (2 * E + N);
        } else if (cp2 && pl->spl > 1) {
            const std::vector<int> steps = cp2_launch_steps(K, pl->spl);
            int k = 1;
            for (size_t n = 0; n < steps.size(); ++n) {
                const int S = steps[n];
                const double reads = (k == 1 ? E : 3 * E) + 2 * N;  // x_{k-1} (and x_{k-2}, base), u, f
                const double writes = E + N + (S >= 2 && n + 1 < steps.size() ? E : 0.0);
                tot += 4.0 * (reads + writes) + mb;
                k += S;
            }
            *bytes_per_launch = tot / (double)steps.size();
        } else if (pl->spl > 1) {
            const std::vector<Cp2Launch> plan = fista_stream_plan(K, pl->spl, 0);
            for (const Cp2Launch &l : plan) {
                double b;
                if (l.steps == 1) {
                    b = l.k0 == 1 ? 4.0 * (3 * E + N) : (l.k0 == 2 ? 4.0 * (3 * E) : 4.0 * (4 * E));
                } else {
                    const double reads = l.k0 == 1 ? E + N : (l.k0 == 2 ? 2 * E : 3 * E);
                    const double writes = E + (l.ic >= 0 ? E : 0.0) + (l.k0 == 1 && plan.size() > 1 ? E : 0.0);
                    b = 4.0 * (reads + writes);
                }
                tot += b;
            }
            *bytes_per_launch = tot / (double)plan.size();
        } else {
            for (int k = 1; k <= K; ++k) {
                if (cp2) tot += (k == 1 ? 4.0 * (2 * E + 3 * N) : 4.0 * (4 * E + 3 * N)) + mb;
                else tot += k == 1 ? 4.0 * (3 * E + N) : (k == 2 ? 4.0 * (3 * E) : 4.0 * (4 * E));
            }
            *bytes_per_launch = tot / K;
        }
    }
    return DTV_OK;
}

extern "C" int dtv_dd_backward_kernel_time(const dtv_dd_plan *pl, int32_t which, double *avg_ms, int64_t *launches,
                                           const char **name, double *bytes_per_launch)
{
    if (!pl) return fail(DTV_EINVAL, "null argument");
    if (which != 0 && which != 1) return fail(DTV_EINVAL, "which must be 0 (reverse steps) or 1 (recording forward)");
    if (avg_ms) *avg_ms = pl->tb_ms[which];
    if (launches) *launches = pl->tb_count[which];
    if (name) *name = which == 0 ? (pl->pbwd ? "k_persist_bwd" : "k_fused_bwd") : "k_fused_fista (recording)";
    if (bytes_per_launch) {
        // Algorithmic HBM bytes of one launch (E = edge dofs of the torn p~, N = pixels, K = n_inner,
        // 4 bytes each; a step record is kRecGroups 16-byte groups per thread of 16 pixels, R = 9
        // bytes per pixel; phatbar is written on the interface copies only, a negligible part):
        //   reverse steps: read the K records, pbar^(n+1), p~^n, f and fbar; write pbar^n and fbar
        //                                                                           4 (3E + 3N) + R K N
        //   recording forward: read p~^n and f; write p~^(n+1) and the K records     4 (2E + N) + R K N
        //   (the lambda state and the interface copies are a negligible part)
        double E = 0.0, N = 0.0;
        for (const ImgHost &h : pl->imgs) {
            E += (double)(h.H + h.ny) * h.W + (double)h.H * (h.W + h.nx);
            N += (double)h.H * h.W;
        }
        const double R = (double)kRecGroups * 16.0 / 16.0;
        const double rec = R * (double)pl->prm.n_inner * N;
        *bytes_per_launch = which == 0 ? 4.0 * (3 * E + 3 * N) + rec : 4.0 * (2 * E + N) + rec;
        if (which == 0 && pl->pbwd && pl->tb_count[0] > 0) {
            // the persistent reverse, per launch: read pbar, per outer step the K records, p~^n, f and
            // fbar, and write fbar, then write pbar                  4 (2E) + steps (4 (E + 3N) + R K N)
            const double steps = (double)pl->saved_outer / (double)pl->tb_count[0];
            *bytes_per_launch = 8.0 * E + steps * (4.0 * (E + 3 * N) + rec);
        }
    }
    return DTV_OK;
}

extern "C" int dtv_dd_choice(const dtv_dd_plan *pl, int32_t *schedule, int32_t *rows, int32_t *source)
{
    if (!pl) return fail(DTV_EINVAL, "null argument");
    if (schedule) *schedule = pl->schedule;
    if (rows) *rows = pl->rows;
    if (source) *source = pl->choice_source;
    return DTV_OK;
}

// ---------------------------------------------------------------------------
// the solve that allocates nothing: the library's own device array is the workspace

static __device__ __align__(256) unsigned char scratch[DTV_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices];       // device address of `scratch` on each device, looked up once
uint64_t g_scratch_owner[kMaxDevices];  // id of the plan whose metadata that device's array holds (0: none)
}  // namespace

// Stream-ordered upload of the plan's metadata into a workspace and zeroing of its rotation buffers
// (their non-dof edges must hold 0): what dtv_dd_bind_workspace does, with no host wait and with a
// fill kernel instead of memsets.
static int upload_async(dtv_dd_plan *pl, char *ws, hipStream_t s)
{
    HIP_TRY(hipMemcpyAsync(ws + pl->off_imgs, pl->h_imgs.data(), sizeof(ImgDev) * pl->h_imgs.size(),
                           hipMemcpyHostToDevice, s),
            "upload image descriptors");
    HIP_TRY(hipMemcpyAsync(ws + pl->off_info, pl->h_info.data(), sizeof(int) * pl->h_info.size(), hipMemcpyHostToDevice,
                           s),
            "upload info words");
    if (!pl->h_beta.empty())
        HIP_TRY(hipMemcpyAsync(ws + pl->off_beta, pl->h_beta.data(), sizeof(float) * pl->h_beta.size(),
                               hipMemcpyHostToDevice, s),
                "upload momentum table");
    if (!pl->h_cp2tab.empty())
        HIP_TRY(hipMemcpyAsync(ws + pl->off_cp2tab, pl->h_cp2tab.data(), sizeof(float) * pl->h_cp2tab.size(),
                               hipMemcpyHostToDevice, s),
                "upload primal-dual step table");
    for (int ri = 0; ri < kRowChoices; ++ri)
        HIP_TRY(hipMemcpyAsync(ws + pl->off_tiles[ri], pl->h_tiles[ri].data(), sizeof(StreamTile) * pl->h_tiles[ri].size(),
                               hipMemcpyHostToDevice, s),
                "upload work list");
    for (int S = 2; S <= kMaxMultiSteps; ++S)
        for (int ri = 0; ri < kRowChoices; ++ri)
            if (!pl->h_mtiles[S - 2][ri].empty())
                HIP_TRY(hipMemcpyAsync(ws + pl->off_mtiles[S - 2][ri], pl->h_mtiles[S - 2][ri].data(),
                                       sizeof(StreamTile) * pl->h_mtiles[S - 2][ri].size(), hipMemcpyHostToDevice, s),
                        "upload work list");
    HIP_TRY(hipMemcpyAsync(ws + pl->off_subs, pl->h_subs.data(), sizeof(SubTile) * pl->h_subs.size(),
                           hipMemcpyHostToDevice, s),
            "upload subdomain list");
    if (!pl->p_subs.empty())
        HIP_TRY(hipMemcpyAsync(ws + pl->off_psubs, pl->p_subs.data(), sizeof(SubTile) * pl->p_subs.size(),
                               hipMemcpyHostToDevice, s),
                "upload subdomain groups");
    for (int k = 0; k < 4; ++k)
        if (pl->buf_size(k)) HIP_TRY(launch_fill_zero(ws + pl->off_buf[k], pl->buf_size(k), s), "clear buffers");
    return DTV_OK;
}

extern "C" int dtv_dd_solve_noalloc(dtv_dd_plan *pl, const float *d_f, const uint8_t *d_mask, float *d_u,
                                    float *d_p1, float *d_p2, float *d_lambda, void *stream)
{
    int rc = check_solve_args(pl, d_f, d_mask, d_u, d_p1, d_p2, d_lambda);
    if (rc != DTV_OK) return rc;
    const dtv_dd_params &P = pl->prm;
    if (P.diag_every != 0 || P.gap_tol > 0.0 || P.save_for_backward || P.time_kernels)
        return fail(DTV_EINVAL, "dtv_dd_solve_noalloc takes no diagnostics, gap_tol, save_for_backward or "
                                "time_kernels");
    if (pl->ws_bytes > (size_t)DTV_SCRATCH_BYTES)
        return fail(DTV_ENOWS, "the plan needs " + std::to_string(pl->ws_bytes) +
                                   " bytes of workspace, more than the library's scratch array (" +
                                   std::to_string((size_t)DTV_SCRATCH_BYTES) +
                                   " bytes); bind a workspace and call dtv_dd_solve, or set up the plan with "
                                   "schedule = DTV_SCHED_PERSIST (no rotation buffers)");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "current device");
    if (dev < 0 || dev >= kMaxDevices) return fail(DTV_EINVAL, "device index beyond the scratch table");
    hipStream_t s = (hipStream_t)stream;
    char *scr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {  // once per device, with that device current
            void *ptr = nullptr;
            HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch array address");
            if (!ptr || ((uintptr_t)ptr & 255) != 0) return fail(DTV_EHIP, "scratch array address is not 256-byte aligned");
            g_scratch_ptr[dev] = (char *)ptr;
        }
        scr = g_scratch_ptr[dev];
        if (g_scratch_owner[dev] != pl->uid) {
            g_scratch_owner[dev] = 0;
            rc = upload_async(pl, scr, s);
            if (rc != DTV_OK) return rc;
            g_scratch_owner[dev] = pl->uid;
        }
    }
    // run on the scratch array; the bound workspace (if any) is untouched
    struct WsSwap {
        dtv_dd_plan *pl;
        char *saved;
        ~WsSwap() { pl->ws = saved; }
    } swap{pl, pl->ws};
    pl->ws = scr;
    return solve_impl(pl, d_f, d_mask, d_u, d_p1, d_p2, d_lambda, nullptr, nullptr, stream, true);
}

extern "C" void dtv_dd_destroy(dtv_dd_plan *pl) { delete pl; }

extern "C" const char *dtv_last_error(void) { return g_err.c_str(); }
