/*
 * dd_oracle.c -- plain FP64 CPU oracle for the primal-dual nonoverlapping
 * domain decomposition of dual total-variation problems
 * (C.-O. Lee and J. Park, "A finite element nonoverlapping domain
 * decomposition method with Lagrange multipliers for the dual total
 * variation minimizations", arXiv 1901.00682).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Layout (the oracle's own, unrelated to the GPU layout): one set of
 * arrays per subdomain s, subdomains numbered row-major over the
 * ny x nx grid.  Subdomain s covers rows [ra, rb) and columns [ca, cb),
 * h = rb - ra, w = cb - ca.
 *   p1_s[k*w + x], k = 0..h, x = 0..w-1 : normal component on the
 *       horizontal pixel edge above local row k (k = h: below the last row),
 *       positive in the +row direction (Sec. 2.3, RT0 dofs).
 *   p2_s[y*(w+1) + k], y = 0..h-1, k = 0..w : normal component on the
 *       vertical pixel edge left of local column k, positive in +column.
 *   Edges on the image boundary carry no dof (H_0(div), Sec. 2.3) and stay 0.
 *   Edges on an interface carry one copy per side (torn space, Sec. 2.4).
 *
 * Everything is double precision; no FMA contraction is relied upon.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_L2 0
#define ORC_L1 1
#define ORC_CV 2
#define ORC_FISTA 0
#define ORC_CP2 1

typedef struct {
    int H, W, ny, nx;
    double alpha;
    int fidelity;      /* ORC_L2, ORC_L1 or ORC_CV (Sec. 3) */
    int inner;         /* ORC_FISTA or ORC_CP2 (local solver) */
    int no_prox_term;  /* 1: drop the 1/(2 tau)|p - phat|^2 term of the local
                          problem (the limit 1/tau -> 0); used only to compare a
                          1x1 decomposition with the undecomposed dual problem */
    double tau, sigma;          /* outer step sizes of Algorithm 1 */
    double tau0, sigma0, gamma; /* accelerated local primal-dual (Sec. 5) */
    int n_inner;                /* local iterations per outer step */
    double cv_c1, cv_c2;        /* ORC_CV: the two intensities of the convex
                                   Chan-Vese model, eq. (CCV) */
    double inner_tol;           /* > 0: stop a local solve once the relative
                                   change of its dual iterate falls below
                                   inner_tol (the inner stopping rule of Sec. 5.1,
                                   for either local solver); n_inner is then the
                                   cap */
} orc_params;

typedef struct {
    int r, c;            /* position in the subdomain grid */
    int ra, rb, ca, cb;  /* pixel rows [ra, rb), columns [ca, cb) */
    int h, w;
    double *p1, *p2;     /* local dual variable (torn) */
    double *u;           /* local primal variable */
    double *f;           /* local data */
    unsigned char *m;    /* 1 = observed pixel, 0 = pixel in the inpainting set D */
    double *h1, *h2;     /* proximal anchor phat restricted to the subdomain */
    long steps_total;    /* local steps taken over all outer steps */
    int steps_max;       /* most local steps in one outer step */
    double margin;       /* smallest |log(dsq / (tol^2 nsq))| over the stopping tests so far
                            (how far every decision was from the threshold; test aid) */
    /* work arrays of the local solvers */
    double *a1, *a2, *b1, *b2, *v, *q1, *q2;
} orc_sub;

typedef struct {
    orc_params prm;
    int *row_cuts, *col_cuts;
    int nsub;
    orc_sub *sub;
    /* Lagrange multipliers, one per interface dof (Sec. 4, eq. DD):
       lam_h[(r-1)*W + j]: horizontal interface between subdomain rows r-1 and r;
       lam_v[(c-1)*H + i]: vertical interface between subdomain columns c-1 and c. */
    double *lam_h, *lam_v;
    /* interface copies of the previous outer iterate p^(n-1):
       s side (upper / left subdomain) and t side (lower / right). */
    double *prev_hs, *prev_ht, *prev_vs, *prev_vt;
    int n_done;
} orc_state;

/* ------------------------------------------------------------------ */
/* small helpers                                                        */

static double *dalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

static int sub_row_of(const orc_state *st, int i)
{
    int r = 0;
    while (st->row_cuts[r + 1] <= i) r++;
    return r;
}

static int sub_col_of(const orc_state *st, int j)
{
    int c = 0;
    while (st->col_cuts[c + 1] <= j) c++;
    return c;
}

static orc_sub *sub_at(const orc_state *st, int r, int c) { return &st->sub[r * st->prm.nx + c]; }

/* Is the horizontal edge above local row k of S a dof?  Edges on the image
   boundary are not (H_0(div)); interface edges are (torn space). */
static int dof1(const orc_state *st, const orc_sub *S, int k)
{
    if (k == 0) return S->ra > 0;
    if (k == S->h) return S->rb < st->prm.H;
    return 1;
}

static int dof2(const orc_state *st, const orc_sub *S, int k)
{
    if (k == 0) return S->ca > 0;
    if (k == S->w) return S->cb < st->prm.W;
    return 1;
}

/* Projection onto the box set C, eq. (proj_C): p / max{1, |p|}. */
static double proj_box(double p) { return p / fmax(1.0, fabs(p)); }

/* ------------------------------------------------------------------ */
/* local operators (Sec. 2.3 / 2.4)                                     */

/* div_s p: outward flux of each unit pixel of the subdomain. */
static void div_local(const orc_sub *S, const double *p1, const double *p2, double *out)
{
    int h = S->h, w = S->w;
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++)
            out[y * w + x] = (p1[(y + 1) * w + x] - p1[y * w + x])
                           + (p2[y * (w + 1) + x + 1] - p2[y * (w + 1) + x]);
}

/* div_s^* v, the adjoint of div_s on the local torn space: on an edge it is
   v(pixel before the edge) - v(pixel after the edge), with v taken as 0
   outside the subdomain (so interface dofs see one side only) and 0 on
   non-dof edges. */
static void divT_local(const orc_state *st, const orc_sub *S, const double *v, double *q1, double *q2)
{
    int h = S->h, w = S->w;
    for (int k = 0; k <= h; k++)
        for (int x = 0; x < w; x++) {
            double before = k > 0 ? v[(k - 1) * w + x] : 0.0;
            double after = k < h ? v[k * w + x] : 0.0;
            q1[k * w + x] = dof1(st, S, k) ? before - after : 0.0;
        }
    for (int y = 0; y < h; y++)
        for (int k = 0; k <= w; k++) {
            double before = k > 0 ? v[y * w + k - 1] : 0.0;
            double after = k < w ? v[y * w + k] : 0.0;
            q2[y * (w + 1) + k] = dof2(st, S, k) ? before - after : 0.0;
        }
}

/* g = (f - c1)^2 - (f - c2)^2 of the convex Chan-Vese model, eq. (CCV). */
static double cv_g(const orc_params *P, double f)
{
    double a = f - P->cv_c1, b = f - P->cv_c2;
    return a * a - b * b;
}

/* prox of a*F at one pixel, a = sigma*alpha (Sec. 3 and the inpainting prox
   of Sec. 5):
     L2: argmin (a/2)(u - f)^2 + (1/2)(u - z)^2 = (z + a f)/(1 + a);
     L1: f + shr(z - f, a), eq. (shrinkage) with 0/|0| = 0;
     CV: F(u) = <u, g> + chi_{0 <= u <= 1}(u) gives the projection of z - a g
         onto [0, 1] (Sec. 3, segmentation). */
static double prox_fidelity(const orc_params *P, double z, double f, unsigned char m, double a)
{
    if (!m) return z; /* pixel in the inpainting set D */
    if (P->fidelity == ORC_L2) return (z + a * f) / (1.0 + a);
    if (P->fidelity == ORC_CV) return fmin(fmax(z - a * cv_g(P, f), 0.0), 1.0);
    double d = z - f;
    double mag = fmax(fabs(d) - a, 0.0);
    double sgn = d > 0 ? 1.0 : (d < 0 ? -1.0 : 0.0);
    return f + mag * sgn;
}

/* ------------------------------------------------------------------ */
/* local solvers                                                        */

/* |z - x|^2 and |z|^2 over every dof of the subdomain (z the new dual
   iterate, x the previous one; non-dof edges hold 0 in both). */
static void rel_change(const orc_sub *S, const double *z1, const double *z2, const double *x1, const double *x2,
                       double *dsq, double *nsq)
{
    int n1 = (S->h + 1) * S->w, n2 = S->h * (S->w + 1);
    double d = 0.0, n = 0.0;
    for (int e = 0; e < n1; e++) {
        d += (z1[e] - x1[e]) * (z1[e] - x1[e]);
        n += z1[e] * z1[e];
    }
    for (int e = 0; e < n2; e++) {
        d += (z2[e] - x2[e]) * (z2[e] - x2[e]);
        n += z2[e] * z2[e];
    }
    *dsq = d;
    *nsq = n;
}

/* The inner stopping rule of Sec. 5.1: after local step `taken` (of at most
   n_inner), stop when |p^(k+1) - p^(k)|_2 < inner_tol |p^(k+1)|_2, or when the
   iterate did not move.  Records how close the decision came to the threshold
   (test aid). */
static int inner_converged(const orc_params *P, orc_sub *S, int taken, double dsq, double nsq)
{
    if (!(P->inner_tol > 0.0) || taken >= P->n_inner) return 0;
    double thr = P->inner_tol * P->inner_tol * nsq;
    if (dsq > 0.0 && thr > 0.0) {
        double m = fabs(log(dsq / thr));
        if (m < S->margin) S->margin = m;
    }
    return dsq == 0.0 || dsq < thr;
}

/* Projected FISTA (Beck and Teboulle) on the local dual problem of
   eq. (DD_local_dual) for the ROF fidelity without mask:
     min_{p in C_s} (alpha/2)|f_s + div_s p / alpha|^2 + (1/(2 tau))|p - phat_s|^2.
   Gradient: div_s^*(f_s + div_s p / alpha) + (p - phat_s)/tau, Lipschitz
   bound L = 8/alpha + 1/tau (|div_s|^2 <= 8).  Warm start from the previous
   outer iterate (Sec. 5), momentum restarted every outer step. */
static void local_fista(const orc_state *st, orc_sub *S)
{
    const orc_params *P = &st->prm;
    int h = S->h, w = S->w;
    int n1 = (h + 1) * w, n2 = h * (w + 1);
    double inv_tau = P->no_prox_term ? 0.0 : 1.0 / P->tau;
    double L = 8.0 / P->alpha + inv_tau;
    double *x1 = S->p1, *x2 = S->p2; /* x_k */
    double *y1 = S->a1, *y2 = S->a2; /* extrapolated point y_k */
    double *z1 = S->b1, *z2 = S->b2; /* x_{k+1} */
    memcpy(y1, x1, sizeof(double) * n1);
    memcpy(y2, x2, sizeof(double) * n2);
    double t = 1.0;
    int taken = 0;
    for (int it = 0; it < P->n_inner; it++) {
        div_local(S, y1, y2, S->v);
        for (int i = 0; i < h * w; i++) S->v[i] = S->f[i] + S->v[i] / P->alpha;
        divT_local(st, S, S->v, S->q1, S->q2);
        for (int e = 0; e < n1; e++) {
            double g = S->q1[e] + (y1[e] - S->h1[e]) * inv_tau;
            z1[e] = proj_box(y1[e] - g / L);
        }
        for (int e = 0; e < n2; e++) {
            double g = S->q2[e] + (y2[e] - S->h2[e]) * inv_tau;
            z2[e] = proj_box(y2[e] - g / L);
        }
        /* non-dof edges: q is 0 there and y, phat are 0, so z is 0 already;
           enforce it explicitly anyway */
        for (int x = 0; x < w; x++) {
            if (!dof1(st, S, 0)) z1[x] = 0.0;
            if (!dof1(st, S, h)) z1[h * w + x] = 0.0;
        }
        for (int y = 0; y < h; y++) {
            if (!dof2(st, S, 0)) z2[y * (w + 1)] = 0.0;
            if (!dof2(st, S, w)) z2[y * (w + 1) + w] = 0.0;
        }
        /* relative change of the local iterate, |x_{k+1} - x_k|_2 / |x_{k+1}|_2,
           over every dof of the subdomain (Sec. 5.1, inner stopping rule) */
        double dsq, nsq;
        rel_change(S, z1, z2, x1, x2, &dsq, &nsq);
        double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
        double beta = (t - 1.0) / tn;
        for (int e = 0; e < n1; e++) {
            y1[e] = z1[e] + beta * (z1[e] - x1[e]);
            x1[e] = z1[e];
        }
        for (int e = 0; e < n2; e++) {
            y2[e] = z2[e] + beta * (z2[e] - x2[e]);
            x2[e] = z2[e];
        }
        t = tn;
        taken = it + 1;
        if (inner_converged(P, S, taken, dsq, nsq)) break;
    }
    S->steps_total += taken;
    if (taken > S->steps_max) S->steps_max = taken;
    /* primal recovery for ROF: u_s = f_s + div_s p_s / alpha (Sec. 4) */
    div_local(S, x1, x2, S->v);
    for (int i = 0; i < h * w; i++) S->u[i] = S->f[i] + S->v[i] / P->alpha;
}

/* Accelerated primal-dual method (Chambolle-Pock 2011, Algorithm 2) on the
   local saddle problem eq. (local) of Sec. 5, with x = p_s (the 1/tau
   uniformly convex part G_s^*), y = u_s and K = div_s:
     u   <- prox_{sigma_k alpha F_s}(u + sigma_k div_s xbar)
     p'  <- prox_{tau_k G_s^*}(p - tau_k div_s^* u)
          = proj_C((tau (p - tau_k div_s^* u) + tau_k phat)/(tau + tau_k))
     theta = 1/sqrt(1 + 2 gamma tau_k), tau_k <- theta tau_k,
     sigma_k <- sigma_k / theta, xbar = p' + theta (p' - p).
   Warm start (p_s, u_s) from the previous outer step, step sizes reset.
   With inner_tol the relative-change rule of Sec. 5.1 on p stops the solve
   (the state is then (p^(k), u^(k)) of the last step taken). */
static void local_cp2(const orc_state *st, orc_sub *S)
{
    const orc_params *P = &st->prm;
    int h = S->h, w = S->w;
    int n1 = (h + 1) * w, n2 = h * (w + 1);
    double *x1 = S->p1, *x2 = S->p2;
    double *xb1 = S->a1, *xb2 = S->a2; /* xbar */
    double *z1 = S->b1, *z2 = S->b2;   /* new p */
    memcpy(xb1, x1, sizeof(double) * n1);
    memcpy(xb2, x2, sizeof(double) * n2);
    double tk = P->tau0, sk = P->sigma0;
    int taken = 0;
    for (int it = 0; it < P->n_inner; it++) {
        div_local(S, xb1, xb2, S->v);
        for (int i = 0; i < h * w; i++)
            S->u[i] = prox_fidelity(P, S->u[i] + sk * S->v[i], S->f[i], S->m[i], sk * P->alpha);
        divT_local(st, S, S->u, S->q1, S->q2);
        for (int e = 0; e < n1; e++) {
            double pbar = x1[e] - tk * S->q1[e];
            z1[e] = P->no_prox_term ? proj_box(pbar)
                                    : proj_box((P->tau * pbar + tk * S->h1[e]) / (P->tau + tk));
        }
        for (int e = 0; e < n2; e++) {
            double pbar = x2[e] - tk * S->q2[e];
            z2[e] = P->no_prox_term ? proj_box(pbar)
                                    : proj_box((P->tau * pbar + tk * S->h2[e]) / (P->tau + tk));
        }
        for (int x = 0; x < w; x++) {
            if (!dof1(st, S, 0)) z1[x] = 0.0;
            if (!dof1(st, S, h)) z1[h * w + x] = 0.0;
        }
        for (int y = 0; y < h; y++) {
            if (!dof2(st, S, 0)) z2[y * (w + 1)] = 0.0;
            if (!dof2(st, S, w)) z2[y * (w + 1) + w] = 0.0;
        }
        double dsq, nsq;
        rel_change(S, z1, z2, x1, x2, &dsq, &nsq);
        double theta = 1.0 / sqrt(1.0 + 2.0 * P->gamma * tk);
        tk = theta * tk;
        sk = sk / theta;
        for (int e = 0; e < n1; e++) {
            xb1[e] = z1[e] + theta * (z1[e] - x1[e]);
            x1[e] = z1[e];
        }
        for (int e = 0; e < n2; e++) {
            xb2[e] = z2[e] + theta * (z2[e] - x2[e]);
            x2[e] = z2[e];
        }
        taken = it + 1;
        if (inner_converged(P, S, taken, dsq, nsq)) break;
    }
    S->steps_total += taken;
    if (taken > S->steps_max) S->steps_max = taken;
}

/* ------------------------------------------------------------------ */
/* state management                                                     */

void orc_destroy(orc_state *st)
{
    if (!st) return;
    for (int s = 0; s < st->nsub; s++) {
        orc_sub *S = &st->sub[s];
        free(S->p1); free(S->p2); free(S->u); free(S->f); free(S->m);
        free(S->h1); free(S->h2);
        free(S->a1); free(S->a2); free(S->b1); free(S->b2);
        free(S->v); free(S->q1); free(S->q2);
    }
    free(st->sub);
    free(st->row_cuts); free(st->col_cuts);
    free(st->lam_h); free(st->lam_v);
    free(st->prev_hs); free(st->prev_ht); free(st->prev_vs); free(st->prev_vt);
    free(st);
}

/* Create the state of Algorithm 1: p^(0) = p^(-1) = 0, lambda^(0) = 0, and
   u^(0) = f (the warm start of the first local primal-dual solve).
   mask may be NULL (every pixel observed).  Returns NULL on bad input. */
orc_state *orc_create(const orc_params *prm, const int *row_cuts, const int *col_cuts,
                      const double *f, const unsigned char *mask)
{
    if (!prm || prm->H < 1 || prm->W < 1 || prm->ny < 1 || prm->nx < 1 || !(prm->alpha > 0)) return NULL;
    if (prm->fidelity < ORC_L2 || prm->fidelity > ORC_CV) return NULL;
    /* the local FISTA solves the ROF dual only; the Chan-Vese model has no mask */
    if (prm->inner == ORC_FISTA && (prm->fidelity != ORC_L2 || mask)) return NULL;
    if (prm->fidelity == ORC_CV && mask) return NULL;
    if (row_cuts[0] != 0 || row_cuts[prm->ny] != prm->H) return NULL;
    if (col_cuts[0] != 0 || col_cuts[prm->nx] != prm->W) return NULL;
    for (int r = 0; r < prm->ny; r++) if (row_cuts[r + 1] <= row_cuts[r]) return NULL;
    for (int c = 0; c < prm->nx; c++) if (col_cuts[c + 1] <= col_cuts[c]) return NULL;

    orc_state *st = (orc_state *)calloc(1, sizeof(orc_state));
    st->prm = *prm;
    int H = prm->H, W = prm->W, ny = prm->ny, nx = prm->nx;
    st->row_cuts = (int *)malloc(sizeof(int) * (ny + 1));
    st->col_cuts = (int *)malloc(sizeof(int) * (nx + 1));
    memcpy(st->row_cuts, row_cuts, sizeof(int) * (ny + 1));
    memcpy(st->col_cuts, col_cuts, sizeof(int) * (nx + 1));
    st->nsub = ny * nx;
    st->sub = (orc_sub *)calloc(st->nsub, sizeof(orc_sub));
    for (int r = 0; r < ny; r++)
        for (int c = 0; c < nx; c++) {
            orc_sub *S = sub_at(st, r, c);
            S->r = r; S->c = c;
            S->ra = row_cuts[r]; S->rb = row_cuts[r + 1];
            S->ca = col_cuts[c]; S->cb = col_cuts[c + 1];
            S->h = S->rb - S->ra; S->w = S->cb - S->ca;
            size_t n1 = (size_t)(S->h + 1) * S->w, n2 = (size_t)S->h * (S->w + 1), np = (size_t)S->h * S->w;
            S->p1 = dalloc(n1); S->p2 = dalloc(n2);
            S->h1 = dalloc(n1); S->h2 = dalloc(n2);
            S->a1 = dalloc(n1); S->a2 = dalloc(n2);
            S->b1 = dalloc(n1); S->b2 = dalloc(n2);
            S->q1 = dalloc(n1); S->q2 = dalloc(n2);
            S->u = dalloc(np); S->f = dalloc(np); S->v = dalloc(np);
            S->margin = INFINITY;
            S->m = (unsigned char *)malloc(np ? np : 1);
            for (int y = 0; y < S->h; y++)
                for (int x = 0; x < S->w; x++) {
                    size_t g = (size_t)(S->ra + y) * W + (S->ca + x);
                    S->f[y * S->w + x] = f[g];
                    S->u[y * S->w + x] = f[g];
                    S->m[y * S->w + x] = mask ? (mask[g] != 0) : 1;
                }
        }
    st->lam_h = dalloc((size_t)(ny - 1) * W);
    st->lam_v = dalloc((size_t)(nx - 1) * H);
    st->prev_hs = dalloc((size_t)(ny - 1) * W);
    st->prev_ht = dalloc((size_t)(ny - 1) * W);
    st->prev_vs = dalloc((size_t)(nx - 1) * H);
    st->prev_vt = dalloc((size_t)(nx - 1) * H);
    return st;
}

/* Addresses of the two copies of interface dofs.
   Horizontal interface r (between subdomain rows r-1 and r), column j. */
static double *copy_hs(const orc_state *st, int r, int j, double **t_out)
{
    int c = sub_col_of(st, j);
    orc_sub *s = sub_at(st, r - 1, c), *t = sub_at(st, r, c);
    *t_out = &t->p1[0 * t->w + (j - t->ca)];
    return &s->p1[s->h * s->w + (j - s->ca)];
}

/* Vertical interface c (between subdomain columns c-1 and c), row i. */
static double *copy_vs(const orc_state *st, int c, int i, double **t_out)
{
    int r = sub_row_of(st, i);
    orc_sub *s = sub_at(st, r, c - 1), *t = sub_at(st, r, c);
    *t_out = &t->p2[(i - t->ra) * (t->w + 1) + 0];
    return &s->p2[(i - s->ra) * (s->w + 1) + s->w];
}

/* ------------------------------------------------------------------ */
/* Algorithm 1                                                          */

/* One outer iteration of Algorithm 1.  order: a permutation of the
   subdomains giving the order of the local solves (NULL: natural order,
   solved in parallel).  The local solves of one outer step read only
   step-n data, so the order does not change the result. */
static void outer_step(orc_state *st, const int *order)
{
    const orc_params *P = &st->prm;
    int H = P->H, W = P->W, ny = P->ny, nx = P->nx;

    /* lambda^(n+1) = lambda^(n) + sigma B(2 p^(n) - p^(n-1)), with
       (B p)|_e = p_s . n - p_t . n for the lower-numbered subdomain s. */
    for (int r = 1; r < ny; r++)
        for (int j = 0; j < W; j++) {
            double *pt, *ps = copy_hs(st, r, j, &pt);
            size_t e = (size_t)(r - 1) * W + j;
            st->lam_h[e] += P->sigma * ((2.0 * *ps - st->prev_hs[e]) - (2.0 * *pt - st->prev_ht[e]));
        }
    for (int c = 1; c < nx; c++)
        for (int i = 0; i < H; i++) {
            double *pt, *ps = copy_vs(st, c, i, &pt);
            size_t e = (size_t)(c - 1) * H + i;
            st->lam_v[e] += P->sigma * ((2.0 * *ps - st->prev_vs[e]) - (2.0 * *pt - st->prev_vt[e]));
        }

    /* phat^(n+1) = p^(n) - tau B^* lambda^(n+1): B^* puts +lambda on the s
       copy and -lambda on the t copy. */
    for (int s = 0; s < st->nsub; s++) {
        orc_sub *S = &st->sub[s];
        memcpy(S->h1, S->p1, sizeof(double) * (S->h + 1) * S->w);
        memcpy(S->h2, S->p2, sizeof(double) * S->h * (S->w + 1));
    }
    for (int r = 1; r < ny; r++)
        for (int j = 0; j < W; j++) {
            int c = sub_col_of(st, j);
            orc_sub *s = sub_at(st, r - 1, c), *t = sub_at(st, r, c);
            size_t e = (size_t)(r - 1) * W + j;
            s->h1[s->h * s->w + (j - s->ca)] -= P->tau * st->lam_h[e];
            t->h1[0 * t->w + (j - t->ca)] += P->tau * st->lam_h[e];
        }
    for (int c = 1; c < nx; c++)
        for (int i = 0; i < H; i++) {
            int r = sub_row_of(st, i);
            orc_sub *s = sub_at(st, r, c - 1), *t = sub_at(st, r, c);
            size_t e = (size_t)(c - 1) * H + i;
            s->h2[(i - s->ra) * (s->w + 1) + s->w] -= P->tau * st->lam_v[e];
            t->h2[(i - t->ra) * (t->w + 1) + 0] += P->tau * st->lam_v[e];
        }

    /* keep the interface copies of p^(n) for the next multiplier update */
    for (int r = 1; r < ny; r++)
        for (int j = 0; j < W; j++) {
            double *pt, *ps = copy_hs(st, r, j, &pt);
            size_t e = (size_t)(r - 1) * W + j;
            st->prev_hs[e] = *ps;
            st->prev_ht[e] = *pt;
        }
    for (int c = 1; c < nx; c++)
        for (int i = 0; i < H; i++) {
            double *pt, *ps = copy_vs(st, c, i, &pt);
            size_t e = (size_t)(c - 1) * H + i;
            st->prev_vs[e] = *ps;
            st->prev_vt[e] = *pt;
        }

    /* local problems, independent of each other */
    if (order) {
        for (int q = 0; q < st->nsub; q++) {
            orc_sub *S = &st->sub[order[q]];
            if (P->inner == ORC_FISTA) local_fista(st, S); else local_cp2(st, S);
        }
    } else {
#pragma omp parallel for schedule(dynamic, 1)
        for (int s = 0; s < st->nsub; s++) {
            orc_sub *S = &st->sub[s];
            if (P->inner == ORC_FISTA) local_fista(st, S); else local_cp2(st, S);
        }
    }
    st->n_done++;
}

/* ------------------------------------------------------------------ */
/* assembled quantities and diagnostics                                 */

/* u = direct sum of the local u_s. */
void orc_get_u(const orc_state *st, double *u)
{
    int W = st->prm.W;
    for (int s = 0; s < st->nsub; s++) {
        const orc_sub *S = &st->sub[s];
        for (int y = 0; y < S->h; y++)
            for (int x = 0; x < S->w; x++) u[(size_t)(S->ra + y) * W + S->ca + x] = S->u[y * S->w + x];
    }
}

/* Anisotropic discrete TV, TV(u) = sum over interior edges |u_b - u_a|
   (Prop. equiv with the forward differences of eq. FFD). */
double orc_tv(int H, int W, const double *u)
{
    double tv = 0.0;
    for (int i = 0; i < H; i++)
        for (int j = 0; j < W; j++) {
            if (i + 1 < H) tv += fabs(u[(size_t)(i + 1) * W + j] - u[(size_t)i * W + j]);
            if (j + 1 < W) tv += fabs(u[(size_t)i * W + j + 1] - u[(size_t)i * W + j]);
        }
    return tv;
}

/* Primal energy J(u) = alpha F(u) + TV(u), eq. (model).  For the Chan-Vese
   fidelity F(u) = <u, g>; the indicator of [0, 1] is left out (the local
   prox keeps every iterate inside). */
double orc_primal_energy(const orc_state *st, const double *u, const double *f, const unsigned char *mask)
{
    const orc_params *P = &st->prm;
    size_t n = (size_t)P->H * P->W;
    double fid = 0.0;
    for (size_t i = 0; i < n; i++) {
        if (mask && !mask[i]) continue;
        double d = u[i] - f[i];
        if (P->fidelity == ORC_CV) fid += u[i] * cv_g(P, f[i]);
        else fid += P->fidelity == ORC_L2 ? 0.5 * d * d : fabs(d);
    }
    return P->alpha * fid + orc_tv(P->H, P->W, u);
}

/* Global conforming field p_avg: interior dofs from the owning subdomain,
   interface dofs the mean of the two copies, boundary edges 0.
   Global layout: g1[i*W + j], i = 0..H (edge above row i);
                  g2[i*(W+1) + j], j = 0..W (edge left of column j). */
static void assemble_pavg(const orc_state *st, double *g1, double *g2)
{
    int H = st->prm.H, W = st->prm.W;
    memset(g1, 0, sizeof(double) * (size_t)(H + 1) * W);
    memset(g2, 0, sizeof(double) * (size_t)H * (W + 1));
    for (int s = 0; s < st->nsub; s++) {
        const orc_sub *S = &st->sub[s];
        for (int k = 1; k < S->h; k++)
            for (int x = 0; x < S->w; x++) g1[(size_t)(S->ra + k) * W + S->ca + x] = S->p1[k * S->w + x];
        for (int y = 0; y < S->h; y++)
            for (int k = 1; k < S->w; k++) g2[(size_t)(S->ra + y) * (W + 1) + S->ca + k] = S->p2[y * (S->w + 1) + k];
    }
    for (int r = 1; r < st->prm.ny; r++)
        for (int j = 0; j < W; j++) {
            double *pt, *ps = copy_hs(st, r, j, &pt);
            g1[(size_t)st->row_cuts[r] * W + j] = 0.5 * (*ps + *pt);
        }
    for (int c = 1; c < st->prm.nx; c++)
        for (int i = 0; i < H; i++) {
            double *pt, *ps = copy_vs(st, c, i, &pt);
            g2[(size_t)i * (W + 1) + st->col_cuts[c]] = 0.5 * (*ps + *pt);
        }
}

/* Diagnostics of the current iterate:
     out[0] = J(u), the primal energy of the assembled u;
     out[1] = D(p_avg) = -(alpha F)^*(div p_avg), the dual value of the
              conforming average: for L2 -<f, d> - |d|^2/(2 alpha), for the
              Chan-Vese fidelity sum over pixels of min(0, alpha g - d)
              (d = div p_avg; finite for L2 and CV without mask, NaN
              otherwise);
     out[2] = J - D, the primal-dual gap (>= 0 by weak duality; NaN when D is);
     out[3] = |B p|_2, the interface jump. */
void orc_diagnostics(const orc_state *st, const double *f_global, const unsigned char *mask, double *out)
{
    const orc_params *P = &st->prm;
    int H = P->H, W = P->W;
    size_t n = (size_t)H * W;
    double *u = dalloc(n);
    orc_get_u(st, u);
    double J = orc_primal_energy(st, u, f_global, mask);
    double D = NAN;
    int has_mask = 0;
    if (mask)
        for (size_t i = 0; i < n; i++) if (!mask[i]) { has_mask = 1; break; }
    if ((P->fidelity == ORC_L2 || P->fidelity == ORC_CV) && !has_mask) {
        double *g1 = dalloc((size_t)(H + 1) * W), *g2 = dalloc((size_t)H * (W + 1));
        assemble_pavg(st, g1, g2);
        double lin = 0.0, quad = 0.0, cv = 0.0;
        for (int i = 0; i < H; i++)
            for (int j = 0; j < W; j++) {
                double d = (g1[(size_t)(i + 1) * W + j] - g1[(size_t)i * W + j])
                         + (g2[(size_t)i * (W + 1) + j + 1] - g2[(size_t)i * (W + 1) + j]);
                double fv = f_global[(size_t)i * W + j];
                lin += fv * d;
                quad += d * d;
                cv += fmin(0.0, P->alpha * cv_g(P, fv) - d);
            }
        D = P->fidelity == ORC_CV ? cv : -lin - quad / (2.0 * P->alpha);
        free(g1); free(g2);
    }
    double nb = 0.0;
    for (int r = 1; r < P->ny; r++)
        for (int j = 0; j < W; j++) {
            double *pt, *ps = copy_hs(st, r, j, &pt);
            nb += (*ps - *pt) * (*ps - *pt);
        }
    for (int c = 1; c < P->nx; c++)
        for (int i = 0; i < H; i++) {
            double *pt, *ps = copy_vs(st, c, i, &pt);
            nb += (*ps - *pt) * (*ps - *pt);
        }
    out[0] = J;
    out[1] = D;
    out[2] = J - D;
    out[3] = sqrt(nb);
    free(u);
}

/* Run n_outer outer steps.  Every diag_every steps (0: never) a row
   [n, J, D, gap, |Bp|] is appended to stats (room for max_rows rows).
   f_global / mask are the inputs given to orc_create (for the energies).
   Returns the number of rows written. */
int orc_run(orc_state *st, int n_outer, const int *order, int diag_every,
            const double *f_global, const unsigned char *mask, double *stats, int max_rows)
{
    int rows = 0;
    for (int n = 0; n < n_outer; n++) {
        outer_step(st, order);
        if (diag_every > 0 && st->n_done % diag_every == 0 && stats && rows < max_rows) {
            double d[4];
            orc_diagnostics(st, f_global, mask, d);
            stats[rows * 5 + 0] = st->n_done;
            for (int q = 0; q < 4; q++) stats[rows * 5 + 1 + q] = d[q];
            rows++;
        }
    }
    return rows;
}

/* ------------------------------------------------------------------ */
/* state export / import (sizes, concatenated per-subdomain layout)      */

/* out[0] = dofs in the concatenated torn p (sum over s of (h+1)w + h(w+1)),
   out[1] = number of multipliers ((ny-1)W + (nx-1)H),
   out[2] = H*W. */
void orc_sizes(const orc_state *st, long *out)
{
    long np = 0;
    for (int s = 0; s < st->nsub; s++) {
        const orc_sub *S = &st->sub[s];
        np += (long)(S->h + 1) * S->w + (long)S->h * (S->w + 1);
    }
    out[0] = np;
    out[1] = (long)(st->prm.ny - 1) * st->prm.W + (long)(st->prm.nx - 1) * st->prm.H;
    out[2] = (long)st->prm.H * st->prm.W;
}

/* p: concatenation over s of p1_s then p2_s.  lam: lam_h then lam_v.
   prev: prev_hs, prev_ht, prev_vs, prev_vt (each sized like lam_h / lam_v). */
void orc_export(const orc_state *st, double *u, double *p, double *lam, double *prev, long *n_done)
{
    int H = st->prm.H, W = st->prm.W, ny = st->prm.ny, nx = st->prm.nx;
    size_t nh = (size_t)(ny - 1) * W, nv = (size_t)(nx - 1) * H;
    if (u) orc_get_u(st, u);
    if (p) {
        size_t o = 0;
        for (int s = 0; s < st->nsub; s++) {
            const orc_sub *S = &st->sub[s];
            size_t n1 = (size_t)(S->h + 1) * S->w, n2 = (size_t)S->h * (S->w + 1);
            memcpy(p + o, S->p1, sizeof(double) * n1); o += n1;
            memcpy(p + o, S->p2, sizeof(double) * n2); o += n2;
        }
    }
    if (lam) {
        memcpy(lam, st->lam_h, sizeof(double) * nh);
        memcpy(lam + nh, st->lam_v, sizeof(double) * nv);
    }
    if (prev) {
        memcpy(prev, st->prev_hs, sizeof(double) * nh);
        memcpy(prev + nh, st->prev_ht, sizeof(double) * nh);
        memcpy(prev + 2 * nh, st->prev_vs, sizeof(double) * nv);
        memcpy(prev + 2 * nh + nv, st->prev_vt, sizeof(double) * nv);
    }
    if (n_done) *n_done = st->n_done;
}

void orc_import(orc_state *st, const double *u, const double *p, const double *lam, const double *prev, long n_done)
{
    int H = st->prm.H, W = st->prm.W, ny = st->prm.ny, nx = st->prm.nx;
    size_t nh = (size_t)(ny - 1) * W, nv = (size_t)(nx - 1) * H;
    if (u)
        for (int s = 0; s < st->nsub; s++) {
            orc_sub *S = &st->sub[s];
            for (int y = 0; y < S->h; y++)
                for (int x = 0; x < S->w; x++) S->u[y * S->w + x] = u[(size_t)(S->ra + y) * W + S->ca + x];
        }
    if (p) {
        size_t o = 0;
        for (int s = 0; s < st->nsub; s++) {
            orc_sub *S = &st->sub[s];
            size_t n1 = (size_t)(S->h + 1) * S->w, n2 = (size_t)S->h * (S->w + 1);
            memcpy(S->p1, p + o, sizeof(double) * n1); o += n1;
            memcpy(S->p2, p + o, sizeof(double) * n2); o += n2;
        }
    }
    if (lam) {
        memcpy(st->lam_h, lam, sizeof(double) * nh);
        memcpy(st->lam_v, lam + nh, sizeof(double) * nv);
    }
    if (prev) {
        memcpy(st->prev_hs, prev, sizeof(double) * nh);
        memcpy(st->prev_ht, prev + nh, sizeof(double) * nh);
        memcpy(st->prev_vs, prev + 2 * nh, sizeof(double) * nv);
        memcpy(st->prev_vt, prev + 2 * nh + nv, sizeof(double) * nv);
    }
    st->n_done = (int)n_done;
}

/* ------------------------------------------------------------------ */
/* the linear operators, exposed so that tests can pin them              */

/* u = div~ p: each pixel takes the local divergence of its own subdomain. */
void orc_apply_div(const orc_state *st, const double *p, double *u)
{
    int W = st->prm.W;
    size_t o = 0;
    for (int s = 0; s < st->nsub; s++) {
        orc_sub *S = &st->sub[s];
        size_t n1 = (size_t)(S->h + 1) * S->w, n2 = (size_t)S->h * (S->w + 1);
        div_local(S, p + o, p + o + n1, S->v);
        o += n1 + n2;
        for (int y = 0; y < S->h; y++)
            for (int x = 0; x < S->w; x++) u[(size_t)(S->ra + y) * W + S->ca + x] = S->v[y * S->w + x];
    }
}

/* p = div~^* u (one-sided on interface dofs, 0 on boundary edges). */
void orc_apply_divT(const orc_state *st, const double *u, double *p)
{
    int W = st->prm.W;
    size_t o = 0;
    for (int s = 0; s < st->nsub; s++) {
        orc_sub *S = &st->sub[s];
        size_t n1 = (size_t)(S->h + 1) * S->w, n2 = (size_t)S->h * (S->w + 1);
        for (int y = 0; y < S->h; y++)
            for (int x = 0; x < S->w; x++) S->v[y * S->w + x] = u[(size_t)(S->ra + y) * W + S->ca + x];
        divT_local(st, S, S->v, p + o, p + o + n1);
        o += n1 + n2;
    }
}

/* offsets of each subdomain's block in the concatenated p */
static size_t sub_offset(const orc_state *st, int s_index)
{
    size_t o = 0;
    for (int s = 0; s < s_index; s++) {
        const orc_sub *S = &st->sub[s];
        o += (size_t)(S->h + 1) * S->w + (size_t)S->h * (S->w + 1);
    }
    return o;
}

/* lam = B p (jump operator of Sec. 2.4). */
void orc_apply_B(const orc_state *st, const double *p, double *lam)
{
    int H = st->prm.H, W = st->prm.W, ny = st->prm.ny, nx = st->prm.nx;
    size_t nh = (size_t)(ny - 1) * W;
    for (int r = 1; r < ny; r++)
        for (int j = 0; j < W; j++) {
            int c = sub_col_of(st, j);
            int si = (r - 1) * nx + c, ti = r * nx + c;
            const orc_sub *s = &st->sub[si], *t = &st->sub[ti];
            double ps = p[sub_offset(st, si) + (size_t)s->h * s->w + (j - s->ca)];
            double pt = p[sub_offset(st, ti) + (j - t->ca)];
            lam[(size_t)(r - 1) * W + j] = ps - pt;
        }
    for (int c = 1; c < nx; c++)
        for (int i = 0; i < H; i++) {
            int r = sub_row_of(st, i);
            int si = r * nx + c - 1, ti = r * nx + c;
            const orc_sub *s = &st->sub[si], *t = &st->sub[ti];
            size_t s2 = sub_offset(st, si) + (size_t)(s->h + 1) * s->w;
            size_t t2 = sub_offset(st, ti) + (size_t)(t->h + 1) * t->w;
            double ps = p[s2 + (size_t)(i - s->ra) * (s->w + 1) + s->w];
            double pt = p[t2 + (size_t)(i - t->ra) * (t->w + 1)];
            lam[nh + (size_t)(c - 1) * H + i] = ps - pt;
        }
}

/* p = B^* lam (zero away from interface copies). */
void orc_apply_BT(const orc_state *st, const double *lam, double *p)
{
    int H = st->prm.H, W = st->prm.W, ny = st->prm.ny, nx = st->prm.nx;
    size_t nh = (size_t)(ny - 1) * W;
    long sz[3];
    orc_sizes(st, sz);
    memset(p, 0, sizeof(double) * (size_t)sz[0]);
    for (int r = 1; r < ny; r++)
        for (int j = 0; j < W; j++) {
            int c = sub_col_of(st, j);
            int si = (r - 1) * nx + c, ti = r * nx + c;
            const orc_sub *s = &st->sub[si], *t = &st->sub[ti];
            double l = lam[(size_t)(r - 1) * W + j];
            p[sub_offset(st, si) + (size_t)s->h * s->w + (j - s->ca)] += l;
            p[sub_offset(st, ti) + (j - t->ca)] -= l;
        }
    for (int c = 1; c < nx; c++)
        for (int i = 0; i < H; i++) {
            int r = sub_row_of(st, i);
            int si = r * nx + c - 1, ti = r * nx + c;
            const orc_sub *s = &st->sub[si], *t = &st->sub[ti];
            size_t s2 = sub_offset(st, si) + (size_t)(s->h + 1) * s->w;
            size_t t2 = sub_offset(st, ti) + (size_t)(t->h + 1) * t->w;
            double l = lam[nh + (size_t)(c - 1) * H + i];
            p[s2 + (size_t)(i - s->ra) * (s->w + 1) + s->w] += l;
            p[t2 + (size_t)(i - t->ra) * (t->w + 1)] -= l;
        }
}

/* elementwise projection onto C, exposed for the closed-form pin */
void orc_proj_box(long n, const double *p, double *out)
{
    for (long i = 0; i < n; i++) out[i] = proj_box(p[i]);
}

/* elementwise prox of sigma*alpha*F, exposed for the closed-form pins */
void orc_prox(int fidelity, long n, const double *z, const double *f, const unsigned char *m, double a,
              double c1, double c2, double *out)
{
    orc_params P;
    memset(&P, 0, sizeof P);
    P.fidelity = fidelity;
    P.cv_c1 = c1;
    P.cv_c2 = c2;
    for (long i = 0; i < n; i++) out[i] = prox_fidelity(&P, z[i], f[i], m ? m[i] : 1, a);
}

int orc_n_done(const orc_state *st) { return st->n_done; }

/* Local steps per subdomain (row-major over the grid): out[2 s] = total over
   all outer steps run so far, out[2 s + 1] = most in one outer step. */
double orc_inner_margin(const orc_state *st)
{
    double m = INFINITY;
    for (int s = 0; s < st->nsub; s++) m = fmin(m, st->sub[s].margin);
    return m;
}

void orc_inner_counts(const orc_state *st, long *out)
{
    for (int s = 0; s < st->nsub; s++) {
        out[2 * s] = st->sub[s].steps_total;
        out[2 * s + 1] = st->sub[s].steps_max;
    }
}

#ifdef _OPENMP
#include <omp.h>
#endif
/* number of threads the parallel loops of the oracle use */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loop over subdomains from now on (n >= 1). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* reverse mode of the unrolled solve (FISTA local solver, L2, no mask)  */
/*
 * The forward map is Algorithm 1 exactly as outer_step() runs it with
 * local_fista(); the final image is u = f + div~ p^N / alpha.  Given
 * ubar = dl/du this computes dl/df and dl/dalpha by reverse accumulation:
 *   - outer steps are reversed one at a time from stored snapshots
 *     (p^n, lambda^n, prev^n) and their inner iterates recomputed;
 *   - x_k = proj(z_k): zbar = xbar * 1{|z_k| < 1} (0 on non-dof edges);
 *   - z_k = y - (1/L)[div*(f + div y / alpha) + (y - phat)/tau] is affine in
 *     (y, phat, f) with L = 8/alpha + 1/tau, so
 *       ybar += zbar - (1/L)[div*(div zbar)/alpha + zbar/tau],
 *       phatbar += zbar / (L tau),  fbar -= div zbar / L,
 *       alphabar += <zbar, dz/dalpha>,
 *     dz/dalpha = -a'[div* f + (y - phat)/tau] - b' div* div y with
 *     a = 1/L, b = 1/(alpha L), a' = 8/(alpha L)^2, b' = -1/(tau (alpha L)^2);
 *   - y_k = x_k + beta_k (x_k - x_{k-1}) with constant beta_k;
 *   - phat = p - tau B^* lambda^{n+1};
 *   - lambda^{n+1} = lambda^n + sigma B(2 p^n - prev^n), prev^{n+1} = p^n|_Gamma.
 * Returns 0, or -1 for unsupported settings.
 */

typedef struct {
    double *x;     /* x_0 .. x_K, each n1 + n2 (p1 block then p2 block) */
    double *y;     /* y_0 .. y_{K-1} */
    double *z;     /* z_1 .. z_K */
    double *zb, *yb, *xb;  /* adjoint work, n1 + n2 each; xb holds x_0 .. x_K adjoints */
    double *v;     /* pixel work */
    double *w;     /* pixel work */
} rev_work;

/* apply div_s to a concatenated (p1, p2) block */
static void div_blk(const orc_sub *S, const double *p, double *out)
{
    div_local(S, p, p + (size_t)(S->h + 1) * S->w, out);
}

static void divT_blk(const orc_state *st, const orc_sub *S, const double *v, double *q)
{
    divT_local(st, S, v, q, q + (size_t)(S->h + 1) * S->w);
}

/* forward FISTA of one subdomain from x_0 = p with anchor phat (h1, h2),
   storing every iterate; the arithmetic is that of local_fista() */
static void fista_record(const orc_state *st, const orc_sub *S, const double *x0, const double *hat, rev_work *W)
{
    const orc_params *P = &st->prm;
    int h = S->h, w = S->w;
    size_t n = (size_t)(h + 1) * w + (size_t)h * (w + 1);
    double inv_tau = 1.0 / P->tau, L = 8.0 / P->alpha + inv_tau;
    double *q = W->yb; /* scratch */
    memcpy(W->x, x0, sizeof(double) * n);
    memcpy(W->y, x0, sizeof(double) * n);
    double t = 1.0;
    for (int k = 1; k <= P->n_inner; k++) {
        const double *y = W->y + (size_t)(k - 1) * n;
        double *z = W->z + (size_t)(k - 1) * n;
        double *xk = W->x + (size_t)k * n;
        const double *xm = W->x + (size_t)(k - 1) * n;
        div_blk(S, y, W->v);
        for (int i = 0; i < h * w; i++) W->v[i] = S->f[i] + W->v[i] / P->alpha;
        divT_blk(st, S, W->v, q);
        for (size_t e = 0; e < n; e++) {
            double g = q[e] + (y[e] - hat[e]) * inv_tau;
            z[e] = y[e] - g / L;
        }
        /* non-dof edges: z is 0 there (q, y, phat all 0) */
        for (size_t e = 0; e < n; e++) xk[e] = proj_box(z[e]);
        double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
        double beta = (t - 1.0) / tn;
        if (k < P->n_inner) {
            double *yn = W->y + (size_t)k * n;
            for (size_t e = 0; e < n; e++) yn[e] = xk[e] + beta * (xk[e] - xm[e]);
        }
        t = tn;
    }
}

/* reverse of fista_record: xbar_K in W->xb + K n on entry; on exit
   W->xb holds xbar_0 (first block), hatbar accumulated, fbar_s and abar
   accumulated */
static void fista_reverse(const orc_state *st, const orc_sub *S, const double *hat, rev_work *W, double *hatbar,
                          double *fbar_s, double *abar)
{
    const orc_params *P = &st->prm;
    int h = S->h, w = S->w, K = P->n_inner;
    size_t n = (size_t)(h + 1) * w + (size_t)h * (w + 1);
    double tau = P->tau, alpha = P->alpha;
    double L = 8.0 / alpha + 1.0 / tau;
    double a = 1.0 / L;
    double da = 8.0 / (alpha * L * alpha * L);
    double db = -1.0 / (tau * (alpha * L) * (alpha * L));
    /* momentum coefficients beta_k, k = 1..K-1 (y_k = x_k + beta_k (x_k - x_{k-1})) */
    double *beta = (double *)calloc((size_t)K + 1, sizeof(double));
    double t = 1.0;
    for (int k = 1; k <= K; k++) {
        double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
        beta[k] = (t - 1.0) / tn;
        t = tn;
    }
    double *q = (double *)malloc(sizeof(double) * n);
    double *dfz = (double *)malloc(sizeof(double) * (size_t)h * w); /* div zbar */
    double *dy = (double *)malloc(sizeof(double) * (size_t)h * w);  /* div y */
    /* xbar_k, k = 0..K-1 start at 0 */
    memset(W->xb, 0, sizeof(double) * n * (size_t)K);
    for (int k = K; k >= 1; k--) {
        const double *y = W->y + (size_t)(k - 1) * n;
        const double *z = W->z + (size_t)(k - 1) * n;
        const double *xbk = W->xb + (size_t)k * n;
        /* projection: derivative 1 where |z| < 1, 0 where the box is active */
        for (size_t e = 0; e < n; e++) W->zb[e] = fabs(z[e]) < 1.0 ? xbk[e] : 0.0;
        /* zero the non-dof edges */
        {
            double *z1 = W->zb, *z2 = W->zb + (size_t)(h + 1) * w;
            for (int x = 0; x < w; x++) {
                if (!dof1(st, S, 0)) z1[x] = 0.0;
                if (!dof1(st, S, h)) z1[(size_t)h * w + x] = 0.0;
            }
            for (int yy = 0; yy < h; yy++) {
                if (!dof2(st, S, 0)) z2[(size_t)yy * (w + 1)] = 0.0;
                if (!dof2(st, S, w)) z2[(size_t)yy * (w + 1) + w] = 0.0;
            }
        }
        /* linear part */
        div_blk(S, W->zb, dfz);
        for (int i = 0; i < h * w; i++) W->v[i] = dfz[i] / alpha;
        divT_blk(st, S, W->v, q);
        for (size_t e = 0; e < n; e++) W->yb[e] = W->zb[e] - a * (q[e] + W->zb[e] / tau);
        for (size_t e = 0; e < n; e++) hatbar[e] += a / tau * W->zb[e];
        for (int i = 0; i < h * w; i++) fbar_s[i] -= a * dfz[i];
        /* dz/dalpha */
        div_blk(S, y, dy);
        double s_f = 0.0, s_y = 0.0, s_dd = 0.0;
        for (int i = 0; i < h * w; i++) {
            s_f += dfz[i] * S->f[i];
            s_dd += dfz[i] * dy[i];
        }
        for (size_t e = 0; e < n; e++) s_y += W->zb[e] * (y[e] - hat[e]);
        *abar += -da * (s_f + s_y / tau) - db * s_dd;
        /* y_{k-1} = x_{k-1} + beta_{k-1} (x_{k-1} - x_{k-2}); y_0 = x_0 */
        double *xb1 = W->xb + (size_t)(k - 1) * n;
        if (k - 1 >= 1) {
            double bk = beta[k - 1];
            double *xb2 = W->xb + (size_t)(k - 2) * n;
            for (size_t e = 0; e < n; e++) {
                xb1[e] += (1.0 + bk) * W->yb[e];
                xb2[e] -= bk * W->yb[e];
            }
        } else {
            for (size_t e = 0; e < n; e++) xb1[e] += W->yb[e];
        }
    }
    free(beta); free(q); free(dfz); free(dy);
}

/* Positions of the two copies of every interface dof in the concatenated
   p (p1_s then p2_s per subdomain): is[e] on side s, it[e] on side t, for the
   multiplier ordering lam_h then lam_v. */
static void interface_maps(const orc_state *st, long *is, long *it)
{
    int H = st->prm.H, W = st->prm.W, ny = st->prm.ny, nx = st->prm.nx;
    long *off = (long *)malloc(sizeof(long) * (size_t)(st->nsub + 1));
    off[0] = 0;
    for (int s = 0; s < st->nsub; s++) {
        const orc_sub *S = &st->sub[s];
        off[s + 1] = off[s] + (long)(S->h + 1) * S->w + (long)S->h * (S->w + 1);
    }
    size_t nh = (size_t)(ny - 1) * W;
    for (int r = 1; r < ny; r++)
        for (int j = 0; j < W; j++) {
            int c = sub_col_of(st, j);
            int si = (r - 1) * nx + c, ti = r * nx + c;
            const orc_sub *S = &st->sub[si], *T = &st->sub[ti];
            size_t e = (size_t)(r - 1) * W + j;
            is[e] = off[si] + (long)S->h * S->w + (j - S->ca);
            it[e] = off[ti] + (j - T->ca);
        }
    for (int c = 1; c < nx; c++)
        for (int i = 0; i < H; i++) {
            int r = sub_row_of(st, i);
            int si = r * nx + c - 1, ti = r * nx + c;
            const orc_sub *S = &st->sub[si], *T = &st->sub[ti];
            size_t e = nh + (size_t)(c - 1) * H + i;
            is[e] = off[si] + (long)(S->h + 1) * S->w + (long)(i - S->ra) * (S->w + 1) + S->w;
            it[e] = off[ti] + (long)(T->h + 1) * T->w + (long)(i - T->ra) * (T->w + 1);
        }
    free(off);
}

int orc_backward(orc_state *st, int n_outer, const double *f_global, const unsigned char *mask, const double *ubar,
                 double *fbar, double *abar_out)
{
    const orc_params *P = &st->prm;
    (void)f_global;
    if (P->inner != ORC_FISTA || P->fidelity != ORC_L2 || P->no_prox_term || st->n_done != 0 || mask) return -1;
    int H = P->H, W = P->W, ny = P->ny, nx = P->nx, K = P->n_inner;
    long sz[3];
    orc_sizes(st, sz);
    size_t np = (size_t)sz[0], nl = (size_t)sz[1];
    size_t nh = (size_t)(ny - 1) * W, nv = (size_t)(nx - 1) * H;
    size_t nl1 = nl ? nl : 1;
    long *is = (long *)malloc(sizeof(long) * nl1), *it = (long *)malloc(sizeof(long) * nl1);
    interface_maps(st, is, it);

    /* forward with snapshots of (p, lambda, prev) before every outer step */
    double *sp = (double *)malloc(sizeof(double) * np * (size_t)(n_outer + 1));
    double *sl = (double *)malloc(sizeof(double) * nl1 * (size_t)(n_outer + 1));
    double *sv = (double *)malloc(sizeof(double) * 2 * nl1 * (size_t)(n_outer + 1));
    for (int n = 0; n <= n_outer; n++) {
        orc_export(st, NULL, sp + np * n, sl + nl1 * n, sv + 2 * nl1 * n, NULL);
        if (n < n_outer) outer_step(st, NULL);
    }

    /* u = f + div~ p^N / alpha */
    double abar = 0.0;
    double *dv = (double *)malloc(sizeof(double) * (size_t)H * W);
    orc_apply_div(st, sp + np * n_outer, dv);
    for (size_t i = 0; i < (size_t)H * W; i++) {
        fbar[i] = ubar[i];
        abar += -ubar[i] * dv[i] / (P->alpha * P->alpha);
        dv[i] = ubar[i] / P->alpha;
    }
    double *Pb = (double *)calloc(np, sizeof(double));   /* adjoint of p^{n+1} */
    orc_apply_divT(st, dv, Pb);
    double *lamb = (double *)calloc(nl1, sizeof(double)); /* adjoint of lambda^{n+1} from later steps */
    double *pvs = (double *)calloc(nl1, sizeof(double));  /* adjoint of prev_s^{n+1} */
    double *pvt = (double *)calloc(nl1, sizeof(double));  /* adjoint of prev_t^{n+1} */
    double *Pn = (double *)malloc(sizeof(double) * np), *hat = (double *)malloc(sizeof(double) * np);
    double *hatb = (double *)malloc(sizeof(double) * np), *Pb0 = (double *)malloc(sizeof(double) * np);
    double *lam1 = (double *)malloc(sizeof(double) * nl1);

    size_t nmax = 0, pmax = 0;
    for (int s = 0; s < st->nsub; s++) {
        const orc_sub *S = &st->sub[s];
        size_t n = (size_t)(S->h + 1) * S->w + (size_t)S->h * (S->w + 1);
        if (n > nmax) nmax = n;
        if ((size_t)S->h * S->w > pmax) pmax = (size_t)S->h * S->w;
    }
    rev_work Wk;
    Wk.x = (double *)malloc(sizeof(double) * nmax * (size_t)(K + 1));
    Wk.y = (double *)malloc(sizeof(double) * nmax * (size_t)(K + 1));
    Wk.z = (double *)malloc(sizeof(double) * nmax * (size_t)(K + 1));
    Wk.xb = (double *)malloc(sizeof(double) * nmax * (size_t)(K + 1));
    Wk.zb = (double *)malloc(sizeof(double) * nmax);
    Wk.yb = (double *)malloc(sizeof(double) * nmax);
    Wk.v = (double *)malloc(sizeof(double) * pmax);
    Wk.w = (double *)malloc(sizeof(double) * pmax);
    double *fbar_s = (double *)malloc(sizeof(double) * pmax);

    for (int n = n_outer - 1; n >= 0; n--) {
        const double *lam = sl + nl1 * n, *pv = sv + 2 * nl1 * n;
        memcpy(Pn, sp + np * n, sizeof(double) * np);
        /* redo the multiplier update and the anchor of step n exactly as outer_step does */
        for (size_t e = 0; e < nl; e++) {
            double prev_s = e < nh ? pv[e] : pv[2 * nh + (e - nh)];
            double prev_t = e < nh ? pv[nh + e] : pv[2 * nh + nv + (e - nh)];
            lam1[e] = lam[e] + P->sigma * ((2.0 * Pn[is[e]] - prev_s) - (2.0 * Pn[it[e]] - prev_t));
        }
        memcpy(hat, Pn, sizeof(double) * np);
        for (size_t e = 0; e < nl; e++) {
            hat[is[e]] -= P->tau * lam1[e];
            hat[it[e]] += P->tau * lam1[e];
        }
        /* local solves in reverse */
        memset(hatb, 0, sizeof(double) * np);
        size_t o = 0;
        for (int s = 0; s < st->nsub; s++) {
            orc_sub *S = &st->sub[s];
            size_t nn = (size_t)(S->h + 1) * S->w + (size_t)S->h * (S->w + 1);
            fista_record(st, S, Pn + o, hat + o, &Wk);
            memcpy(Wk.xb + (size_t)K * nn, Pb + o, sizeof(double) * nn);
            memset(fbar_s, 0, sizeof(double) * (size_t)S->h * S->w);
            fista_reverse(st, S, hat + o, &Wk, hatb + o, fbar_s, &abar);
            memcpy(Pb0 + o, Wk.xb, sizeof(double) * nn);
            for (int y = 0; y < S->h; y++)
                for (int x = 0; x < S->w; x++) fbar[(size_t)(S->ra + y) * W + S->ca + x] += fbar_s[y * S->w + x];
            o += nn;
        }
        /* phat = p^n - tau B^* lambda^{n+1} */
        for (size_t e = 0; e < np; e++) Pb0[e] += hatb[e];
        for (size_t e = 0; e < nl; e++) {
            double lt = lamb[e] - P->tau * (hatb[is[e]] - hatb[it[e]]); /* total adjoint of lambda^{n+1} */
            /* prev^{n+1} = p^n on the interface copies */
            Pb0[is[e]] += pvs[e];
            Pb0[it[e]] += pvt[e];
            /* lambda^{n+1} = lambda^n + sigma ((2 p_s - prev_s) - (2 p_t - prev_t)) */
            Pb0[is[e]] += 2.0 * P->sigma * lt;
            Pb0[it[e]] -= 2.0 * P->sigma * lt;
            pvs[e] = -P->sigma * lt;
            pvt[e] = P->sigma * lt;
            lamb[e] = lt;
        }
        memcpy(Pb, Pb0, sizeof(double) * np);
    }
    /* p^0, lambda^0, prev^0 are constants: nothing flows further */
    *abar_out = abar;
    free(is); free(it); free(sp); free(sl); free(sv); free(dv); free(Pb); free(lamb); free(pvs); free(pvt);
    free(Pn); free(hat); free(hatb); free(Pb0); free(lam1);
    free(Wk.x); free(Wk.y); free(Wk.z); free(Wk.xb); free(Wk.zb); free(Wk.yb); free(Wk.v); free(Wk.w); free(fbar_s);
    return 0;
}
