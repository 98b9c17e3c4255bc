// The multi-step streaming launch of the local FISTA solver (fista_multi.hip).
#pragma once

#include "cp2_multi.h"
#include "dtvdd_internal.h"

namespace dtv {

// S consecutive projected-FISTA steps k .. k + S - 1 in one streaming launch (fista_multi.hip), on
// strips of R rows and multi_cols(S) columns (the primal-dual multi-step work lists).  Reads
// x_{k-1} (x_0 = p~^n when k = 1), x_{k-2} (k >= 3), and c' (k >= 2) or the multipliers and f
// (k = 1); writes x_{k+S-1}, x_{k+S-2} unless this launch ends the outer step, and c' when k = 1
// and launches follow.
struct FistaMultiArgs {
    const ImgDev *imgs;
    const StreamTile *tiles;
    int ntiles;
    const int *info;
    const float *xa1, *xa2;   // x_{k-1}
    const float *xb1, *xb2;   // x_{k-2} (k >= 3)
    const float *lam;         // lambda state (k = 1)
    const float *f;           // image (k = 1)
    float *c1, *c2;           // c': written when k = 1 and store_c, read when k >= 2
    float *outk1, *outk2;     // x_{k+S-2} (written when store_prev)
    float *outn1, *outn2;     // x_{k+S-1}
    float beta[kMaxMultiSteps];  // momentum of step k + L (used where k + L >= 3)
    float tau, inv_tau;
    int store_c, store_prev;
};

hipError_t launch_fista_multi(const FistaMultiArgs &a, int mode, int rows, int steps, hipStream_t s,
                              hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

}  // namespace dtv
