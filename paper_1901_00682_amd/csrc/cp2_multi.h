// The multi-step streaming launch of the local primal-dual solver (cp2_multi.hip).
#pragma once

#include "dtvdd_internal.h"

namespace dtv {

constexpr int kMaxMultiSteps = 5;  // local steps per launch: 2 .. kMaxMultiSteps

// output columns per wave of an S-step launch (lanes S .. 64 - S)
__host__ __device__ constexpr int multi_cols(int S) { return 65 - 2 * S; }

// S consecutive primal-dual steps k .. k + S - 1 in one streaming launch (cp2_multi.hip): reads
// x_{k-1}, x_{k-2}, the anchor, u_{k-1}, f and the mask; writes x_{k+S-1}, u_{k+S-1} and, unless the
// launch ends the outer step (whose next step does not extrapolate), x_{k+S-2}.
// Level L of the launch runs step k + L with the scalars of index L below.
struct Cp2MultiArgs {
    const ImgDev *imgs;
    const StreamTile *tiles;  // strips of R rows and multi_cols(S) columns
    int ntiles;
    const int *info;
    const float *xa1, *xa2;   // x_{k-1}
    const float *xb1, *xb2;   // x_{k-2} (read when step k extrapolates)
    const float *base1, *base2;
    const float *lam;
    const float *f;
    const uint8_t *mask;      // NULL: all observed
    const float *u_in;        // u_{k-1}
    float *u_out;             // u_{k+S-1}
    float *outk1, *outk2;     // x_{k+S-2} (written when store_prev)
    float *outn1, *outn2;     // x_{k+S-1}
    // step k + L: theta[L] extrapolates the iterate it reads (theta_{k+L-1} of xbar_{k+L-1}; level 0
    // uses it only when step k extrapolates), sigma_k, tau_k and the two weights of the p update
    float theta[kMaxMultiSteps], sk[kMaxMultiSteps], tk[kMaxMultiSteps], ck[kMaxMultiSteps], ca[kMaxMultiSteps];
    float tau;
    int fidelity;
    float cv_c1, cv_c2;
    int store_prev;
};

hipError_t launch_cp2_multi(const Cp2MultiArgs &a, bool extrapolate, int rows, int steps, hipStream_t s,
                            hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

}  // namespace dtv
