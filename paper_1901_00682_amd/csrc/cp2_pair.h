// The two-step streaming launch of the local primal-dual solver (cp2_pair.hip).
#pragma once

#include "dtvdd_internal.h"

namespace dtv {

constexpr int kPairCols = 61;  // output columns per wave (lanes 2..62)

// Two consecutive primal-dual steps k and k + 1 in one streaming launch (cp2_pair.hip): reads
// x_{k-1}, x_{k-2}, the anchor, u_{k-1}, f and the mask; writes x_k, x_{k+1} and u_{k+1}.
struct Cp2PairArgs {
    const ImgDev *imgs;
    const StreamTile *tiles;  // strips of R rows and kPairCols columns
    int ntiles;
    const int *info;
    const float *xa1, *xa2;   // x_{k-1}
    const float *xb1, *xb2;   // x_{k-2} (read when step k extrapolates)
    const float *base1, *base2;
    const float *lam;
    const float *f;
    const uint8_t *mask;      // NULL: all observed
    const float *u_in;        // u_{k-1}
    float *u_out;             // u_{k+1}
    float *outk1, *outk2;     // x_k
    float *outn1, *outn2;     // x_{k+1}
    float theta_a, sk_a, tk_a, ck_a, ca_a;  // step k (theta_a: theta_{k-1} of xbar_{k-1})
    float theta_b, sk_b, tk_b, ck_b, ca_b;  // step k + 1 (theta_b: theta_k of xbar_k)
    float tau;
    int fidelity;
    float cv_c1, cv_c2;
};

hipError_t launch_cp2_pair(const Cp2PairArgs &a, bool extrapolate, int rows, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);

}  // namespace dtv
