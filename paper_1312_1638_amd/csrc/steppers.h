// Kernels of the adaptive Dormand-Prince 5(4) stepper (DOPRI5, one of the
// time steppers of the paper's functionality table).  The state, the stage
// slopes k_1..k_7 and every step-size quantity are FP64 and stay in device
// memory: step sizes, times and accept decisions are per problem, read and
// written by the kernels, so a whole attempt replays as one graph with no
// host round trip.
//
// State layout (per element block): [Nu][N_V][ld], element n = index % ld;
// columns n >= nelem are padding and take no step.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fr {

// y = u + h_p sum_{j < nk} a_j k_j over one block (h_p = dt[prob[n]]);
// padding columns get y = u.  nk in 1..6.
struct DpStage {
  double a[6];
  const double *k[6];
};
hipError_t launch_dp_stage(int nk, int64_t len, int64_t ld, int64_t nelem, const int32_t *prob,
                           const double *dt, const DpStage &st, const double *u, double *y,
                           hipStream_t s);

// Per-element partial sums of (e_i / (atol + rtol max(|u_i|, |y_i|)))^2 over
// the element's points (split into gridDim.y ranges) and fields, with
// e = h_p sum_j E_j k_j (E = b - bhat, seven slopes; a null slope is
// skipped).  part[chunk * pstride + n].
struct DpError {
  double E[7];
  const double *k[7];
  double atol, rtol;
};
hipError_t launch_dp_error(int nvars, int nupts, int64_t ld, int64_t nelem, int nchunk,
                           int64_t pstride, const int32_t *prob, const double *dt,
                           const DpError &er, const double *u, const double *y, double *part,
                           hipStream_t s);

// One thread per problem: err = sqrt(ssq / ndof); accept when err < 1;
// t += h (exactly tend when h reached it); next h by the controller (growth
// min(10, 0.9 err^-1/5), 10 at err = 0, at most 1 after a rejection in the
// same step; shrink max(0.2, 0.9 err^-1/5), 0.2 for a non-finite err), cut
// to tend - t.  h <= 0: the problem stands still.  rej: the rejection flag
// carried between attempts; counts (optional): [p][0] accepted, [p][1]
// rejected attempts.
hipError_t launch_dp_control(int nprob, const double *ssq, const double *ndof, double *t,
                             double *dt, const double *tend, int32_t *acc, int32_t *rej,
                             int32_t *counts, hipStream_t s);

// Accepted problems take the new state and the first-same-as-last slope:
// u = y, k1 = k7.
hipError_t launch_dp_commit(int64_t len, int64_t ld, int64_t nelem, const int32_t *prob,
                            const int32_t *acc, const double *y, const double *k7, double *u,
                            double *k1, hipStream_t s);

// h = min(h, tend - t) per problem (a new integration's first step).
hipError_t launch_dp_clamp(int nprob, const double *t, const double *tend, double *dt,
                           hipStream_t s);

}  // namespace fr
