// Kernels of the adaptive DOPRI5 stepper (see steppers.h).  All of them are
// bound by HBM traffic: the stage combinations stream two state entries per
// thread (16-byte loads and stores), the error pass reads each slope once
// with lanes along elements, and the control kernel is one thread per
// problem.
#include "steppers.h"

#include <cmath>

namespace fr {

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

template <int NK>
__global__ __launch_bounds__(256) void dp_stage_kernel(int64_t len2, int64_t ld, int64_t nelem,
                                                       const int32_t *__restrict__ prob,
                                                       const double *__restrict__ dt, DpStage st,
                                                       const double *__restrict__ u,
                                                       double *__restrict__ y) {
  const int64_t i2 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i2 >= len2) return;
  const int64_t i = 2 * i2;          // ld is even: both entries lie in one row
  const int64_t n = i % ld;
  const double h0 = n < nelem ? dt[prob ? prob[n] : 0] : 0.0;
  const double h1 = n + 1 < nelem ? dt[prob ? prob[n + 1] : 0] : 0.0;
  double sx = 0, sy = 0;
#pragma unroll
  for (int j = 0; j < NK; ++j) {
    const double2 kv = *reinterpret_cast<const double2 *>(st.k[j] + i);
    sx += st.a[j] * kv.x;
    sy += st.a[j] * kv.y;
  }
  const double2 uv = *reinterpret_cast<const double2 *>(u + i);
  double2 out;
  out.x = uv.x + h0 * sx;
  out.y = uv.y + h1 * sy;
  *reinterpret_cast<double2 *>(y + i) = out;
}

hipError_t launch_dp_stage(int nk, int64_t len, int64_t ld, int64_t nelem, const int32_t *prob,
                           const double *dt, const DpStage &st, const double *u, double *y,
                           hipStream_t s) {
  if (len <= 0) return hipSuccess;
  if (len % 2 || ld % 2) return hipErrorInvalidValue;
  const int64_t len2 = len / 2;
  switch (nk) {
#define FR_DP_NK(K)                                                                      \
  case K:                                                                                \
    dp_stage_kernel<K><<<nblk(len2), 256, 0, s>>>(len2, ld, nelem, prob, dt, st, u, y); \
    break;
    FR_DP_NK(1) FR_DP_NK(2) FR_DP_NK(3) FR_DP_NK(4) FR_DP_NK(5) FR_DP_NK(6)
#undef FR_DP_NK
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Workgroup: 64 elements (lanes) x 4 waves that split the point range of
// this blockIdx.y chunk; the waves combine in LDS in a fixed order.
__global__ __launch_bounds__(256) void dp_error_kernel(int nvars, int nupts, int64_t ld,
                                                       int64_t nelem, int64_t pstride,
                                                       const int32_t *__restrict__ prob,
                                                       const double *__restrict__ dt, DpError er,
                                                       const double *__restrict__ u,
                                                       const double *__restrict__ y,
                                                       double *__restrict__ part) {
  __shared__ double red[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t n = (int64_t)blockIdx.x * 64 + tx;
  const int rc = (nupts + (int)gridDim.y - 1) / (int)gridDim.y;
  const int rbeg = (int)blockIdx.y * rc, rend = rbeg + rc < nupts ? rbeg + rc : nupts;
  double sum = 0;
  if (n < nelem) {
    const double h = dt[prob ? prob[n] : 0];
    for (int r = rbeg + ty; r < rend; r += 4)
      for (int al = 0; al < nvars; ++al) {
        const int64_t i = ((int64_t)r * nvars + al) * ld + n;
        double e = 0;
#pragma unroll
        for (int j = 0; j < 7; ++j)
          if (er.k[j]) e += er.E[j] * er.k[j][i];
        e *= h;
        const double sc = er.atol + er.rtol * fmax(fabs(u[i]), fabs(y[i]));
        const double q = e / sc;
        sum += q * q;
      }
  }
  red[ty][tx] = sum;
  __syncthreads();
  if (ty == 0 && n < nelem)
    part[(int64_t)blockIdx.y * pstride + n] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
}

hipError_t launch_dp_error(int nvars, int nupts, int64_t ld, int64_t nelem, int nchunk,
                           int64_t pstride, const int32_t *prob, const double *dt,
                           const DpError &er, const double *u, const double *y, double *part,
                           hipStream_t s) {
  if (nelem <= 0) return hipSuccess;
  if (nchunk < 1) return hipErrorInvalidValue;
  dim3 grid((unsigned)((nelem + 63) / 64), (unsigned)nchunk);
  dp_error_kernel<<<grid, 256, 0, s>>>(nvars, nupts, ld, nelem, pstride, prob, dt, er, u, y,
                                       part);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void dp_control_kernel(int nprob, const double *ssq,
                                                         const double *ndof, double *t,
                                                         double *dt, const double *tend,
                                                         int32_t *acc, int32_t *rej,
                                                         int32_t *counts) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= nprob) return;
  const double h = dt[p];
  if (!(h > 0)) {
    acc[p] = 0;
    return;
  }
  const double err = sqrt(ssq[p] / ndof[p]);
  const double tp = t[p];
  double tn = tp, hn;
  if (err < 1.0) {
    double fac = err == 0.0 ? 10.0 : fmin(10.0, 0.9 * pow(err, -0.2));
    if (rej[p]) fac = fmin(1.0, fac);
    tn = (tend && h >= tend[p] - tp) ? tend[p] : tp + h;
    hn = h * fac;
    acc[p] = 1;
    rej[p] = 0;
    if (counts) counts[2 * p] += 1;
  } else {
    const double fac = isfinite(err) ? fmax(0.2, 0.9 * pow(err, -0.2)) : 0.2;
    hn = h * fac;
    acc[p] = 0;
    rej[p] = 1;
    if (counts) counts[2 * p + 1] += 1;
  }
  if (tend) hn = fmin(hn, tend[p] - tn);
  t[p] = tn;
  dt[p] = hn;
}

hipError_t launch_dp_control(int nprob, const double *ssq, const double *ndof, double *t,
                             double *dt, const double *tend, int32_t *acc, int32_t *rej,
                             int32_t *counts, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  dp_control_kernel<<<nblk(nprob), 256, 0, s>>>(nprob, ssq, ndof, t, dt, tend, acc, rej, counts);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void dp_commit_kernel(int64_t len2, int64_t ld, int64_t nelem,
                                                        const int32_t *__restrict__ prob,
                                                        const int32_t *__restrict__ acc,
                                                        const double *__restrict__ y,
                                                        const double *__restrict__ k7,
                                                        double *__restrict__ u,
                                                        double *__restrict__ k1) {
  const int64_t i2 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i2 >= len2) return;
  const int64_t i = 2 * i2;
  const int64_t n = i % ld;
  const bool a0 = n < nelem && acc[prob ? prob[n] : 0];
  const bool a1 = n + 1 < nelem && acc[prob ? prob[n + 1] : 0];
  if (a0 && a1) {
    *reinterpret_cast<double2 *>(u + i) = *reinterpret_cast<const double2 *>(y + i);
    *reinterpret_cast<double2 *>(k1 + i) = *reinterpret_cast<const double2 *>(k7 + i);
  } else {
    if (a0) { u[i] = y[i]; k1[i] = k7[i]; }
    if (a1) { u[i + 1] = y[i + 1]; k1[i + 1] = k7[i + 1]; }
  }
}

hipError_t launch_dp_commit(int64_t len, int64_t ld, int64_t nelem, const int32_t *prob,
                            const int32_t *acc, const double *y, const double *k7, double *u,
                            double *k1, hipStream_t s) {
  if (len <= 0) return hipSuccess;
  if (len % 2 || ld % 2) return hipErrorInvalidValue;
  const int64_t len2 = len / 2;
  dp_commit_kernel<<<nblk(len2), 256, 0, s>>>(len2, ld, nelem, prob, acc, y, k7, u, k1);
  return hipGetLastError();
}

__global__ void dp_clamp_kernel(int nprob, const double *t, const double *tend, double *dt) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < nprob) dt[p] = fmin(dt[p], tend[p] - t[p]);
}

hipError_t launch_dp_clamp(int nprob, const double *t, const double *tend, double *dt,
                           hipStream_t s) {
  if (nprob <= 0 || !tend) return hipSuccess;
  dp_clamp_kernel<<<nblk(nprob), 256, 0, s>>>(nprob, t, tend, dt);
  return hipGetLastError();
}

}  // namespace fr
