// Kernels of the hand-written adjoint (vector-Jacobian product) of the FR
// right-hand side, and the RK4 register arithmetic of the step adjoint.
// Reverse order of the forward chain; every flux point belongs to exactly
// one pair, so the pair kernels write both sides without atomics.
#include "adjoint.h"
#include "physics.h"

namespace fr {

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// lt = -J^-1 lam at solution points (0 in padding columns)
__global__ __launch_bounds__(256) void negscale_kernel(int nvars, int nupts, int64_t ld,
                                                       int64_t nelem, const double *rcpdjac,
                                                       const double *lam, double *lt) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)nupts * ld) return;
  const int64_t r = t / ld, n = t - r * ld;
  const double s = n < nelem ? -rcpdjac[t] : 0.0;
  for (int a = 0; a < nvars; ++a) {
    const int64_t i = (r * nvars + a) * ld + n;
    lt[i] = n < nelem ? s * lam[i] : 0.0;
  }
}

hipError_t launch_negscale(int nvars, int nupts, int64_t ld, int64_t nelem, const double *rcpdjac,
                           const double *lam, double *lt, hipStream_t s) {
  negscale_kernel<<<nblk((int64_t)nupts * ld), 256, 0, s>>>(nvars, nupts, ld, nelem, rcpdjac, lam,
                                                            lt);
  return hipGetLastError();
}

// Point-wise reverse of the transformed flux: fb_j = sum_i S_ij Fb_i, then
// ub = (df/du)^T fb written to ulam, qb = (df/dq)^T fb over Fb's storage.
template <int D, int NS>
__global__ __launch_bounds__(256) void tflux_vjp_kernel(AdjPointArgs a) {
  constexpr int NV = D + 2;
  const int64_t plane = (int64_t)a.nupts * a.ld;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= plane) return;
  const int64_t r = t / a.ld, n = t - r * a.ld;
  const int64_t rowstride = (int64_t)NV * a.ld, cstride = (int64_t)a.nupts * rowstride;
  const int64_t base = r * rowstride + n;
  if (n >= a.nelem) {
#pragma unroll
    for (int al = 0; al < NV; ++al) a.ulam[base + al * a.ld] = 0.0;
    return;
  }
  double u[NV], Fb[D][NV], fb[D][NV], ub[NV];
#pragma unroll
  for (int al = 0; al < NV; ++al) { u[al] = a.u[base + al * a.ld]; ub[al] = 0; }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int al = 0; al < NV; ++al) Fb[i][al] = a.fb[i * cstride + base + al * a.ld];
  double S[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) S[i][j] = a.smat[(i * D + j) * plane + t];
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int al = 0; al < NV; ++al) {
      double s = 0;
#pragma unroll
      for (int i = 0; i < D; ++i) s += S[i][j] * Fb[i][al];
      fb[j][al] = s;
    }
  inviscid_flux_vjp<D>(u, a.gamma, fb, 0.0, nullptr, ub);
  if (NS) {
    double q[D][NV], qb[D][NV], nfb[D][NV];
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int al = 0; al < NV; ++al) {
        q[j][al] = a.q[j * cstride + base + al * a.ld];
        qb[j][al] = 0;
        nfb[j][al] = -fb[j][al];
      }
    viscous_flux_vjp<D>(u, q, a.gamma, a.mu, a.prandtl, nfb, ub, qb);
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int al = 0; al < NV; ++al) a.fb[j * cstride + base + al * a.ld] = qb[j][al];
  }
#pragma unroll
  for (int al = 0; al < NV; ++al) a.ulam[base + al * a.ld] = ub[al];
}

hipError_t launch_tflux_vjp(const AdjPointArgs &a, int ns, hipStream_t s) {
  const unsigned nb = nblk((int64_t)a.nupts * a.ld);
  if (a.ndims == 2) {
    if (ns) tflux_vjp_kernel<2, 1><<<nb, 256, 0, s>>>(a);
    else tflux_vjp_kernel<2, 0><<<nb, 256, 0, s>>>(a);
  } else {
    if (ns) tflux_vjp_kernel<3, 1><<<nb, 256, 0, s>>>(a);
    else tflux_vjp_kernel<3, 0><<<nb, 256, 0, s>>>(a);
  }
  return hipGetLastError();
}

// Reverse of the gradient transform q_j = r sum_i S_ij qt_i: qtb_i = r sum_j S_ij qb_j
template <int D>
__global__ __launch_bounds__(256) void gradcoru_t_kernel(AdjPointArgs a) {
  constexpr int NV = D + 2;
  const int64_t plane = (int64_t)a.nupts * a.ld;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= plane) return;
  const int64_t r = t / a.ld, n = t - r * a.ld;
  if (n >= a.nelem) return;
  double S[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) S[i][j] = a.smat[(i * D + j) * plane + t];
  const double rj = a.rcpdjac[t];
  const int64_t rowstride = (int64_t)NV * a.ld, cstride = (int64_t)a.nupts * rowstride;
  const int64_t base = r * rowstride + n;
#pragma unroll
  for (int al = 0; al < NV; ++al) {
    double qb[D];
#pragma unroll
    for (int j = 0; j < D; ++j) qb[j] = a.fb[j * cstride + base + al * a.ld];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double s = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) s += S[i][j] * qb[j];
      a.fb[i * cstride + base + al * a.ld] = rj * s;
    }
  }
}

hipError_t launch_gradcoru_t(const AdjPointArgs &a, hipStream_t s) {
  const unsigned nb = nblk((int64_t)a.nupts * a.ld);
  if (a.ndims == 2) gradcoru_t_kernel<2><<<nb, 256, 0, s>>>(a);
  else gradcoru_t_kernel<3><<<nb, 256, 0, s>>>(a);
  return hipGetLastError();
}

struct SideA {
  int64_t base, ld, qbase, qstride;
};

template <bool MULTI>
__device__ __forceinline__ SideA side_a(const AdjPairArgs &a, const int32_t *blk, int64_t k) {
  SideA s;
  if (MULTI) {
    const int b = blk[k];
    s.base = a.blk_ufbase[b]; s.ld = a.blk_ld[b];
    s.qbase = a.blk_qfbase ? a.blk_qfbase[b] : 0;
    s.qstride = a.blk_qstride ? a.blk_qstride[b] : 0;
  } else {
    s.base = 0; s.ld = a.ld0; s.qbase = 0; s.qstride = a.qstride0;
  }
  return s;
}

// Reverse of the common normal flux: Fb = mL D~b_L - mR D~b_R, then
// (uLb, uRb, qLb, qRb) = (dF/d.)^T Fb, written over D~b (U^f shaped) and into
// Q^f-shaped qfb.
template <int D, int NS, bool MULTI>
__global__ __launch_bounds__(256) void comm_flux_vjp_kernel(AdjPairArgs a) {
  constexpr int NV = D + 2;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= a.npairs) return;
  const SideA L = side_a<MULTI>(a, a.lblk, k), R = side_a<MULTI>(a, a.rblk, k);
  const int64_t iL = a.lidx[k], iR = a.ridx[k];
  double uL[NV], uR[NV], n[D], Fb[NV], uLb[NV], uRb[NV];
  const double mL = a.magL[k], mR = a.magR[k];
#pragma unroll
  for (int al = 0; al < NV; ++al) {
    uL[al] = a.uf[L.base + iL + al * L.ld];
    uR[al] = a.uf[R.base + iR + al * R.ld];
    Fb[al] = mL * a.ufb[L.base + iL + al * L.ld] - mR * a.ufb[R.base + iR + al * R.ld];
    uLb[al] = 0;
    uRb[al] = 0;
  }
#pragma unroll
  for (int d = 0; d < D; ++d) n[d] = a.nrm[d * a.npairs + k];
  rusanov_vjp<D>(uL, uR, n, a.gamma, Fb, uLb, uRb);
  if (NS) {
    double qL[D][NV], qR[D][NV], qLb[D][NV], qRb[D][NV], fvLb[D][NV], fvRb[D][NV];
    const double wl = 0.5 + a.beta, wr = 0.5 - a.beta;
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int al = 0; al < NV; ++al) {
        qL[j][al] = a.qf[L.qbase + j * L.qstride + iL + al * L.ld];
        qR[j][al] = a.qf[R.qbase + j * R.qstride + iR + al * R.ld];
        qLb[j][al] = 0;
        qRb[j][al] = 0;
        fvLb[j][al] = -n[j] * wl * Fb[al];
        fvRb[j][al] = -n[j] * wr * Fb[al];
      }
    viscous_flux_vjp<D>(uL, qL, a.gamma, a.mu, a.prandtl, fvLb, uLb, qLb);
    viscous_flux_vjp<D>(uR, qR, a.gamma, a.mu, a.prandtl, fvRb, uRb, qRb);
#pragma unroll
    for (int al = 0; al < NV; ++al) {
      uLb[al] += a.tau * Fb[al];
      uRb[al] -= a.tau * Fb[al];
    }
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int al = 0; al < NV; ++al) {
        a.qfb[L.qbase + j * L.qstride + iL + al * L.ld] = qLb[j][al];
        a.qfb[R.qbase + j * R.qstride + iR + al * R.ld] = qRb[j][al];
      }
  }
#pragma unroll
  for (int al = 0; al < NV; ++al) {
    a.ufb[L.base + iL + al * L.ld] = uLb[al];
    a.ufb[R.base + iR + al * R.ld] = uRb[al];
  }
}

hipError_t launch_comm_flux_vjp(const AdjPairArgs &a, int ns, hipStream_t s) {
  if (a.npairs <= 0) return hipSuccess;
  const unsigned nb = nblk(a.npairs);
  const bool multi = a.lblk != nullptr;
#define FR_CFV(D_, NS_)                                                        \
  if (multi) comm_flux_vjp_kernel<D_, NS_, true><<<nb, 256, 0, s>>>(a);         \
  else comm_flux_vjp_kernel<D_, NS_, false><<<nb, 256, 0, s>>>(a);
  if (a.ndims == 2) {
    if (ns) { FR_CFV(2, 1) } else { FR_CFV(2, 0) }
  } else {
    if (ns) { FR_CFV(3, 1) } else { FR_CFV(3, 0) }
  }
#undef FR_CFV
  return hipGetLastError();
}

// Reverse of the common solution: c = wl uL + wr uR was written to both
// sides, so s = Cb_L + Cb_R and uLb += wl s, uRb += wr s (into ufb).
template <int D, bool MULTI>
__global__ __launch_bounds__(256) void con_u_vjp_kernel(AdjPairArgs a) {
  constexpr int NV = D + 2;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= a.npairs) return;
  const SideA L = side_a<MULTI>(a, a.lblk, k), R = side_a<MULTI>(a, a.rblk, k);
  const int64_t iL = a.lidx[k], iR = a.ridx[k];
  const double wl = 0.5 - a.beta, wr = 0.5 + a.beta;
#pragma unroll
  for (int al = 0; al < NV; ++al) {
    const double s = a.qfb[L.qbase + iL + al * L.ld] + a.qfb[R.qbase + iR + al * R.ld];
    a.ufb[L.base + iL + al * L.ld] += wl * s;
    a.ufb[R.base + iR + al * R.ld] += wr * s;
  }
}

hipError_t launch_con_u_vjp(const AdjPairArgs &a, hipStream_t s) {
  if (a.npairs <= 0) return hipSuccess;
  const unsigned nb = nblk(a.npairs);
  const bool multi = a.lblk != nullptr;
  if (a.ndims == 2) {
    if (multi) con_u_vjp_kernel<2, true><<<nb, 256, 0, s>>>(a);
    else con_u_vjp_kernel<2, false><<<nb, 256, 0, s>>>(a);
  } else {
    if (multi) con_u_vjp_kernel<3, true><<<nb, 256, 0, s>>>(a);
    else con_u_vjp_kernel<3, false><<<nb, 256, 0, s>>>(a);
  }
  return hipGetLastError();
}

// out = x + c * dt[prob(n)] * y over a block's state (every row and field);
// y may be null (out = x).  Padding columns copy x.
__global__ __launch_bounds__(256) void axpy_dt_kernel(int64_t len, int64_t ld, int64_t nelem,
                                                      const int32_t *prob, const double *dt,
                                                      double c, const double *x, const double *y,
                                                      double *out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= len) return;
  const int64_t n = i % ld;
  double v = x[i];
  if (y && n < nelem) v += c * dt[prob ? prob[n] : 0] * y[i];
  out[i] = v;
}

hipError_t launch_axpy_dt(int64_t len, int64_t ld, int64_t nelem, const int32_t *prob,
                          const double *dt, double c, const double *x, const double *y,
                          double *out, hipStream_t s) {
  axpy_dt_kernel<<<nblk(len), 256, 0, s>>>(len, ld, nelem, prob, dt, c, x, y, out);
  return hipGetLastError();
}

// acc += w; kb = a dt lam + b dt w (RK4 step adjoint bookkeeping), kb
// optionally scaled by -1/J for the next right-hand-side adjoint, lam
// optionally copied (the step's first call, lam_{n+1} kept for later stages)
__global__ __launch_bounds__(256) void rk_adj_kernel(int64_t len, int64_t ld, int64_t nelem,
                                                     const int32_t *prob, const double *dt,
                                                     double ca, double cb, const double *lam,
                                                     const double *w, double *acc, double *kb,
                                                     int first, int nvars,
                                                     const double *rcpdjac, double *lcopy) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= len) return;
  const int64_t row = i / ld, n = i - row * ld;
  const bool live = n < nelem;
  const double d = live ? dt[prob ? prob[n] : 0] : 0.0;
  const double wi = first ? 0.0 : w[i];
  const double l = lam[i];
  if (lcopy) lcopy[i] = l;
  acc[i] = (first ? l : acc[i]) + wi;
  if (kb) {
    const double kv = ca * d * l + cb * d * wi;
    // row = point r times nvars plus the field
    kb[i] = !rcpdjac ? kv : live ? -rcpdjac[(row / nvars) * ld + n] * kv : 0.0;
  }
}

hipError_t launch_rk_adj(int64_t len, int64_t ld, int64_t nelem, const int32_t *prob,
                         const double *dt, double ca, double cb, const double *lam,
                         const double *w, double *acc, double *kb, int first, int nvars,
                         const double *rcpdjac, double *lcopy, hipStream_t s) {
  if (rcpdjac && nvars < 1) return hipErrorInvalidValue;
  rk_adj_kernel<<<nblk(len), 256, 0, s>>>(len, ld, nelem, prob, dt, ca, cb, lam, w, acc, kb,
                                          first, nvars, rcpdjac, lcopy);
  return hipGetLastError();
}

// d E_k / d u at every solution point, E_k = sum W J |m|^2 / (2 rho):
// (-W J |v|^2 / 2, W J v, 0); 0 in padding.
__global__ __launch_bounds__(256) void ke_grad_kernel(int nvars, int ndims, int nupts, int64_t ld,
                                                      int64_t nelem, const double *wdjac,
                                                      const double *u, double *g) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)nupts * ld) return;
  const int64_t r = t / ld, n = t - r * ld;
  const int64_t base = r * nvars * ld + n;
  if (n >= nelem) {
    for (int a = 0; a < nvars; ++a) g[base + a * ld] = 0.0;
    return;
  }
  const double w = wdjac[t];
  const double rho = u[base];
  double v2 = 0;
  for (int i = 0; i < ndims; ++i) {
    const double v = u[base + (1 + i) * ld] / rho;
    v2 += v * v;
    g[base + (1 + i) * ld] = w * v;
  }
  g[base] = -0.5 * w * v2;
  g[base + (ndims + 1) * ld] = 0.0;
}

hipError_t launch_ke_grad(int nvars, int ndims, int nupts, int64_t ld, int64_t nelem,
                          const double *wdjac, const double *u, double *g, hipStream_t s) {
  ke_grad_kernel<<<nblk((int64_t)nupts * ld), 256, 0, s>>>(nvars, ndims, nupts, ld, nelem, wdjac,
                                                           u, g);
  return hipGetLastError();
}

}  // namespace fr
