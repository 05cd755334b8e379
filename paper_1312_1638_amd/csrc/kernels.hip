// HIP kernels of the FR right-hand side for gfx950 (CDNA4).
//
//  * Operator products (Appendix A) live in gemm.h / gemm_*.hip.
//  * Point-wise kernels (gradient transform, transformed flux) are one thread
//    per (solution point, element): every access is a unit-stride row of the
//    SoA state, so a wavefront reads 64 consecutive elements.
//  * Interface kernels are one thread per flux-point pair (each pair visited
//    once, same value to both sides), with pair constants stored in pair
//    order and pairs sorted by their left flux point, so the left side and
//    the constants are coalesced; workgroups are remapped so that each XCD
//    processes a contiguous range of pairs.
#include "kernels.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "physics.h"

namespace fr {

// ============================================================================
// Point-wise kernels
// ============================================================================
template <int D, typename TQ>
__global__ __launch_bounds__(256) void gradcoru_kernel(PointArgs a) {
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
  TQ *q = (TQ *)a.q;
  const int64_t rowstride = (int64_t)NV * a.ld, cstride = (int64_t)a.nupts * rowstride;
  const int64_t base = r * rowstride + n;
#pragma unroll
  for (int al = 0; al < NV; ++al) {
    double qt[D];
#pragma unroll
    for (int i = 0; i < D; ++i) qt[i] = (double)q[i * cstride + base + al * a.ld];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double s = 0;
#pragma unroll
      for (int i = 0; i < D; ++i) s += S[i][j] * qt[i];
      q[j * cstride + base + al * a.ld] = (TQ)(rj * s);
    }
  }
}

// Deviation form (Navier-Stokes): u - u_ref at every solution point and the
// element's reference state u_ref (its first solution point) at point 0.
template <int NV, typename TQ>
__global__ __launch_bounds__(256) void devstate_kernel(PointArgs a) {
  const int64_t plane = (int64_t)a.nupts * a.ld;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= plane) return;
  const int64_t r = t / a.ld, n = t - r * a.ld;
  if (n >= a.nelem) return;
  const int64_t base = r * NV * a.ld + n;
  TQ *ud = (TQ *)a.udev;
#pragma unroll
  for (int al = 0; al < NV; ++al) {
    const double ub = a.u[n + al * a.ld];
    ud[base + al * a.ld] = (TQ)(a.u[base + al * a.ld] - ub);
    if (r == 0) a.uref[al * a.ld + n] = ub;
  }
}

// MULTI: a multi-block launch (each workgroup's block from a.slots), a
// separate instantiation so that the slot loads, which count as divergent,
// stay out of the single-block kernel.
template <int D, int NS, typename TQ, bool MULTI = false>
__global__ __launch_bounds__(256) void tflux_kernel(PointArgs a) {
  constexpr int NV = D + 2;
  int64_t wg = blockIdx.x;
  if constexpr (MULTI) {
    // multi-block launch: this workgroup's block and its index within it
    int k = 0;
    while (k + 1 < a.nslots && wg >= a.slots[k + 1].wg_begin) ++k;
    const PointSlot &sl = a.slots[k];
    wg -= sl.wg_begin;
    a.u += sl.off_u;
    a.q = (TQ *)a.q + sl.off_q;
    if (a.fout) a.fout = (TQ *)a.fout + sl.off_q;
    if (a.udev) {
      a.udev = (TQ *)a.udev + sl.off_u;
      a.uref += sl.off_ref;
    }
    a.nupts = sl.nupts; a.ld = sl.ld; a.nelem = sl.nelem;
    a.smat = sl.smat; a.rcpdjac = sl.rcpdjac;
  }
  const int64_t plane = (int64_t)a.nupts * a.ld;
  const int64_t t = wg * 256 + threadIdx.x;
  if (t >= plane) return;
  const int64_t r = t / a.ld, n = t - r * a.ld;
  if (n >= a.nelem) return;
  const int64_t rowstride = (int64_t)NV * a.ld, cstride = (int64_t)a.nupts * rowstride;
  const int64_t base = r * rowstride + n;
  double u[NV];
#pragma unroll
  for (int al = 0; al < NV; ++al) u[al] = a.u[base + al * a.ld];
  TQ *q = (TQ *)a.q;
  TQ *qo = a.fout ? (TQ *)a.fout : q;
  double f[D][NV], p, v[D];
  inviscid_flux<D>(u, a.gamma, f, p, v);
  if (a.udev) {
    // deviation form: the element's reference state (its first solution
    // point); F~ from f(u) - f(u_ref) (the inviscid flux of the reference:
    // its viscous flux is zero); Euler also writes u - u_ref for the
    // interpolation here (Navier-Stokes writes it in a pass of its own
    // before step 1, which needs it before any flux)
    double ub[NV], fb[D][NV], pb, vb[D];
#pragma unroll
    for (int al = 0; al < NV; ++al) ub[al] = a.u[n + al * a.ld];
    inviscid_flux<D>(ub, a.gamma, fb, pb, vb);
    if (!NS) {
      TQ *ud = (TQ *)a.udev;
#pragma unroll
      for (int al = 0; al < NV; ++al) {
        ud[base + al * a.ld] = (TQ)(u[al] - ub[al]);
        if (r == 0) a.uref[al * a.ld + n] = ub[al];
      }
    }
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int al = 0; al < NV; ++al) f[j][al] -= fb[j][al];
  }
  if (NS) {
    double g[D][NV], fv[D][NV];
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int al = 0; al < NV; ++al) g[j][al] = (double)q[j * cstride + base + al * a.ld];
    viscous_flux<D>(u, g, a.gamma, a.mu, a.prandtl, fv);
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int al = 0; al < NV; ++al) f[j][al] -= fv[j][al];
  }
  double S[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) S[i][j] = a.smat[(i * D + j) * plane + t];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int al = 0; al < NV; ++al) {
      double s = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) s += S[i][j] * f[j][al];
      qo[i * cstride + base + al * a.ld] = (TQ)s;
    }
}

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename TQ>
static hipError_t gradcoru_t(const PointArgs &a, hipStream_t s) {
  unsigned nb = blocks_for((int64_t)a.nupts * a.ld);
  if (a.ndims == 2) gradcoru_kernel<2, TQ><<<nb, 256, 0, s>>>(a);
  else gradcoru_kernel<3, TQ><<<nb, 256, 0, s>>>(a);
  return hipGetLastError();
}
hipError_t launch_gradcoru(const PointArgs &a, hipStream_t s) {
  return a.q_f32 ? gradcoru_t<float>(a, s) : gradcoru_t<double>(a, s);
}

template <typename TQ, bool MULTI>
static hipError_t tflux_m(const PointArgs &a, int ns, unsigned nb, hipStream_t s) {
  if (a.ndims == 2) {
    if (ns) tflux_kernel<2, 1, TQ, MULTI><<<nb, 256, 0, s>>>(a);
    else tflux_kernel<2, 0, TQ, MULTI><<<nb, 256, 0, s>>>(a);
  } else {
    if (ns) tflux_kernel<3, 1, TQ, MULTI><<<nb, 256, 0, s>>>(a);
    else tflux_kernel<3, 0, TQ, MULTI><<<nb, 256, 0, s>>>(a);
  }
  return hipGetLastError();
}
template <typename TQ>
static hipError_t tflux_t(const PointArgs &a, int ns, hipStream_t s) {
  if (a.slots) return tflux_m<TQ, true>(a, ns, (unsigned)a.nwg, s);
  return tflux_m<TQ, false>(a, ns, blocks_for((int64_t)a.nupts * a.ld), s);
}
hipError_t launch_devstate(const PointArgs &a, hipStream_t s) {
  if (!a.udev || !a.uref) return hipErrorInvalidValue;
  const unsigned nb = blocks_for((int64_t)a.nupts * a.ld);
  if (a.nvars == 4) devstate_kernel<4, float><<<nb, 256, 0, s>>>(a);
  else if (a.nvars == 5) devstate_kernel<5, float><<<nb, 256, 0, s>>>(a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_tflux(const PointArgs &a, int ns, hipStream_t s) {
  return a.q_f32 ? tflux_t<float>(a, ns, s) : tflux_t<double>(a, ns, s);
}

// ============================================================================
// Interface kernels
// ============================================================================
// Workgroup id remapped so that XCD x (which receives ids x, x+8, ...)
// processes the contiguous range [x*per, (x+1)*per) of pair workgroups.
__device__ __forceinline__ int64_t xcd_block(unsigned nreal) {
  const unsigned per = gridDim.x / 8;
  const unsigned b = blockIdx.x;
  const unsigned m = (b % 8) * per + b / 8;
  return m < nreal ? (int64_t)m : -1;
}

struct Side {
  int64_t base, ld, qbase, qstride, rbase;
};

template <bool MULTI>
__device__ __forceinline__ Side side_of(const PairArgs &a, const int32_t *blk, int64_t k,
                                        bool q) {
  Side s;
  if (MULTI) {
    const int b = blk[k];
    s.base = a.blk_ufbase[b];
    s.ld = a.blk_ld[b];
    s.qbase = q ? a.blk_qfbase[b] : 0;
    s.qstride = q ? a.blk_qstride[b] : 0;
    s.rbase = a.uref ? a.blk_refbase[b] : 0;
  } else {
    s.base = 0; s.ld = a.ld0; s.qbase = 0; s.qstride = a.qstride0; s.rbase = 0;
  }
  return s;
}

// Deviation form (reduced precision): the reference state of the
// element of flux point i (index sigma NV ld + n within its block) and the
// normal component of its flux, n . f(u_ref).
template <int D>
__device__ __forceinline__ void side_reference(const PairArgs &a, const Side &S, int64_t i,
                                               const double *n, double ub[D + 2],
                                               double fn[D + 2]) {
  constexpr int NV = D + 2;
  const double *r = a.uref + S.rbase + i % S.ld;
#pragma unroll
  for (int al = 0; al < NV; ++al) ub[al] = r[al * S.ld];
  double f[D][NV], p, v[D];
  inviscid_flux<D>(ub, a.gamma, f, p, v);
#pragma unroll
  for (int al = 0; al < NV; ++al) {
    double s = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) s += n[d] * f[d][al];
    fn[al] = s;
  }
}

// Deviation form: the reference state of the element of flux point i.
template <int D>
__device__ __forceinline__ void side_state(const PairArgs &a, const Side &S, int64_t i,
                                           double ub[D + 2]) {
  const double *r = a.uref + S.rbase + i % S.ld;
#pragma unroll
  for (int al = 0; al < D + 2; ++al) ub[al] = r[al * S.ld];
}

template <int D, bool MULTI, typename T>
__global__ __launch_bounds__(256) void con_u_kernel(PairArgs a, unsigned nreal) {
  constexpr int NV = D + 2;
  const int64_t wg = xcd_block(nreal);
  if (wg < 0) return;
  const int64_t k = wg * 256 + threadIdx.x;
  if (k >= a.npairs) return;
  const Side L = side_of<MULTI>(a, a.lblk, k, true), R = side_of<MULTI>(a, a.rblk, k, true);
  const int64_t iL = a.lidx[k], iR = a.ridx[k];
  const T *uf = (const T *)a.uf;
  T *cf = (T *)a.cf;
  const double wl = 0.5 - a.beta, wr = 0.5 + a.beta;
  // deviation form: U^f holds each side's deviation from its element's
  // reference; the common solution is formed from the full states and
  // stored on each side as that side's deviation
  double rL[NV] = {}, rR[NV] = {};
  if (a.uref) {
    side_state<D>(a, L, iL, rL);
    side_state<D>(a, R, iR, rR);
  }
#pragma unroll
  for (int al = 0; al < NV; ++al) {
    const double c = wl * ((double)uf[L.base + iL + al * L.ld] + rL[al]) +
                     wr * ((double)uf[R.base + iR + al * R.ld] + rR[al]);
    cf[L.qbase + iL + al * L.ld] = (T)(c - rL[al]);
    cf[R.qbase + iR + al * R.ld] = (T)(c - rR[al]);
  }
}

template <int D, int NS, bool MULTI, typename T>
__global__ __launch_bounds__(256) void comm_flux_kernel(PairArgs a, unsigned nreal) {
  constexpr int NV = D + 2;
  const int64_t wg = xcd_block(nreal);
  if (wg < 0) return;
  const int64_t k = wg * 256 + threadIdx.x;
  if (k >= a.npairs) return;
  const Side L = side_of<MULTI>(a, a.lblk, k, NS), R = side_of<MULTI>(a, a.rblk, k, NS);
  const int64_t iL = a.lidx[k], iR = a.ridx[k];
  T *uf = (T *)a.uf;
  double uL[NV], uR[NV], n[D], F[NV];
#pragma unroll
  for (int al = 0; al < NV; ++al) {
    uL[al] = (double)uf[L.base + iL + al * L.ld];
    uR[al] = (double)uf[R.base + iR + al * R.ld];
  }
#pragma unroll
  for (int d = 0; d < D; ++d) n[d] = a.nrm[d * a.npairs + k];
  double fnL[NV], fnR[NV];
  const bool dev = a.uref != nullptr;
  if (dev) {
    double ub[NV];
    side_reference<D>(a, L, iL, n, ub, fnL);
#pragma unroll
    for (int al = 0; al < NV; ++al) uL[al] += ub[al];
    side_reference<D>(a, R, iR, n, ub, fnR);
#pragma unroll
    for (int al = 0; al < NV; ++al) uR[al] += ub[al];
  }
  rusanov<D>(uL, uR, n, a.gamma, F);
  if (NS) {
    const T *qf = (const T *)a.qf;
    double qL[D][NV], qR[D][NV], fvL[D][NV], fvR[D][NV];
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int al = 0; al < NV; ++al) {
        qL[j][al] = (double)qf[L.qbase + j * L.qstride + iL + al * L.ld];
        qR[j][al] = (double)qf[R.qbase + j * R.qstride + iR + al * R.ld];
      }
    viscous_flux<D>(uL, qL, a.gamma, a.mu, a.prandtl, fvL);
    viscous_flux<D>(uR, qR, a.gamma, a.mu, a.prandtl, fvR);
    const double wl = 0.5 + a.beta, wr = 0.5 - a.beta;
#pragma unroll
    for (int al = 0; al < NV; ++al) {
      double fv = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) fv += n[j] * (wl * fvL[j][al] + wr * fvR[j][al]);
      F[al] = F[al] - fv + a.tau * (uL[al] - uR[al]);
    }
  }
  const double mL = a.magL[k], mR = a.magR[k];
  T *df = a.dfout ? (T *)a.dfout : uf;
#pragma unroll
  for (int al = 0; al < NV; ++al) {
    // deviation form: each side less its reference's own normal flux
    df[L.base + iL + al * L.ld] = (T)(mL * (dev ? F[al] - fnL[al] : F[al]));
    df[R.base + iR + al * R.ld] = (T)(-mR * (dev ? F[al] - fnR[al] : F[al]));
  }
}

// Boundary flux points: the common solution (from the ghost of the LDG
// terms) and the common normal flux (inviscid ghost in the Rusanov flux, LDG
// ghost and ghost gradient in the viscous flux and penalty), with the
// boundary element as the L side.
template <int D, bool MULTI, typename T>
__global__ __launch_bounds__(256) void bc_con_u_kernel(PairArgs a) {
  constexpr int NV = D + 2;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= a.npairs) return;
  const Side L = side_of<MULTI>(a, a.lblk, k, true);
  const int64_t i = a.lidx[k];
  const T *uf = (const T *)a.uf;
  T *cf = (T *)a.cf;
  double u[NV], ginv[NV], gldg[NV], rL[NV] = {};
  // deviation form: the full state for the ghosts, the common solution
  // stored as the deviation from the element's reference
  if (a.uref) side_state<D>(a, L, i, rL);
#pragma unroll
  for (int al = 0; al < NV; ++al) u[al] = (double)uf[L.base + i + al * L.ld] + rL[al];
  bool qzero;
  bc_ghosts<D>(u, a.bcpar + (int64_t)a.bcid[k] * FR_BC_NPAR, a.gamma, ginv, gldg, qzero);
  const double wl = 0.5 - a.beta, wr = 0.5 + a.beta;
#pragma unroll
  for (int al = 0; al < NV; ++al)
    cf[L.qbase + i + al * L.ld] = (T)(wl * u[al] + wr * gldg[al] - rL[al]);
}

template <int D, int NS, bool MULTI, typename T>
__global__ __launch_bounds__(256) void bc_comm_flux_kernel(PairArgs a) {
  constexpr int NV = D + 2;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= a.npairs) return;
  const Side L = side_of<MULTI>(a, a.lblk, k, NS);
  const int64_t i = a.lidx[k];
  T *uf = (T *)a.uf;
  double u[NV], ginv[NV], gldg[NV], n[D], F[NV];
#pragma unroll
  for (int al = 0; al < NV; ++al) u[al] = (double)uf[L.base + i + al * L.ld];
#pragma unroll
  for (int d = 0; d < D; ++d) n[d] = a.nrm[d * a.npairs + k];
  double fn[NV];
  const bool dev = a.uref != nullptr;
  if (dev) {
    double ub[NV];
    side_reference<D>(a, L, i, n, ub, fn);
#pragma unroll
    for (int al = 0; al < NV; ++al) u[al] += ub[al];
  }
  bool qzero;
  bc_ghosts<D>(u, a.bcpar + (int64_t)a.bcid[k] * FR_BC_NPAR, a.gamma, ginv, gldg, qzero);
  rusanov<D>(u, ginv, n, a.gamma, F);
  if (NS) {
    const T *qf = (const T *)a.qf;
    double qL[D][NV], qR[D][NV], fvL[D][NV], fvR[D][NV];
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int al = 0; al < NV; ++al) {
        qL[j][al] = (double)qf[L.qbase + j * L.qstride + i + al * L.ld];
        qR[j][al] = qzero ? 0.0 : qL[j][al];
      }
    viscous_flux<D>(u, qL, a.gamma, a.mu, a.prandtl, fvL);
    viscous_flux<D>(gldg, qR, a.gamma, a.mu, a.prandtl, fvR);
    const double wl = 0.5 + a.beta, wr = 0.5 - a.beta;
#pragma unroll
    for (int al = 0; al < NV; ++al) {
      double fv = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) fv += n[j] * (wl * fvL[j][al] + wr * fvR[j][al]);
      F[al] = F[al] - fv + a.tau * (u[al] - gldg[al]);
    }
  }
  const double m = a.magL[k];
  T *df = a.dfout ? (T *)a.dfout : uf;
#pragma unroll
  for (int al = 0; al < NV; ++al) df[L.base + i + al * L.ld] = (T)(m * (dev ? F[al] - fn[al] : F[al]));
}

template <typename T>
static hipError_t bc_con_u_t(const PairArgs &a, hipStream_t s) {
  const unsigned grid = (unsigned)((a.npairs + 255) / 256);
  const bool multi = a.lblk != nullptr;
  if (a.ndims == 2) {
    if (multi) bc_con_u_kernel<2, true, T><<<grid, 256, 0, s>>>(a);
    else bc_con_u_kernel<2, false, T><<<grid, 256, 0, s>>>(a);
  } else {
    if (multi) bc_con_u_kernel<3, true, T><<<grid, 256, 0, s>>>(a);
    else bc_con_u_kernel<3, false, T><<<grid, 256, 0, s>>>(a);
  }
  return hipGetLastError();
}
hipError_t launch_bc_con_u(const PairArgs &a, hipStream_t s) {
  if (a.npairs <= 0) return hipSuccess;
  return a.uf_f32 ? bc_con_u_t<float>(a, s) : bc_con_u_t<double>(a, s);
}

template <typename T, int NS>
static void bc_comm_flux_go(const PairArgs &a, hipStream_t s) {
  const unsigned grid = (unsigned)((a.npairs + 255) / 256);
  const bool multi = a.lblk != nullptr;
  if (a.ndims == 2) {
    if (multi) bc_comm_flux_kernel<2, NS, true, T><<<grid, 256, 0, s>>>(a);
    else bc_comm_flux_kernel<2, NS, false, T><<<grid, 256, 0, s>>>(a);
  } else {
    if (multi) bc_comm_flux_kernel<3, NS, true, T><<<grid, 256, 0, s>>>(a);
    else bc_comm_flux_kernel<3, NS, false, T><<<grid, 256, 0, s>>>(a);
  }
}
hipError_t launch_bc_comm_flux(const PairArgs &a, int ns, hipStream_t s) {
  if (a.npairs <= 0) return hipSuccess;
  if (a.uf_f32) {
    if (ns) bc_comm_flux_go<float, 1>(a, s); else bc_comm_flux_go<float, 0>(a, s);
  } else {
    if (ns) bc_comm_flux_go<double, 1>(a, s); else bc_comm_flux_go<double, 0>(a, s);
  }
  return hipGetLastError();
}

static void pair_grid(int64_t npairs, unsigned &grid, unsigned &nreal) {
  nreal = (unsigned)((npairs + 255) / 256);
  grid = (nreal + 7) / 8 * 8;
}

template <typename T>
static hipError_t con_u_t(const PairArgs &a, hipStream_t s) {
  unsigned grid, nreal;
  pair_grid(a.npairs, grid, nreal);
  const bool multi = a.lblk != nullptr;
  if (a.ndims == 2) {
    if (multi) con_u_kernel<2, true, T><<<grid, 256, 0, s>>>(a, nreal);
    else con_u_kernel<2, false, T><<<grid, 256, 0, s>>>(a, nreal);
  } else {
    if (multi) con_u_kernel<3, true, T><<<grid, 256, 0, s>>>(a, nreal);
    else con_u_kernel<3, false, T><<<grid, 256, 0, s>>>(a, nreal);
  }
  return hipGetLastError();
}
hipError_t launch_con_u(const PairArgs &a, hipStream_t s) {
  if (a.npairs <= 0) return hipSuccess;
  return a.uf_f32 ? con_u_t<float>(a, s) : con_u_t<double>(a, s);
}

template <typename T>
static hipError_t comm_flux_t(const PairArgs &a, int ns, hipStream_t s) {
  unsigned grid, nreal;
  pair_grid(a.npairs, grid, nreal);
  const bool multi = a.lblk != nullptr;
#define FR_CF(D_, NS_)                                                                    \
  if (multi) comm_flux_kernel<D_, NS_, true, T><<<grid, 256, 0, s>>>(a, nreal);           \
  else comm_flux_kernel<D_, NS_, false, T><<<grid, 256, 0, s>>>(a, nreal);
  if (a.ndims == 2) {
    if (ns) { FR_CF(2, 1) } else { FR_CF(2, 0) }
  } else {
    if (ns) { FR_CF(3, 1) } else { FR_CF(3, 0) }
  }
#undef FR_CF
  return hipGetLastError();
}
hipError_t launch_comm_flux(const PairArgs &a, int ns, hipStream_t s) {
  if (a.npairs <= 0) return hipSuccess;
  return a.uf_f32 ? comm_flux_t<float>(a, ns, s) : comm_flux_t<double>(a, ns, s);
}

// ============================================================================
// Reductions (FP64, fixed summation order)
// ============================================================================
// Per-element integrals: a workgroup takes 64 elements; its 4 waves split
// the solution points (rho = wave, wave + 4, ...) and combine in LDS in a
// fixed order.  part[n][c]: c < nvars the field integrals, c = nvars the
// kinetic energy.
// Per-element quadrature of every conserved field and of the kinetic energy
// 0.5 |m|^2 / rho.  Workgroup: 64 elements x 4 waves; blockIdx.y splits the
// solution points into `nchunk` ranges (enough workgroups for small meshes).
// Partials go to part[(chunk * (nvars + 1) + c) * pstride + n].
__global__ __launch_bounds__(256) void elem_integrals_kernel(int nvars, int ndims, int nupts,
                                                             int64_t ld, int64_t nelem,
                                                             int64_t pstride,
                                                             const double *wdjac,
                                                             const double *u, double *part) {
  __shared__ double red[4][6][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t n = (int64_t)blockIdx.x * 64 + tx;
  const int rc = (nupts + (int)gridDim.y - 1) / (int)gridDim.y;
  const int rbeg = (int)blockIdx.y * rc, rend = rbeg + rc < nupts ? rbeg + rc : nupts;
  double s[6] = {0, 0, 0, 0, 0, 0};
  if (n < nelem) {
    for (int r = rbeg + ty; r < rend; r += 4) {
      const double w = wdjac[(int64_t)r * ld + n];
      const double *ur = u + (int64_t)r * nvars * ld + n;
      double m2 = 0;
      for (int al = 0; al < nvars; ++al) {
        const double v = ur[al * ld];
        s[al] += w * v;
        if (al >= 1 && al <= ndims) m2 += v * v;
      }
      s[nvars] += w * 0.5 * m2 / ur[0];
    }
  }
  for (int c = 0; c <= nvars; ++c) red[ty][c][tx] = s[c];
  __syncthreads();
  if (ty == 0 && n < nelem)
    for (int c = 0; c <= nvars; ++c)
      part[((int64_t)blockIdx.y * (nvars + 1) + c) * pstride + n] =
          (red[0][c][tx] + red[1][c][tx]) + (red[2][c][tx] + red[3][c][tx]);
}

hipError_t launch_elem_integrals(int nvars, int ndims, int nupts, int64_t ld, int64_t nelem,
                                 int nchunk, int64_t pstride, const double *wdjac,
                                 const double *u, double *part, hipStream_t s) {
  if (nelem <= 0) return hipSuccess;
  dim3 grid((unsigned)((nelem + 63) / 64), (unsigned)nchunk);
  elem_integrals_kernel<<<grid, 256, 0, s>>>(nvars, ndims, nupts, ld, nelem, pstride, wdjac, u,
                                             part);
  return hipGetLastError();
}

// Per-problem sums of the element partials.  Workgroup (problem, slice):
// `per` (a multiple of 64) consecutive entries of the problem's element list,
// 64 lanes across entries x 4 waves that split
// the point ranges, then a fixed-shape LDS tree; a second kernel adds the
// slice sums of each problem with another fixed-shape tree (bitwise
// reproducible for a given mesh).
template <int NC>
__global__ __launch_bounds__(256) void problem_sums_kernel(int nchunk, int64_t pstride,
                                                           int64_t per,
                                                           const int64_t *pstart,
                                                           const int64_t *plist,
                                                           const double *part, double *out) {
  __shared__ double red[NC][256];
  const int prob = blockIdx.x, nslice = gridDim.y, slice = blockIdx.y;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t b = pstart[prob], e = pstart[prob + 1];
  const int64_t lo = b + (int64_t)slice * per;
  const int64_t hi = lo + per < e ? lo + per : e;
  double s[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) s[c] = 0;
  for (int64_t i = lo + tx; i < hi; i += 64) {
    const int64_t el = plist[i];
    for (int ch = ty; ch < nchunk; ch += 4)
#pragma unroll
      for (int c = 0; c < NC; ++c) s[c] += part[((int64_t)ch * NC + c) * pstride + el];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) red[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int c = 0; c < NC; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if ((int)threadIdx.x < NC)
    out[((int64_t)prob * nslice + slice) * NC + threadIdx.x] = red[threadIdx.x][0];
}

template <int NC>
__global__ __launch_bounds__(256) void slice_sums_kernel(int nslice, const double *part2,
                                                         double *out) {
  __shared__ double red[NC][256];
  const int prob = blockIdx.x;
  double s[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) s[c] = 0;
  for (int sl = threadIdx.x; sl < nslice; sl += 256)
#pragma unroll
    for (int c = 0; c < NC; ++c) s[c] += part2[((int64_t)prob * nslice + sl) * NC + c];
#pragma unroll
  for (int c = 0; c < NC; ++c) red[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int c = 0; c < NC; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if ((int)threadIdx.x < NC) out[(int64_t)prob * NC + threadIdx.x] = red[threadIdx.x][0];
}

template <int NC>
static void problem_sums_t(int nprob, int nchunk, int64_t pstride, int nslice, int64_t per,
                           const int64_t *pstart, const int64_t *plist, const double *part,
                           double *part2, double *out, hipStream_t s) {
  dim3 grid((unsigned)nprob, (unsigned)nslice);
  problem_sums_kernel<NC><<<grid, 256, 0, s>>>(nchunk, pstride, per, pstart, plist, part,
                                               nslice == 1 ? out : part2);
  if (nslice > 1) slice_sums_kernel<NC><<<nprob, 256, 0, s>>>(nslice, part2, out);
}

hipError_t launch_problem_sums(int ncomp, int nprob, int nchunk, int64_t pstride, int nslice,
                               int64_t per, const int64_t *pstart, const int64_t *plist,
                               const double *part, double *part2, double *out, hipStream_t s) {
  if (per < 64 || per % 64 || nslice < 1) return hipErrorInvalidValue;
  if (ncomp == 1)
    problem_sums_t<1>(nprob, nchunk, pstride, nslice, per, pstart, plist, part, part2, out, s);
  else if (ncomp == 5)
    problem_sums_t<5>(nprob, nchunk, pstride, nslice, per, pstart, plist, part, part2, out, s);
  else if (ncomp == 6)
    problem_sums_t<6>(nprob, nchunk, pstride, nslice, per, pstart, plist, part, part2, out, s);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Fixed scratch of the integrals for callers that cannot allocate: a static
// device array, one copy per GPU, held until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is a stand-in,
// not a device address); it passes the address that hipGetSymbolAddress
// returns for the current device, resolved once per device and kept here.
static __device__ __align__(256) double scratch[kIntegralScratchDoubles];

hipError_t integral_scratch(double **ptr) {
  static std::mutex mu;
  static std::map<int, double *> addr;  // device ordinal -> address of its copy
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    it = addr.emplace(dev, static_cast<double *>(p)).first;
  }
  *ptr = it->second;
  return hipSuccess;
}

__global__ __launch_bounds__(256) void check_finite_kernel(const double *u, int64_t n,
                                                           int32_t *flag) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    if (!isfinite(u[i])) flag[0] = 1;
}

hipError_t launch_check_finite(const double *u, int64_t n, int32_t *flag, hipStream_t s) {
  unsigned nb = (unsigned)std::min<int64_t>(4096, (n + 255) / 256);
  if (nb == 0) return hipSuccess;
  check_finite_kernel<<<nb, 256, 0, s>>>(u, n, flag);
  return hipGetLastError();
}

}  // namespace fr
