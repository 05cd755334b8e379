// Point-wise physics of the compressible Euler / Navier-Stokes equations
// (paper section 4, Appendix B) and their vector-Jacobian products, written
// by hand in reverse statement order.  Conserved variables u = (rho, rho v,
// E); gradients q[j][a] = d u_a / d x_j; fluxes f[j][a].
#pragma once

#include <hip/hip_runtime.h>

namespace fr {

template <int D>
__device__ __forceinline__ void primitives(const double *u, double gamma, double &rho, double *v,
                                           double &p) {
  rho = u[0];
  const double ir = 1.0 / rho;
  double ke = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) { v[i] = u[1 + i] * ir; ke += u[1 + i] * v[i]; }
  p = (gamma - 1.0) * (u[D + 1] - 0.5 * ke);
}

// reverse of primitives: given pb and vb[D], accumulate into ub
template <int D>
__device__ __forceinline__ void primitives_vjp(const double *u, double gamma, double pb,
                                               const double *vb, double *ub) {
  const double ir = 1.0 / u[0];
  double rb = 0;
  ub[D + 1] += (gamma - 1.0) * pb;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double v = u[1 + i] * ir;
    // p = (g-1)(E - 1/2 sum m_i v_i):  dp/dm_i = -(g-1) v_i / 2, dp/dv_i = -(g-1) m_i / 2
    const double vbi = vb[i] - 0.5 * (gamma - 1.0) * u[1 + i] * pb;
    ub[1 + i] += -0.5 * (gamma - 1.0) * v * pb + vbi * ir;
    rb -= vbi * v * ir;
  }
  ub[0] += rb;
}

// f[j][alpha] of the Euler equations
template <int D>
__device__ __forceinline__ void inviscid_flux(const double *u, double gamma, double f[D][D + 2],
                                              double &p, double *v) {
  double rho;
  primitives<D>(u, gamma, rho, v, p);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    f[j][0] = u[1 + j];
#pragma unroll
    for (int i = 0; i < D; ++i) f[j][1 + i] = u[1 + i] * v[j] + (i == j ? p : 0.0);
    f[j][D + 1] = (u[D + 1] + p) * v[j];
  }
}

// ub += (d f / d u)^T fb, with extra cotangents pb_in (of p) and vb_in (of v)
template <int D>
__device__ __forceinline__ void inviscid_flux_vjp(const double *u, double gamma,
                                                  const double fb[D][D + 2], double pb_in,
                                                  const double *vb_in, double *ub) {
  double rho, v[D], p;
  primitives<D>(u, gamma, rho, v, p);
  double pb = pb_in, vb[D];
#pragma unroll
  for (int i = 0; i < D; ++i) vb[i] = vb_in ? vb_in[i] : 0.0;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    ub[1 + j] += fb[j][0];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      ub[1 + i] += fb[j][1 + i] * v[j];
      vb[j] += fb[j][1 + i] * u[1 + i];
    }
    pb += fb[j][1 + j];
    ub[D + 1] += fb[j][D + 1] * v[j];
    pb += fb[j][D + 1] * v[j];
    vb[j] += fb[j][D + 1] * (u[D + 1] + p);
  }
  primitives_vjp<D>(u, gamma, pb, vb, ub);
}

// viscous flux fv[j][alpha] from u and q[j][alpha] = d_j u_alpha
template <int D>
__device__ __forceinline__ void viscous_flux(const double *u, const double q[D][D + 2],
                                             double gamma, double mu, double prandtl,
                                             double fv[D][D + 2]) {
  double rho, v[D], p;
  primitives<D>(u, gamma, rho, v, p);
  const double ir = 1.0 / rho;
  double dv[D][D];  // dv[j][i] = d_j v_i
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int i = 0; i < D; ++i) dv[j][i] = (q[j][1 + i] - v[i] * q[j][0]) * ir;
  double divv = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) divv += dv[k][k];
  double v2 = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) v2 += v[i] * v[i];
  const double kappa = mu * gamma / (prandtl * (gamma - 1.0));
  const double por = p * ir;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    double vdm = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) vdm += v[i] * q[j][1 + i];
    const double dp = (gamma - 1.0) * (q[j][D + 1] - vdm + 0.5 * v2 * q[j][0]);
    const double dT = (dp - por * q[j][0]) * ir;
    double e = kappa * dT;
    fv[j][0] = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double tau = mu * (dv[i][j] + dv[j][i]);
      if (i == j) tau -= 2.0 / 3.0 * mu * divv;
      fv[j][1 + i] = tau;
      e += v[i] * tau;
    }
    fv[j][D + 1] = e;
  }
}

// ub += (d fv / d u)^T fvb, qb += (d fv / d q)^T fvb
template <int D>
__device__ __forceinline__ void viscous_flux_vjp(const double *u, const double q[D][D + 2],
                                                 double gamma, double mu, double prandtl,
                                                 const double fvb[D][D + 2], double *ub,
                                                 double qb[D][D + 2]) {
  double rho, v[D], p;
  primitives<D>(u, gamma, rho, v, p);
  const double ir = 1.0 / rho;
  double dv[D][D];
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int i = 0; i < D; ++i) dv[j][i] = (q[j][1 + i] - v[i] * q[j][0]) * ir;
  double divv = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) divv += dv[k][k];
  double v2 = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) v2 += v[i] * v[i];
  const double kappa = mu * gamma / (prandtl * (gamma - 1.0));
  const double por = p * ir;
  // reverse sweep
  double vb[D], dvb[D][D], divvb = 0, v2b = 0, porb = 0, irb = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    vb[i] = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) dvb[i][j] = 0;
  }
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const double eb = fvb[j][D + 1];
    // e = kappa dT + sum_i v_i tau_ij ; fv[j][1+i] = tau_ij
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double tau = mu * (dv[i][j] + dv[j][i]);
      if (i == j) tau -= 2.0 / 3.0 * mu * divv;
      const double taub = fvb[j][1 + i] + eb * v[i];
      vb[i] += eb * tau;
      dvb[i][j] += mu * taub;
      dvb[j][i] += mu * taub;
      if (i == j) divvb -= 2.0 / 3.0 * mu * taub;
    }
    const double dTb = kappa * eb;
    // dT = (dp - por q0) ir
    double vdm = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) vdm += v[i] * q[j][1 + i];
    const double dp = (gamma - 1.0) * (q[j][D + 1] - vdm + 0.5 * v2 * q[j][0]);
    const double dpb = dTb * ir;
    porb -= dTb * q[j][0] * ir;
    qb[j][0] -= dTb * por * ir;
    irb += dTb * (dp - por * q[j][0]);
    // dp = (g-1)(qE - vdm + v2 q0 / 2)
    qb[j][D + 1] += (gamma - 1.0) * dpb;
    const double vdmb = -(gamma - 1.0) * dpb;
    v2b += 0.5 * (gamma - 1.0) * q[j][0] * dpb;
    qb[j][0] += 0.5 * (gamma - 1.0) * v2 * dpb;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      vb[i] += vdmb * q[j][1 + i];
      qb[j][1 + i] += vdmb * v[i];
    }
  }
  // divv = sum_k dv[k][k]
#pragma unroll
  for (int k = 0; k < D; ++k) dvb[k][k] += divvb;
  // por = p ir
  const double pb = porb * ir;
  irb += porb * p;
  // v2 = sum v_i^2
#pragma unroll
  for (int i = 0; i < D; ++i) vb[i] += 2.0 * v[i] * v2b;
  // dv[j][i] = (q[j][1+i] - v_i q[j][0]) ir
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double b = dvb[j][i];
      qb[j][1 + i] += b * ir;
      vb[i] -= b * q[j][0] * ir;
      qb[j][0] -= b * v[i] * ir;
      irb += b * (q[j][1 + i] - v[i] * q[j][0]);
    }
  // ir = 1 / rho
  ub[0] -= irb * ir * ir;
  primitives_vjp<D>(u, gamma, pb, vb, ub);
}

// Rusanov flux (Appendix B) in direction n of the left side
template <int D>
__device__ __forceinline__ void rusanov(const double *uL, const double *uR, const double *n,
                                        double gamma, double *F) {
  double fL[D][D + 2], fR[D][D + 2], vL[D], vR[D], pL, pR;
  inviscid_flux<D>(uL, gamma, fL, pL, vL);
  inviscid_flux<D>(uR, gamma, fR, pR, vR);
  double vn = 0;
#pragma unroll
  for (int j = 0; j < D; ++j) vn += n[j] * (vL[j] + vR[j]);
  const double s = sqrt(gamma * (pL + pR) / (uL[0] + uR[0])) + 0.5 * fabs(vn);
#pragma unroll
  for (int a = 0; a < D + 2; ++a) {
    double nf = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) nf += n[j] * (fL[j][a] + fR[j][a]);
    F[a] = 0.5 * nf + 0.5 * s * (uL[a] - uR[a]);
  }
}

// uLb += (dF/duL)^T Fb, uRb += (dF/duR)^T Fb (sign(0) taken as 0)
template <int D>
__device__ __forceinline__ void rusanov_vjp(const double *uL, const double *uR, const double *n,
                                            double gamma, const double *Fb, double *uLb,
                                            double *uRb) {
  double rL, vL[D], pL, rR, vR[D], pR;
  primitives<D>(uL, gamma, rL, vL, pL);
  primitives<D>(uR, gamma, rR, vR, pR);
  double vn = 0;
#pragma unroll
  for (int j = 0; j < D; ++j) vn += n[j] * (vL[j] + vR[j]);
  const double P = pL + pR, Rh = rL + rR;
  const double c = sqrt(gamma * P / Rh);
  const double s = c + 0.5 * fabs(vn);
  double sb = 0;
  double fb[D][D + 2];
#pragma unroll
  for (int a = 0; a < D + 2; ++a) {
    sb += 0.5 * Fb[a] * (uL[a] - uR[a]);
    uLb[a] += 0.5 * s * Fb[a];
    uRb[a] -= 0.5 * s * Fb[a];
#pragma unroll
    for (int j = 0; j < D; ++j) fb[j][a] = 0.5 * n[j] * Fb[a];
  }
  const double sgn = vn > 0 ? 1.0 : (vn < 0 ? -1.0 : 0.0);
  const double vnb = 0.5 * sgn * sb;
  const double Pb = sb * gamma / (2.0 * c * Rh);
  const double Rhb = -sb * c / (2.0 * Rh);
  double vbL[D], vbR[D];
#pragma unroll
  for (int j = 0; j < D; ++j) { vbL[j] = n[j] * vnb; vbR[j] = n[j] * vnb; }
  uLb[0] += Rhb;
  uRb[0] += Rhb;
  inviscid_flux_vjp<D>(uL, gamma, fb, Pb, vbL, uLb);
  inviscid_flux_vjp<D>(uR, gamma, fb, Pb, vbR, uRb);
}

// Boundary ghost states (Appendix C).  par: the boundary's parameters
// [type, rho_f, v_f (3), p_f, C_p T_w, v_w (3)]; type 0 supersonic inflow,
// 1 subsonic outflow, 2 no-slip isothermal wall.  ginv is the ghost of the
// inviscid flux, gldg that of the common solution and of the LDG viscous
// terms; the ghost gradient is zero (inflow, outflow) or q_L (wall).
template <int D>
__device__ __forceinline__ void bc_ghosts(const double *u, const double *par, double gamma,
                                          double *ginv, double *gldg, bool &qzero) {
  const int type = (int)par[0];
  const double rho = u[0];
  if (type == 0) {
    double v2 = 0;
    ginv[0] = par[1];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      ginv[1 + d] = par[1] * par[2 + d];
      v2 += par[2 + d] * par[2 + d];
    }
    ginv[D + 1] = par[5] / (gamma - 1) + 0.5 * par[1] * v2;
    qzero = true;
  } else if (type == 1) {
    double v2 = 0;
    ginv[0] = rho;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      ginv[1 + d] = u[1 + d];
      v2 += (u[1 + d] / rho) * (u[1 + d] / rho);
    }
    ginv[D + 1] = par[5] / (gamma - 1) + 0.5 * rho * v2;
    qzero = true;
  } else {
    double w2 = 0, vw2 = 0;
    ginv[0] = rho;
    gldg[0] = rho;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double w = 2 * par[7 + d] - u[1 + d] / rho;
      ginv[1 + d] = rho * w;
      gldg[1 + d] = rho * par[7 + d];
      w2 += w * w;
      vw2 += par[7 + d] * par[7 + d];
    }
    ginv[D + 1] = rho * (par[6] / gamma + 0.5 * w2);
    gldg[D + 1] = rho * (par[6] / gamma + 0.5 * vw2);
    qzero = false;
    return;
  }
#pragma unroll
  for (int a = 0; a < D + 2; ++a) gldg[a] = ginv[a];
}

}  // namespace fr
