// Host-side set-up: points, orthonormal bases, Appendix A operators,
// metric terms and flux-point pairing.
//
// Route (paper section 2): the nodal basis is l = V^-1 psi with the
// generalised Vandermonde V of an orthonormal modal basis psi (Legendre
// products on quads/hexes, Dubiner polynomials on triangles).  Because psi is
// orthonormal, the DG correction field of flux point sigma -- the solution-
// space polynomial whose moments against every psi equal the face moment of
// a unit jump at sigma -- has modal coefficients omega_sigma psi_k(x_sigma),
// so (div g_sigma)(x_rho) = sum_k psi_k(x_rho) psi_k(x_sigma) omega_sigma with
// no mass matrix.  The operators of Appendix A then follow:
//   M0 = l(x^f), M4 = grad l(x^u), M3 = div g(x^u), M6 = n~ M3,
//   M1 = grad l^T, M2 = n~ M0, and the pre-multiplied M4 - M6 M0, M1 - M3 M2.
#include "setup.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace fr {

typedef long double ld_t;

// ---------------------------------------------------------------------------
// 1-D rules
// ---------------------------------------------------------------------------
static void legendre_pd(int n, ld_t x, ld_t &p, ld_t &dp) {
  ld_t p0 = 1, p1 = x;
  if (n == 0) { p = 1; dp = 0; return; }
  for (int k = 1; k < n; ++k) {
    ld_t p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    p0 = p1; p1 = p2;
  }
  p = p1;
  dp = n * (x * p1 - p0) / (x * x - 1);
}

static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  std::vector<ld_t> xs(n), ws(n);
  const ld_t pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    ld_t z = std::cos(pi * (n - i - 0.25L) / (n + 0.5L));  // ascending guesses
    for (int it = 0; it < 100; ++it) {
      ld_t p, dp;
      legendre_pd(n, z, p, dp);
      ld_t dz = p / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-30L) break;
    }
    ld_t p, dp;
    legendre_pd(n, z, p, dp);
    xs[i] = z;
    ws[i] = 2 / ((1 - z * z) * dp * dp);
  }
  x.assign(xs.begin(), xs.end());
  w.assign(ws.begin(), ws.end());
}

// Gauss-Lobatto-Legendre nodes: +-1 and the roots of P_n'.
static std::vector<double> gauss_lobatto(int n) {
  std::vector<double> out(n + 1);
  out[0] = -1; out[n] = 1;
  const ld_t pi = 3.141592653589793238462643383279502884L;
  for (int i = 1; i < n; ++i) {
    ld_t z = -std::cos(pi * i / n);
    for (int it = 0; it < 100; ++it) {
      ld_t p, dp;
      legendre_pd(n, z, p, dp);
      ld_t d2p = (2 * z * dp - n * (n + 1) * p) / (1 - z * z);
      ld_t dz = dp / d2p;
      z -= dz;
      if (std::fabs(dz) < 1e-30L) break;
    }
    out[i] = (double)z;
  }
  return out;
}

// Normalised Jacobi polynomial P_n^(a,b)(x), orthonormal on [-1,1] with
// weight (1-x)^a (1+x)^b, by its three-term recurrence (the normalised
// recurrence as Hesthaven & Warburton, "Nodal Discontinuous Galerkin
// Methods", 2008, give it in their JacobiP routine).
static ld_t jacobi(int n, int a, int b, ld_t x) {
  ld_t g0 = std::pow(2.0L, a + b + 1) / (a + b + 1) * std::tgamma((ld_t)a + 1) *
            std::tgamma((ld_t)b + 1) / std::tgamma((ld_t)a + b + 1);
  ld_t pm = 1 / std::sqrt(g0);
  if (n == 0) return pm;
  ld_t g1 = (ld_t)(a + 1) * (b + 1) / (a + b + 3) * g0;
  ld_t pc = ((a + b + 2) * x / 2 + (ld_t)(a - b) / 2) / std::sqrt(g1);
  if (n == 1) return pc;
  ld_t aold = 2.0L / (2 + a + b) * std::sqrt((ld_t)(a + 1) * (b + 1) / (a + b + 3));
  for (int i = 1; i < n; ++i) {
    ld_t h1 = 2 * i + a + b;
    ld_t anew = 2 / (h1 + 2) *
                std::sqrt((ld_t)(i + 1) * (i + 1 + a + b) * (i + 1 + a) * (i + 1 + b) /
                          (h1 + 1) / (h1 + 3));
    ld_t bnew = -(ld_t)(a * a - b * b) / h1 / (h1 + 2);
    ld_t pn = (-aold * pm + (x - bnew) * pc) / anew;
    pm = pc; pc = pn; aold = anew;
  }
  return pc;
}

static ld_t djacobi(int n, int a, int b, ld_t x) {
  if (n == 0) return 0;
  return std::sqrt((ld_t)n * (n + a + b + 1)) * jacobi(n - 1, a + 1, b + 1, x);
}

// ---------------------------------------------------------------------------
// Orthonormal modal bases (value and reference gradient)
// ---------------------------------------------------------------------------
struct Modal {
  int etype, p, ndims, n;
  Modal(int et, int pp) : etype(et), p(pp) {
    ndims = et == ET_HEX ? 3 : 2;
    n = et == ET_TRI ? (p + 1) * (p + 2) / 2 : (et == ET_HEX ? (p + 1) * (p + 1) * (p + 1)
                                                            : (p + 1) * (p + 1));
  }
  // psi[k], dpsi[k*ndims + i] at point x
  void eval(const double *x, ld_t *psi, ld_t *dpsi) const {
    if (etype == ET_TRI) {
      ld_t r = x[0], s = x[1];
      ld_t a = (std::fabs(1 - s) > 1e-14L) ? 2 * (1 + r) / (1 - s) - 1 : -1;
      ld_t b = s;
      int k = 0;
      for (int i = 0; i <= p; ++i)
        for (int j = 0; j <= p - i; ++j, ++k) {
          ld_t fa = jacobi(i, 0, 0, a), dfa = djacobi(i, 0, 0, a);
          ld_t gb = jacobi(j, 2 * i + 1, 0, b), dgb = djacobi(j, 2 * i + 1, 0, b);
          ld_t hb = std::pow(0.5L * (1 - b), i);
          psi[k] = std::sqrt(2.0L) * fa * gb * std::pow(1 - b, i);
          ld_t hbm = i > 0 ? std::pow(0.5L * (1 - b), i - 1) : 1;
          ld_t dr = dfa * gb * hbm;
          ld_t ds = dfa * gb * 0.5L * (1 + a) * hbm;
          ld_t t = dgb * hb;
          if (i > 0) t -= 0.5L * i * gb * hbm;
          ds += fa * t;
          ld_t sc = std::pow(2.0L, i + 0.5L);
          dpsi[k * 2 + 0] = sc * dr;
          dpsi[k * 2 + 1] = sc * ds;
        }
      return;
    }
    // tensor: psi_(a,b,c) = prod_d sqrt((2 m+1)/2) P_m(x_d), first index fastest
    int n1 = p + 1;
    ld_t v[3][16], d[3][16];
    for (int dd = 0; dd < ndims; ++dd)
      for (int m = 0; m < n1; ++m) {
        ld_t pv, dv;
        legendre_pd(m, x[dd], pv, dv);
        if (m == 0) dv = 0;
        if (std::fabs(std::fabs((ld_t)x[dd]) - 1) < 1e-15L) {  // P_m'(+-1) closed form
          dv = (m * (m + 1) / 2.0L) * (x[dd] > 0 ? 1 : ((m + 1) % 2 ? 1 : -1));
        }
        ld_t sc = std::sqrt((2 * m + 1) / 2.0L);
        v[dd][m] = sc * pv;
        d[dd][m] = sc * dv;
      }
    int k = 0;
    int nc = ndims == 3 ? n1 : 1;
    for (int c = 0; c < nc; ++c)
      for (int b = 0; b < n1; ++b)
        for (int a = 0; a < n1; ++a, ++k) {
          int idx[3] = {a, b, c};
          ld_t val = 1;
          for (int dd = 0; dd < ndims; ++dd) val *= v[dd][idx[dd]];
          psi[k] = val;
          for (int i = 0; i < ndims; ++i) {
            ld_t g = 1;
            for (int dd = 0; dd < ndims; ++dd) g *= (dd == i ? d[dd][idx[dd]] : v[dd][idx[dd]]);
            dpsi[k * ndims + i] = g;
          }
        }
  }
};

// Inverse by Gauss-Jordan elimination with partial pivoting (long double).
static std::vector<ld_t> invert(std::vector<ld_t> A, int n) {
  std::vector<ld_t> I(n * n, 0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (std::fabs(A[piv * n + c]) < 1e-300L) throw SetupError(3, "singular Vandermonde matrix");
    if (piv != c)
      for (int k = 0; k < n; ++k) { std::swap(A[c * n + k], A[piv * n + k]); std::swap(I[c * n + k], I[piv * n + k]); }
    ld_t inv = 1 / A[c * n + c];
    for (int k = 0; k < n; ++k) { A[c * n + k] *= inv; I[c * n + k] *= inv; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      ld_t f = A[r * n + c];
      if (f == 0) continue;
      for (int k = 0; k < n; ++k) { A[r * n + k] -= f * A[c * n + k]; I[r * n + k] -= f * I[c * n + k]; }
    }
  }
  return I;
}

// ---------------------------------------------------------------------------
// Triangle solution points: Warburton's warp-and-blend construction with
// blend exponent 0 (equispaced lattice warped so its edges carry
// Gauss-Lobatto points): Warburton, J. Eng. Math. 56 (2006), and the
// Warpfactor / Nodes2D routines of Hesthaven & Warburton (2008), whose steps
// this follows.
// ---------------------------------------------------------------------------
static double warp_factor(int n, double r, const std::vector<double> &gll) {
  // interpolant through equispaced nodes of (gll - equispaced), at r
  double warp = 0;
  for (int i = 0; i <= n; ++i) {
    double ri = -1 + 2.0 * i / n;
    double li = 1;
    for (int j = 0; j <= n; ++j)
      if (j != i) li *= (r - (-1 + 2.0 * j / n)) / (ri - (-1 + 2.0 * j / n));
    warp += li * (gll[i] - ri);
  }
  bool inside = std::fabs(r) < 1 - 1e-10;
  if (inside) warp /= (1 - r * r);
  return warp;
}

static std::vector<double> triangle_points(int n) {
  std::vector<double> out;
  if (n == 0) { out = {-1.0 / 3, -1.0 / 3}; return out; }
  std::vector<double> gll = gauss_lobatto(n);
  const double s3 = std::sqrt(3.0), pi = 3.14159265358979323846;
  for (int a = 0; a <= n; ++a)
    for (int b = 0; b <= n - a; ++b) {
      double L1 = (double)a / n, L3 = (double)b / n, L2 = 1 - L1 - L3;
      double x = -L2 + L3, y = (-L2 - L3 + 2 * L1) / s3;
      double w1 = 4 * L2 * L3 * warp_factor(n, L3 - L2, gll);
      double w2 = 4 * L1 * L3 * warp_factor(n, L1 - L3, gll);
      double w3 = 4 * L1 * L2 * warp_factor(n, L2 - L1, gll);
      x += w1 + std::cos(2 * pi / 3) * w2 + std::cos(4 * pi / 3) * w3;
      y += std::sin(2 * pi / 3) * w2 + std::sin(4 * pi / 3) * w3;
      double l1 = (s3 * y + 1) / 3, l2 = (-3 * x - s3 * y + 2) / 6, l3 = (3 * x - s3 * y + 2) / 6;
      out.push_back(-l2 + l3 - l1);
      out.push_back(-l2 - l3 + l1);
    }
  return out;
}

// ---------------------------------------------------------------------------
// Faces of the reference elements: point on face f at parameters t, unit
// outward normal, and the arc/area scale ds/dt.
// ---------------------------------------------------------------------------
static void face_point(int etype, int f, const double *t, double *x, double *nrm, double &scale) {
  scale = 1;
  if (etype == ET_QUAD) {
    static const double N[4][2] = {{0, -1}, {1, 0}, {0, 1}, {-1, 0}};
    double tt = t[0];
    double P[4][2] = {{tt, -1}, {1, tt}, {-tt, 1}, {-1, -tt}};
    x[0] = P[f][0]; x[1] = P[f][1];
    nrm[0] = N[f][0]; nrm[1] = N[f][1];
  } else if (etype == ET_TRI) {
    double tt = t[0], r2 = std::sqrt(0.5);
    double P[3][2] = {{tt, -1}, {-tt, tt}, {-1, -tt}};
    double N[3][2] = {{0, -1}, {r2, r2}, {-1, 0}};
    x[0] = P[f][0]; x[1] = P[f][1];
    nrm[0] = N[f][0]; nrm[1] = N[f][1];
    if (f == 1) scale = std::sqrt(2.0);
  } else {
    double a = t[0], b = t[1];
    double P[6][3] = {{a, b, -1}, {a, -1, b}, {1, a, b}, {a, 1, b}, {-1, a, b}, {a, b, 1}};
    static const double N[6][3] = {{0, 0, -1}, {0, -1, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, 0, 1}};
    for (int d = 0; d < 3; ++d) { x[d] = P[f][d]; nrm[d] = N[f][d]; }
  }
}

// ---------------------------------------------------------------------------
// The VCJH family of correction functions (Vincent, Castonguay and Jameson's
// energy-stable FR schemes, which the paper cites for its DG, SD and HU
// runs).  In one dimension the left correction is
//   g_L = (-1)^p / 2 [P_p - (eta P_{p-1} + P_{p+1}) / (1 + eta)],
//   eta = c (2p + 1) (a_p p!)^2 / 2,  a_p p! = (2p)! / (2^p p!) = (2p - 1)!!,
// with g_L(-1) = 1, g_L(1) = 0, and the right one g_R(xi) = g_L(-xi).
// c = 0 is DG (the right Radau polynomial); SD and HU are
//   c_SD = 2p / ((2p + 1)(p + 1)(a_p p!)^2),  c_HU = 2(p + 1) / ((2p + 1) p (a_p p!)^2).
// ---------------------------------------------------------------------------
static ld_t vcjh_eta(int corr, int p) {
  ld_t k = 1;  // (2p - 1)!!
  for (int j = 1; j <= p; ++j) k *= 2 * j - 1;
  const ld_t scale = k * k;
  ld_t c = 0;
  if (corr == CORR_SD) c = (ld_t)(2 * p) / ((2 * p + 1) * (ld_t)(p + 1) * scale);
  if (corr == CORR_HU) c = (ld_t)(2 * (p + 1)) / ((2 * p + 1) * (ld_t)p * scale);
  return c * (2 * p + 1) * scale / 2;
}

// d g_L / d xi at x; P_k' from P_{k+1}' = P_{k-1}' + (2k + 1) P_k.
static ld_t vcjh_left_deriv(int p, ld_t eta, ld_t x) {
  std::vector<ld_t> P(p + 2), dP(p + 2);
  P[0] = 1; dP[0] = 0;
  P[1] = x; dP[1] = 1;
  for (int k = 1; k <= p; ++k) {
    P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
    dP[k + 1] = dP[k - 1] + (2 * k + 1) * P[k];
  }
  const ld_t sg = (p % 2) ? -0.5L : 0.5L;
  return sg * (dP[p] - (eta * dP[p - 1] + dP[p + 1]) / (1 + eta));
}

RefOps build_ref(int etype, int p, int corr) {
  if (etype < 0 || etype > 2) throw SetupError(1, "bad element type");
  int pmax = etype == ET_HEX ? 4 : 6;
  if (p < 1 || p > pmax) throw SetupError(3, "unsupported order " + std::to_string(p));
  if (corr < CORR_DG || corr > CORR_HU) throw SetupError(1, "bad correction scheme");
  if (corr != CORR_DG && etype == ET_TRI)
    throw SetupError(3, "SD and HU correction functions are built for quads and hexes only");
  RefOps R;
  R.etype = etype; R.p = p; R.corr = corr;
  const int D = R.ndims = etype == ET_HEX ? 3 : 2;
  const int n1 = p + 1;
  std::vector<double> xg, wg;
  gauss_legendre(n1, xg, wg);
  Modal modal(etype, p);
  const int Nu = R.nupts = modal.n;
  // solution points
  if (etype == ET_TRI) {
    R.upts = triangle_points(p);
  } else {
    int nc = D == 3 ? n1 : 1;
    for (int c = 0; c < nc; ++c)
      for (int b = 0; b < n1; ++b)
        for (int a = 0; a < n1; ++a) {
          R.upts.push_back(xg[a]);
          R.upts.push_back(xg[b]);
          if (D == 3) R.upts.push_back(xg[c]);
        }
  }
  // flux points: Gauss-Legendre on each face
  R.nfaces = etype == ET_QUAD ? 4 : (etype == ET_TRI ? 3 : 6);
  R.nfp_face = D == 2 ? n1 : n1 * n1;
  for (int f = 0; f < R.nfaces; ++f)
    for (int k = 0; k < R.nfp_face; ++k) {
      double t[2] = {xg[k % n1], D == 3 ? xg[k / n1] : 0.0};
      double w = D == 3 ? wg[k % n1] * wg[k / n1] : wg[k];
      double x[3], nr[3], sc;
      face_point(etype, f, t, x, nr, sc);
      for (int d = 0; d < D; ++d) { R.fpts.push_back(x[d]); R.fnorm.push_back(nr[d]); }
      R.fface.push_back(f);
      R.fweight.push_back(w * sc);
    }
  const int Nf = R.nfpts = (int)R.fface.size();
  // modal values at solution and flux points
  std::vector<ld_t> psu(Nu * Nu), dpsu(Nu * Nu * D), psf(Nf * Nu), dtmp(Nu * D);
  for (int r = 0; r < Nu; ++r) modal.eval(&R.upts[r * D], &psu[r * Nu], &dpsu[r * Nu * D]);
  for (int s = 0; s < Nf; ++s) modal.eval(&R.fpts[s * D], &psf[s * Nu], dtmp.data());
  // Vandermonde A[sigma][k] = psi_k(x_sigma); nodal l(x) = psi(x) A^-1
  std::vector<ld_t> Ainv = invert(psu, Nu);
  auto nodal = [&](const ld_t *psi, int r) {  // l_r at a point with modal values psi
    ld_t s = 0;
    for (int k = 0; k < Nu; ++k) s += psi[k] * Ainv[k * Nu + r];
    return s;
  };
  R.M0.assign((size_t)Nf * Nu, 0);
  for (int s = 0; s < Nf; ++s)
    for (int r = 0; r < Nu; ++r) R.M0[s * Nu + r] = (double)nodal(&psf[s * Nu], r);
  // M4[i Nu + sigma][rho] = d_i l_rho(x^u_sigma); M1 = its block transpose
  R.M4.assign((size_t)D * Nu * Nu, 0);
  R.M1.assign((size_t)Nu * D * Nu, 0);
  std::vector<ld_t> dcol(Nu);
  for (int s = 0; s < Nu; ++s)
    for (int i = 0; i < D; ++i) {
      for (int k = 0; k < Nu; ++k) dcol[k] = dpsu[s * Nu * D + k * D + i];
      for (int r = 0; r < Nu; ++r) {
        double v = (double)nodal(dcol.data(), r);
        R.M4[(size_t)(i * Nu + s) * Nu + r] = v;
        R.M1[(size_t)s * D * Nu + i * Nu + r] = v;
      }
    }
  // M3[rho][sigma] = sum_k psi_k(x_rho) psi_k(x_sigma) omega_sigma (DG lifting)
  R.M3.assign((size_t)Nu * Nf, 0);
  for (int r = 0; r < Nu; ++r)
    for (int s = 0; s < Nf; ++s) {
      ld_t acc = 0;
      for (int k = 0; k < Nu; ++k) acc += psu[r * Nu + k] * psf[s * Nu + k];
      R.M3[(size_t)r * Nf + s] = (double)(acc * R.fweight[s]);
    }
  // SD / HU on tensor elements: g_sigma = n~_sigma h(xi_i) ell_sigma(xi_tangent)
  // with the face normal n~_sigma = s e_i, h = g_L (s = -1) or g_R (s = +1)
  // and ell_sigma the face Lagrange polynomial that is one at sigma.  At the
  // GL solution points ell_sigma is one on sigma's face-normal line and zero
  // elsewhere, so div g_sigma(x_rho) = -g_L'(-s xi_i(rho)) on that line.
  if (corr != CORR_DG) {
    const ld_t eta = vcjh_eta(corr, p);
    for (int s = 0; s < Nf; ++s) {
      int i = 0;
      for (int d = 1; d < D; ++d)
        if (std::fabs(R.fnorm[s * D + d]) > std::fabs(R.fnorm[s * D + i])) i = d;
      const double sg = R.fnorm[s * D + i];
      for (int r = 0; r < Nu; ++r) {
        bool on = true;
        for (int d = 0; d < D; ++d)
          if (d != i && std::fabs(R.upts[r * D + d] - R.fpts[s * D + d]) > 1e-9) on = false;
        R.M3[(size_t)r * Nf + s] =
            on ? (double)-vcjh_left_deriv(p, eta, -(ld_t)sg * R.upts[r * D + i]) : 0.0;
      }
    }
  }
  // M6[i Nu + rho][sigma] = n~_sigma,i M3[rho][sigma];  M2[sigma][i Nu + rho] = n~_sigma,i M0
  R.M6.assign((size_t)D * Nu * Nf, 0);
  R.M2.assign((size_t)Nf * D * Nu, 0);
  for (int i = 0; i < D; ++i)
    for (int r = 0; r < Nu; ++r)
      for (int s = 0; s < Nf; ++s) {
        R.M6[(size_t)(i * Nu + r) * Nf + s] = R.fnorm[s * D + i] * R.M3[(size_t)r * Nf + s];
        R.M2[(size_t)s * D * Nu + i * Nu + r] = R.fnorm[s * D + i] * R.M0[(size_t)s * Nu + r];
      }
  // pre-multiplied operators (long double accumulation)
  R.M4p.assign((size_t)D * Nu * Nu, 0);
  for (int row = 0; row < D * Nu; ++row)
    for (int c = 0; c < Nu; ++c) {
      ld_t acc = R.M4[(size_t)row * Nu + c];
      for (int s = 0; s < Nf; ++s) acc -= (ld_t)R.M6[(size_t)row * Nf + s] * R.M0[(size_t)s * Nu + c];
      R.M4p[(size_t)row * Nu + c] = (double)acc;
    }
  R.M1p.assign((size_t)Nu * D * Nu, 0);
  for (int r = 0; r < Nu; ++r)
    for (int c = 0; c < D * Nu; ++c) {
      ld_t acc = R.M1[(size_t)r * D * Nu + c];
      for (int s = 0; s < Nf; ++s) acc -= (ld_t)R.M3[(size_t)r * Nf + s] * R.M2[(size_t)s * D * Nu + c];
      R.M1p[(size_t)r * D * Nu + c] = (double)acc;
    }
  // W_rho = int l_rho = A^-1[0][rho] / psi_0 (psi_0 is the constant mode)
  R.W.resize(Nu);
  for (int r = 0; r < Nu; ++r) R.W[r] = (double)(Ainv[0 * Nu + r] / psu[0]);
  return R;
}

// ---------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------
int nnodes_of(int etype, int g) {
  if (etype == ET_QUAD) return (g + 1) * (g + 1);
  if (etype == ET_HEX) return (g + 1) * (g + 1) * (g + 1);
  return (g + 1) * (g + 2) / 2;
}

// shape function values N[k] and gradients dN[k*D + j] at reference point xi
static void shape(int etype, int g, const double *xi, double *N, double *dN) {
  if (etype == ET_TRI) {
    double l[3] = {-(xi[0] + xi[1]) / 2, (1 + xi[0]) / 2, (1 + xi[1]) / 2};
    const double dl[3][2] = {{-0.5, -0.5}, {0.5, 0}, {0, 0.5}};
    if (g == 1) {
      for (int k = 0; k < 3; ++k) { N[k] = l[k]; dN[2 * k] = dl[k][0]; dN[2 * k + 1] = dl[k][1]; }
      return;
    }
    for (int k = 0; k < 3; ++k) {
      N[k] = l[k] * (2 * l[k] - 1);
      for (int j = 0; j < 2; ++j) dN[2 * k + j] = (4 * l[k] - 1) * dl[k][j];
    }
    const int e[3][2] = {{0, 1}, {1, 2}, {2, 0}};
    for (int m = 0; m < 3; ++m) {
      int a = e[m][0], b = e[m][1];
      N[3 + m] = 4 * l[a] * l[b];
      for (int j = 0; j < 2; ++j) dN[2 * (3 + m) + j] = 4 * (l[b] * dl[a][j] + l[a] * dl[b][j]);
    }
    return;
  }
  const int D = etype == ET_HEX ? 3 : 2, n1 = g + 1;
  double v[3][3], d[3][3];
  for (int dd = 0; dd < D; ++dd)
    for (int a = 0; a < n1; ++a) {
      double xa = -1 + 2.0 * a / g, val = 1, der = 0;
      for (int b = 0; b < n1; ++b) {
        if (b == a) continue;
        double xb = -1 + 2.0 * b / g;
        double term = 1 / (xa - xb);
        for (int c = 0; c < n1; ++c)
          if (c != a && c != b) term *= (xi[dd] - (-1 + 2.0 * c / g)) / (xa - (-1 + 2.0 * c / g));
        der += term;
        val *= (xi[dd] - xb) / (xa - xb);
      }
      v[dd][a] = val; d[dd][a] = der;
    }
  int k = 0, nc = D == 3 ? n1 : 1;
  for (int c = 0; c < nc; ++c)
    for (int b = 0; b < n1; ++b)
      for (int a = 0; a < n1; ++a, ++k) {
        int idx[3] = {a, b, c};
        double val = 1;
        for (int dd = 0; dd < D; ++dd) val *= v[dd][idx[dd]];
        N[k] = val;
        for (int j = 0; j < D; ++j) {
          double gg = 1;
          for (int dd = 0; dd < D; ++dd) gg *= (dd == j ? d[dd][idx[dd]] : v[dd][idx[dd]]);
          dN[k * D + j] = gg;
        }
      }
}

// x and J at xi for one element; S = adj J, returns det J
static double map_point(int etype, int g, int D, const double *X, int nn, const double *xi,
                        double *x, double *S, std::vector<double> &N, std::vector<double> &dN) {
  shape(etype, g, xi, N.data(), dN.data());
  // Node coordinates are taken relative to node 0 (the shape functions sum
  // to one and their gradients to zero): the Jacobian of a small element far
  // from the origin then keeps full relative precision instead of losing
  // |x| / h of it to cancellation.
  double J[3][3] = {{0}};
  for (int d = 0; d < D; ++d) x[d] = 0;
  for (int k = 1; k < nn; ++k)
    for (int d = 0; d < D; ++d) {
      const double rel = X[k * D + d] - X[d];
      x[d] += N[k] * rel;
      for (int j = 0; j < D; ++j) J[d][j] += rel * dN[k * D + j];
    }
  for (int d = 0; d < D; ++d) x[d] += X[d];
  if (D == 2) {
    S[0] = J[1][1]; S[1] = -J[0][1]; S[2] = -J[1][0]; S[3] = J[0][0];
    return J[0][0] * J[1][1] - J[0][1] * J[1][0];
  }
  // adjugate: S[i][j] = cofactor C[j][i]
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
      S[i * 3 + j] = J[r0][c0] * J[r1][c1] - J[r0][c1] * J[r1][c0];
    }
  return J[0][0] * S[0] + J[0][1] * S[3] + J[0][2] * S[6];
}

BlockGeom build_geom(const RefOps &ref, int g, int64_t nelem, const double *nodes, int64_t ld) {
  if (g < 1 || g > 2) throw SetupError(3, "geometry order must be 1 or 2");
  BlockGeom G;
  const int D = ref.ndims, Nu = ref.nupts, Nf = ref.nfpts, nn = nnodes_of(ref.etype, g);
  G.nelem = nelem; G.ld = ld;
  G.smat.assign((size_t)D * D * Nu * ld, 0.0);
  G.rcpdjac.assign((size_t)Nu * ld, 0.0);
  G.wdjac.assign((size_t)Nu * ld, 0.0);
  G.xu.resize((size_t)nelem * Nu * D);
  G.xf.resize((size_t)nelem * Nf * D);
  G.fnhat.resize((size_t)nelem * Nf * D);
  G.fmag.resize((size_t)nelem * Nf);
  double hmin = 1e300;
  bool bad = false;
#pragma omp parallel for reduction(min : hmin) reduction(|| : bad)
  for (int64_t e = 0; e < nelem; ++e) {
    std::vector<double> N(nn), dN(nn * D);
    const double *X = nodes + (size_t)e * nn * D;
    double S[9], x[3];
    for (int r = 0; r < Nu; ++r) {
      double dj = map_point(ref.etype, g, D, X, nn, &ref.upts[r * D], x, S, N, dN);
      if (!(dj > 0)) bad = true;
      for (int d = 0; d < D; ++d) G.xu[((size_t)e * Nu + r) * D + d] = x[d];
      for (int i = 0; i < D * D; ++i) G.smat[((size_t)i * Nu + r) * ld + e] = S[i];
      G.rcpdjac[(size_t)r * ld + e] = 1.0 / dj;
      G.wdjac[(size_t)r * ld + e] = ref.W[r] * dj;
    }
    for (int s = 0; s < Nf; ++s) {
      double dj = map_point(ref.etype, g, D, X, nn, &ref.fpts[s * D], x, S, N, dN);
      if (!(dj > 0)) bad = true;
      double nu[3] = {0, 0, 0}, m = 0;
      for (int j = 0; j < D; ++j) {
        for (int i = 0; i < D; ++i) nu[j] += S[i * D + j] * ref.fnorm[s * D + i];
        m += nu[j] * nu[j];
      }
      m = std::sqrt(m);
      G.fmag[(size_t)e * Nf + s] = m;
      for (int d = 0; d < D; ++d) {
        G.xf[((size_t)e * Nf + s) * D + d] = x[d];
        G.fnhat[((size_t)e * Nf + s) * D + d] = nu[d] / m;
      }
    }
    // element extent from its nodes
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int k = 0; k < nn; ++k)
      for (int d = 0; d < D; ++d) {
        lo[d] = std::min(lo[d], X[k * D + d]);
        hi[d] = std::max(hi[d], X[k * D + d]);
      }
    double ext = 1e300;
    for (int d = 0; d < D; ++d) ext = std::min(ext, hi[d] - lo[d]);
    hmin = std::min(hmin, ext);
  }
  if (bad) throw SetupError(2, "non-positive Jacobian determinant");
  G.hmin = hmin;
  return G;
}

// ---------------------------------------------------------------------------
// Pairing of flux points by physical coordinate (paper section 2: the two
// flux points of a pair coincide in physical space)
// ---------------------------------------------------------------------------
PairTable build_pairs(const std::vector<RefOps> &refs, const std::vector<BlockGeom> &geoms,
                      const std::vector<int> &block_ref, int D, int nvars,
                      const FacePairIn *pairs, int64_t npairs, const BcFaceIn *bcfaces,
                      int64_t nbcfaces, int nbcs, BcTable *bct) {
  const int nb = (int)geoms.size();
  double hmin = 1e300;
  for (auto &g : geoms) hmin = std::min(hmin, g.hmin);
  const double tol = 1e-8 * hmin;
  std::vector<std::vector<uint8_t>> used(nb);
  for (int b = 0; b < nb; ++b) used[b].assign((size_t)geoms[b].nelem * refs[block_ref[b]].nfpts, 0);
  struct Rec { int lb, rb; int64_t li, ri; double n[3]; double mL, mR; };
  std::vector<Rec> recs;
  for (int64_t k = 0; k < npairs; ++k) {
    const FacePairIn &P = pairs[k];
    if (P.lblock < 0 || P.lblock >= nb || P.rblock < 0 || P.rblock >= nb)
      throw SetupError(1, "face pair block out of range");
    const RefOps &RL = refs[block_ref[P.lblock]], &RR = refs[block_ref[P.rblock]];
    const BlockGeom &GL = geoms[P.lblock], &GR = geoms[P.rblock];
    if (P.lelem < 0 || P.lelem >= GL.nelem || P.relem < 0 || P.relem >= GR.nelem ||
        P.lface < 0 || P.lface >= RL.nfaces || P.rface < 0 || P.rface >= RR.nfaces)
      throw SetupError(1, "face pair element or face out of range");
    if (RL.nfp_face != RR.nfp_face) throw SetupError(2, "face pair with different flux point counts");
    const int m = RL.nfp_face;
    for (int a = 0; a < m; ++a) {
      int sL = P.lface * m + a;
      const double *xL = &GL.xf[((size_t)P.lelem * RL.nfpts + sL) * D];
      int best = -1;
      double bd = 1e300;
      for (int b = 0; b < m; ++b) {
        int sR = P.rface * m + b;
        const double *xR = &GR.xf[((size_t)P.relem * RR.nfpts + sR) * D];
        double d2 = 0;
        for (int d = 0; d < D; ++d) { double t = xR[d] + P.shift[d] - xL[d]; d2 += t * t; }
        if (d2 < bd) { bd = d2; best = sR; }
      }
      if (std::sqrt(bd) > tol) throw SetupError(2, "flux points of a face pair do not coincide");
      uint8_t &uL = used[P.lblock][(size_t)P.lelem * RL.nfpts + sL];
      uint8_t &uR = used[P.rblock][(size_t)P.relem * RR.nfpts + best];
      if (uL || uR) throw SetupError(2, "flux point paired more than once");
      uL = uR = 1;
      Rec r;
      r.lb = P.lblock; r.rb = P.rblock;
      r.li = (int64_t)sL * nvars * GL.ld + P.lelem;
      r.ri = (int64_t)best * nvars * GR.ld + P.relem;
      for (int d = 0; d < 3; ++d) r.n[d] = d < D ? GL.fnhat[((size_t)P.lelem * RL.nfpts + sL) * D + d] : 0;
      r.mL = GL.fmag[(size_t)P.lelem * RL.nfpts + sL];
      r.mR = GR.fmag[(size_t)P.relem * RR.nfpts + best];
      recs.push_back(r);
    }
  }
  // boundary faces: each of their flux points is its own interface
  struct BRec { int b, bc; int64_t i; double n[3]; double m; };
  std::vector<BRec> brecs;
  for (int64_t k = 0; k < nbcfaces; ++k) {
    const BcFaceIn &F = bcfaces[k];
    if (F.block < 0 || F.block >= nb) throw SetupError(1, "boundary face block out of range");
    const RefOps &R = refs[block_ref[F.block]];
    const BlockGeom &G = geoms[F.block];
    if (F.elem < 0 || F.elem >= G.nelem || F.face < 0 || F.face >= R.nfaces)
      throw SetupError(1, "boundary face element or face out of range");
    if (F.bc < 0 || F.bc >= nbcs) throw SetupError(1, "boundary condition index out of range");
    const int m = R.nfp_face;
    for (int a = 0; a < m; ++a) {
      const int s = F.face * m + a;
      uint8_t &u = used[F.block][(size_t)F.elem * R.nfpts + s];
      if (u) throw SetupError(2, "boundary flux point also paired or listed twice");
      u = 1;
      BRec r;
      r.b = F.block; r.bc = F.bc;
      r.i = (int64_t)s * nvars * G.ld + F.elem;
      for (int d = 0; d < 3; ++d) r.n[d] = d < D ? G.fnhat[((size_t)F.elem * R.nfpts + s) * D + d] : 0;
      r.m = G.fmag[(size_t)F.elem * R.nfpts + s];
      brecs.push_back(r);
    }
  }
  for (int b = 0; b < nb; ++b)
    for (uint8_t u : used[b])
      if (!u) throw SetupError(2, "flux point neither paired nor on a boundary face");
  std::sort(brecs.begin(), brecs.end(), [](const BRec &a, const BRec &b) {
    return a.b != b.b ? a.b < b.b : a.i < b.i;
  });
  if (bct) {
    bct->n = (int64_t)brecs.size();
    bct->blk.resize(bct->n); bct->bc.resize(bct->n); bct->idx.resize(bct->n);
    bct->nrm.resize((size_t)D * bct->n); bct->mag.resize(bct->n);
    for (int64_t i = 0; i < bct->n; ++i) {
      const BRec &r = brecs[i];
      bct->blk[i] = r.b; bct->bc[i] = r.bc; bct->idx[i] = r.i; bct->mag[i] = r.m;
      for (int d = 0; d < D; ++d) bct->nrm[(size_t)d * bct->n + i] = r.n[d];
    }
  }
  // order pairs by (L block, L flux point, L element): consecutive pairs then
  // read consecutive elements of one U^f row, which coalesces the L side
  std::sort(recs.begin(), recs.end(), [](const Rec &a, const Rec &b) {
    return a.lb != b.lb ? a.lb < b.lb : a.li < b.li;
  });
  PairTable T;
  T.n = (int64_t)recs.size();
  T.lblk.resize(T.n); T.rblk.resize(T.n); T.lidx.resize(T.n); T.ridx.resize(T.n);
  T.nrm.resize((size_t)D * T.n); T.magL.resize(T.n); T.magR.resize(T.n);
  for (int64_t i = 0; i < T.n; ++i) {
    const Rec &r = recs[i];
    T.lblk[i] = r.lb; T.rblk[i] = r.rb; T.lidx[i] = r.li; T.ridx[i] = r.ri;
    for (int d = 0; d < D; ++d) T.nrm[(size_t)d * T.n + i] = r.n[d];
    T.magL[i] = r.mL; T.magR[i] = r.mR;
  }
  return T;
}

}  // namespace fr
