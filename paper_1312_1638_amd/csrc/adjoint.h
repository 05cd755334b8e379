// Launchers of the adjoint (vector-Jacobian product) kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fr {

struct AdjPointArgs {
  int ndims, nvars, nupts;
  int64_t ld, nelem;
  const double *smat, *rcpdjac;
  const double *u;        // primal state (block)
  const double *q;        // primal gradients Q [D][Nu][NV][ld] (NS)
  double *fb;             // in: F~ cotangent; out: Q cotangent (NS), in place
  double *ulam;           // out: state cotangent of the point-wise flux
  double gamma, mu, prandtl;
};

struct AdjPairArgs {
  int ndims, nvars;
  int64_t npairs;
  const int32_t *lidx, *ridx, *lblk, *rblk;
  const double *nrm, *magL, *magR;
  const double *uf;       // primal U^f
  const double *qf;       // primal Q^f
  double *ufb;            // in: D~ cotangent; out: U^f cotangent (in place)
  double *qfb;            // out: Q^f cotangent; in (con_u_vjp): C^f cotangent
  const int64_t *blk_ufbase, *blk_qfbase, *blk_ld, *blk_qstride;
  int64_t ld0, qstride0;
  double gamma, mu, prandtl, beta, tau;
};

hipError_t launch_negscale(int nvars, int nupts, int64_t ld, int64_t nelem, const double *rcpdjac,
                           const double *lam, double *lt, hipStream_t s);
hipError_t launch_tflux_vjp(const AdjPointArgs &a, int ns, hipStream_t s);
hipError_t launch_gradcoru_t(const AdjPointArgs &a, hipStream_t s);
hipError_t launch_comm_flux_vjp(const AdjPairArgs &a, int ns, hipStream_t s);
hipError_t launch_con_u_vjp(const AdjPairArgs &a, hipStream_t s);
hipError_t launch_axpy_dt(int64_t len, int64_t ld, int64_t nelem, const int32_t *prob,
                          const double *dt, double c, const double *x, const double *y,
                          double *out, hipStream_t s);
// RK4 step adjoint bookkeeping: acc = (first ? lam : acc) + w and
// kb = ca dt lam + cb dt w.  With rcpdjac (the state's nvars fields per
// point), kb is written already scaled for the right-hand side's adjoint:
// -J^-1 kb (0 in padding), what the negscale kernel would make of it.  With
// lcopy, lam is also copied there (lam and acc may then be one array).
hipError_t launch_rk_adj(int64_t len, int64_t ld, int64_t nelem, const int32_t *prob,
                         const double *dt, double ca, double cb, const double *lam,
                         const double *w, double *acc, double *kb, int first, int nvars,
                         const double *rcpdjac, double *lcopy, hipStream_t s);

hipError_t launch_ke_grad(int nvars, int ndims, int nupts, int64_t ld, int64_t nelem,
                          const double *wdjac, const double *u, double *g, hipStream_t s);

}  // namespace fr
