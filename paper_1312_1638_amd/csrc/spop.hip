// Sparse-row application of an operator matrix: C = A [B1; B2] where A has
// few non-zeros per row.
//
// With Gauss-Legendre points on quads and hexes every Appendix A operator
// couples only points on one coordinate line (interpolation to a face,
// differentiation along a line, the DG lifting along the face normal), so a
// row holds O(p) non-zeros out of up to a few hundred.  Applying such an
// operator as a dense product would make an HBM-bound step compute-bound;
// here each thread owns one state column (alpha, element), threads of a
// wavefront take consecutive elements (coalesced), and each workgroup row
// (blockIdx.y) takes `rpg` operator rows.  The operator is stored padded to a
// fixed width W per row (ELL: padding entries have value 0 and repeat a real
// column), W is a template parameter, so all W loads of a row are issued
// back to back; column indices and values are wave-uniform (scalar loads).
// The grid is one-dimensional and XCD-aware: workgroups are dealt round-robin
// to the 8 XCDs, and the linear id is remapped so that each XCD runs all row
// groups of one column tile back to back; re-reads of that tile's B rows then
// hit the XCD's L2 while they are still there.
#include "kernels.h"

namespace fr {

template <typename T, int EPI, int W, typename TB1, typename TB2, typename TC, int DG = 0>
__global__ __launch_bounds__(256) void spop_kernel(GemmArgs g,
                                                   const int32_t *__restrict__ colidx,
                                                   const double *__restrict__ vals, int rpg,
                                                   int ngroups) {
  // linear id L -> XCD L % 8; the j-th workgroup of an XCD takes row group
  // j % ngroups of column tile 8 (j / ngroups) + L % 8 (tiles padded to a
  // multiple of 8 by the launch)
  const int64_t L = blockIdx.x, j = L >> 3;
  const int64_t tile = (j / ngroups) * 8 + (L & 7);
  const int rgrp = (int)(j % ngroups);
  const int64_t col = tile * 256 + threadIdx.x;
  if (col >= g.N) return;
  const int r0 = rgrp * rpg;
  const int rmax = EPI == EPI_GRADT ? g.Nu : g.M;
  const int r1 = r0 + rpg < rmax ? r0 + rpg : rmax;
  const TB1 *__restrict__ B1b = (const TB1 *)g.B1 + (int64_t)blockIdx.y * g.sB1;
  const TB1 *__restrict__ B1 = B1b + col;
  const TB2 *__restrict__ B2 = (const TB2 *)g.B2 + col;
  int64_t n = 0;
  if (EPI == EPI_NEGDIV || EPI == EPI_RK || EPI == EPI_GRADT) n = col % g.ld;
  const bool live = n < g.nelem;
  double dtv = 0;
  if (EPI == EPI_RK && live) dtv = g.dt[g.prob ? g.prob[n] : 0];
  const int K1 = g.K1;
  const int64_t ldb1 = g.ldb1, ldb2 = g.ldb2;
  // B2 addressed from B1 by an element offset (same element type), so that
  // picking the panel of an entry is a uniform select, not a branch
  const int64_t d2 = ((intptr_t)g.B2 - (intptr_t)B1b) / (int64_t)sizeof(TB1);
  if constexpr (EPI == EPI_GRADT) {
    // rows d Nu + rho, d < DG, of the points rho in [r0, r1) (r1 <= Nu)
    const int64_t plane = (int64_t)g.Nu * g.ld;
    for (int rho = r0; rho < r1; ++rho) {
      double qt[DG];
#pragma unroll
      for (int d = 0; d < DG; ++d) {
        const int row = d * g.Nu + rho;
        const int32_t *__restrict__ ci = colidx + (int64_t)row * W;
        const double *__restrict__ cv = vals + (int64_t)row * W;
        T b[W];
#pragma unroll
        for (int e = 0; e < W; ++e) {
          const int k = ci[e];
          if constexpr (sizeof(TB1) == sizeof(TB2)) {
            const int64_t off = k < K1 ? (int64_t)k * ldb1 : d2 + (int64_t)(k - K1) * ldb2;
            b[e] = (T)B1[off];
          } else {
            b[e] = k < K1 ? (T)B1[(int64_t)k * ldb1] : (T)B2[(int64_t)(k - K1) * ldb2];
          }
        }
        T acc = 0;
#pragma unroll
        for (int e = 0; e < W; ++e) acc += (T)cv[e] * b[e];
        qt[d] = (double)acc;
      }
      const int64_t pt = (int64_t)rho * g.ld + n;
      TC *C = (TC *)g.C;
      if (live) {
        const double rj = g.rcpdjac[pt];
#pragma unroll
        for (int j = 0; j < DG; ++j) {
          double sj = 0;
#pragma unroll
          for (int i = 0; i < DG; ++i) sj += g.smat[(i * DG + j) * plane + pt] * qt[i];
          C[(int64_t)(j * g.Nu + rho) * g.ldc + col] = (TC)(rj * sj);
        }
      } else {
#pragma unroll
        for (int j = 0; j < DG; ++j) C[(int64_t)(j * g.Nu + rho) * g.ldc + col] = (TC)qt[j];
      }
    }
    return;
  }
#pragma unroll 2
  for (int row = r0; row < r1; ++row) {
    const int32_t *__restrict__ ci = colidx + (int64_t)row * W;
    const double *__restrict__ cv = vals + (int64_t)row * W;
    int32_t kc[W];
#pragma unroll
    for (int e = 0; e < W; ++e) kc[e] = ci[e];
    T b[W];
#pragma unroll
    for (int e = 0; e < W; ++e) {
      const int k = kc[e];
      if constexpr (sizeof(TB1) == sizeof(TB2)) {
        const int64_t off = k < K1 ? (int64_t)k * ldb1 : d2 + (int64_t)(k - K1) * ldb2;
        b[e] = (T)B1[off];
      } else {
        b[e] = k < K1 ? (T)B1[(int64_t)k * ldb1] : (T)B2[(int64_t)(k - K1) * ldb2];
      }
    }
    T acc = 0;
#pragma unroll
    for (int e = 0; e < W; ++e) acc += (T)cv[e] * b[e];
    const int64_t idx = (int64_t)row * g.ldc + col;
    if (EPI == EPI_STORE) {
      ((TC *)g.C)[(int64_t)blockIdx.y * g.sC + idx] = (TC)acc;
    } else if (EPI == EPI_ADD) {
      TC *cp = (TC *)g.C + (int64_t)blockIdx.y * g.sC + idx;
      *cp = (TC)((double)*cp + (double)acc);
    } else {
      const double kk = live ? -g.rcpdjac[(int64_t)row * g.ld + n] * (double)acc : 0.0;
      if (EPI == EPI_NEGDIV) {
        g.out[idx] = kk;
      } else {
        const double bdt = g.rk.b * dtv * kk;
        if (g.rk.last) {
          g.out[idx] = g.acc[idx] + bdt;
        } else {
          const double u0 = g.out[idx];
          g.acc[idx] = (g.rk.first ? u0 : g.acc[idx]) + bdt;
          g.stage[idx] = u0 + g.rk.a_next * dtv * kk;
        }
      }
    }
  }
}

template <typename T, int EPI, int W>
static void spop_launch_w(const GemmArgs &g, const SparseOp &sp, int batch, hipStream_t s) {
  const int64_t tiles = ((g.N + 255) / 256 + 7) / 8 * 8;
  const int ngroups = (g.M + sp.rpg - 1) / sp.rpg;
  dim3 grid((unsigned)(tiles * ngroups), batch);
  if constexpr (sizeof(T) == 8) {
    spop_kernel<T, EPI, W, double, double, double><<<grid, 256, 0, s>>>(g, sp.colidx, sp.vals, sp.rpg, ngroups);
  } else if constexpr (EPI == EPI_NEGDIV || EPI == EPI_RK) {
    spop_kernel<T, EPI, W, float, float, double><<<grid, 256, 0, s>>>(g, sp.colidx, sp.vals, sp.rpg, ngroups);
  } else {
    if (!g.b1_f32)
      spop_kernel<T, EPI, W, double, double, float><<<grid, 256, 0, s>>>(g, sp.colidx, sp.vals, sp.rpg, ngroups);
    else if (!g.b2_f32)
      spop_kernel<T, EPI, W, float, double, float><<<grid, 256, 0, s>>>(g, sp.colidx, sp.vals, sp.rpg, ngroups);
    else
      spop_kernel<T, EPI, W, float, float, float><<<grid, 256, 0, s>>>(g, sp.colidx, sp.vals, sp.rpg, ngroups);
  }
}

template <typename T, int W>
static void spop_launch_gradt(const GemmArgs &g, const SparseOp &sp, hipStream_t s) {
  const int64_t tiles = ((g.N + 255) / 256 + 7) / 8 * 8;
  const int ngroups = (g.Nu + sp.rpg - 1) / sp.rpg;
  dim3 grid((unsigned)(tiles * ngroups), 1);
  if constexpr (sizeof(T) == 8) {
    if (g.D == 2)
      spop_kernel<T, EPI_GRADT, W, double, double, double, 2><<<grid, 256, 0, s>>>(g, sp.colidx, sp.vals, sp.rpg, ngroups);
    else
      spop_kernel<T, EPI_GRADT, W, double, double, double, 3><<<grid, 256, 0, s>>>(g, sp.colidx, sp.vals, sp.rpg, ngroups);
  } else {
    // FP32 contexts: C^f in FP32 scratch (panel 1), the FP64 state (panel 2)
    if (g.D == 2)
      spop_kernel<T, EPI_GRADT, W, float, double, float, 2><<<grid, 256, 0, s>>>(g, sp.colidx, sp.vals, sp.rpg, ngroups);
    else
      spop_kernel<T, EPI_GRADT, W, float, double, float, 3><<<grid, 256, 0, s>>>(g, sp.colidx, sp.vals, sp.rpg, ngroups);
  }
}

template <typename T>
static hipError_t spop_gradt_t(const GemmArgs &g, const SparseOp &sp, hipStream_t s) {
  if ((g.D != 2 && g.D != 3) || g.Nu * g.D != g.M || !g.smat) return hipErrorInvalidValue;
  if (sizeof(T) == 4 && (!g.b1_f32 || g.b2_f32 || !g.c_f32)) return hipErrorInvalidValue;
  switch (sp.width) {
#define FR_W(W_) \
  case W_: spop_launch_gradt<T, W_>(g, sp, s); break;
    FR_SPOP_WIDTHS(FR_W)
#undef FR_W
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int EPI>
static hipError_t spop_launch_t(const GemmArgs &g, const SparseOp &sp, int batch, hipStream_t s) {
  switch (sp.width) {
#define FR_W(W_) \
  case W_: spop_launch_w<T, EPI, W_>(g, sp, batch, s); break;
    FR_SPOP_WIDTHS(FR_W)
#undef FR_W
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_spop(int prec, int epi, const GemmArgs &g, const SparseOp &sp, int batch,
                       hipStream_t s) {
  if (g.N <= 0) return hipSuccess;
  if (sp.rpg < 1) return hipErrorInvalidValue;
  if (epi == EPI_GRADT) {
    if (batch != 1) return hipErrorInvalidValue;
    if (prec == PREC_F64) return spop_gradt_t<double>(g, sp, s);
    if (prec == PREC_F32) return spop_gradt_t<float>(g, sp, s);
    return hipErrorInvalidValue;
  }
  if (prec == PREC_F64) {
    switch (epi) {
      case EPI_STORE: return spop_launch_t<double, EPI_STORE>(g, sp, batch, s);
      case EPI_NEGDIV: return spop_launch_t<double, EPI_NEGDIV>(g, sp, batch, s);
      case EPI_RK: return spop_launch_t<double, EPI_RK>(g, sp, batch, s);
      case EPI_ADD: return spop_launch_t<double, EPI_ADD>(g, sp, batch, s);
    }
  } else if (prec == PREC_F32) {
    switch (epi) {
      case EPI_STORE: return spop_launch_t<float, EPI_STORE>(g, sp, batch, s);
      case EPI_NEGDIV: return spop_launch_t<float, EPI_NEGDIV>(g, sp, batch, s);
      case EPI_RK: return spop_launch_t<float, EPI_RK>(g, sp, batch, s);
    }
  }
  return hipErrorInvalidValue;
}

int spop_width(int nnz_max) {
  int best = 0;
#define FR_W(W_) \
  if (best == 0 && W_ >= nnz_max) best = W_;
  FR_SPOP_WIDTHS(FR_W)
#undef FR_W
  return best;
}

}  // namespace fr
