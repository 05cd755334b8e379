// LDS-staged sparse operator product: C = A [B1; B2] for a structurally
// sparse A (kernel template; instantiated in spop_lds_f64.hip and
// spop_lds_f32.hip).
//
// A workgroup owns 64 state columns (one per lane) and all M rows of the
// output.  The K rows of B are streamed through one LDS buffer in chunks of
// kc rows: every wavefront loads whole 64-column rows of the chunk (coalesced,
// all loads independent), then each wavefront accumulates its quarter of the
// output rows (rows w, w + 4, ...) in registers from LDS, using the chunk's
// ELL entries (wave-uniform, scalar loads).  HBM sees each input once and
// each output once; no B row is fetched twice from outside the workgroup,
// however many operator rows use it.
#pragma once

#include "kernels.h"

namespace fr {

template <typename T, int EPI, int W, int MR, typename TB1, typename TB2, typename TC, int DG>
__global__ __launch_bounds__(256) void spop_lds_kernel(GemmArgs g,
                                                       const int32_t *__restrict__ colidx,
                                                       const double *__restrict__ vals, int kc,
                                                       int nchunk,
                                                       const int32_t *__restrict__ cstart,
                                                       const int32_t *__restrict__ cwidth) {
  extern __shared__ __align__(16) unsigned char spop_smem[];
  T *lds = reinterpret_cast<T *>(spop_smem);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t col = (int64_t)blockIdx.x * 64 + lane;
  const bool cvalid = col < g.N;
  const TB1 *__restrict__ B1 = (const TB1 *)g.B1 + (int64_t)blockIdx.y * g.sB1;
  const TB2 *__restrict__ B2 = (const TB2 *)g.B2;
  const int K1 = g.K1, K = g.K1 + g.K2;
  // output slots: operator rows, or (gradient transform) points whose DG
  // rows d Nu + rho are accumulated together
  constexpr int RPS = EPI == EPI_GRADT ? DG : 1;
  const int nslot = EPI == EPI_GRADT ? g.Nu : g.M;
  T acc[MR][RPS];
#pragma unroll
  for (int m = 0; m < MR; ++m)
#pragma unroll
    for (int d = 0; d < RPS; ++d) acc[m][d] = 0;

  for (int c = 0; c < nchunk; ++c) {
    const int k0 = cstart[c];
    const int kn = cstart[c + 1] - k0;
    const int wc = cwidth[c];
    for (int i = w; i < kn; i += 4) {
      const int k = k0 + i;
      T v = 0;
      if (cvalid)
        v = k < K1 ? (T)B1[(int64_t)k * g.ldb1 + col] : (T)B2[(int64_t)(k - K1) * g.ldb2 + col];
      lds[i * 64 + lane] = v;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      const int slot = w + 4 * m;
      if (slot < nslot) {
#pragma unroll
        for (int d = 0; d < RPS; ++d) {
          const int row = EPI == EPI_GRADT ? d * g.Nu + slot : slot;
          const int32_t *__restrict__ ci = colidx + ((int64_t)c * g.M + row) * W;
          const double *__restrict__ cv = vals + ((int64_t)c * g.M + row) * W;
          T s = 0;
#pragma unroll
          for (int e = 0; e < W; ++e)
            if (e < wc) s += (T)cv[e] * lds[ci[e] * 64 + lane];
          acc[m][d] += s;
        }
      }
    }
    __syncthreads();
  }
  if (!cvalid) return;

  int64_t n = 0;
  if (EPI == EPI_NEGDIV || EPI == EPI_RK || EPI == EPI_GRADT) n = col % g.ld;
  const bool live = n < g.nelem;
  double dtv = 0;
  if (EPI == EPI_RK && live) dtv = g.dt[g.prob ? g.prob[n] : 0];
#pragma unroll
  for (int m = 0; m < MR; ++m) {
    const int slot = w + 4 * m;
    if (slot >= nslot) break;
    if constexpr (EPI == EPI_GRADT) {
      TC *C = (TC *)g.C;
      const int64_t plane = (int64_t)g.Nu * g.ld, pt = (int64_t)slot * g.ld + n;
      if (live) {
        const double rj = g.rcpdjac[pt];
#pragma unroll
        for (int j = 0; j < DG; ++j) {
          double sj = 0;
#pragma unroll
          for (int i = 0; i < DG; ++i) sj += g.smat[(i * DG + j) * plane + pt] * (double)acc[m][i];
          C[(int64_t)(j * g.Nu + slot) * g.ldc + col] = (TC)(rj * sj);
        }
      } else {
#pragma unroll
        for (int j = 0; j < DG; ++j) C[(int64_t)(j * g.Nu + slot) * g.ldc + col] = (TC)acc[m][j];
      }
    } else {
      const int64_t idx = (int64_t)slot * g.ldc + col;
      if (EPI == EPI_STORE) {
        ((TC *)g.C)[(int64_t)blockIdx.y * g.sC + idx] = (TC)acc[m][0];
      } else if (EPI == EPI_ADD) {
        TC *cp = (TC *)g.C + (int64_t)blockIdx.y * g.sC + idx;
        *cp = (TC)((double)*cp + (double)acc[m][0]);
      } else {
        const double kk = live ? -g.rcpdjac[(int64_t)slot * g.ld + n] * (double)acc[m][0] : 0.0;
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
}

template <typename T, int EPI, int W, int MR, typename TB1, typename TB2, typename TC, int DG>
void spop_lds_go(const GemmArgs &g, const StagedOp &op, int batch, hipStream_t s) {
  dim3 grid((unsigned)((g.N + 63) / 64), batch);
  const size_t shmem = (size_t)op.kc * 64 * sizeof(T);
  spop_lds_kernel<T, EPI, W, MR, TB1, TB2, TC, DG><<<grid, 256, shmem, s>>>(
      g, op.colidx, op.vals, op.kc, op.nchunk, op.cstart, op.cwidth);
}

// Operand types by precision and epilogue (as for the other operator kernels).
template <typename T, int EPI, int W, int MR, int DG>
void spop_lds_types(const GemmArgs &g, const StagedOp &op, int batch, hipStream_t s) {
  if constexpr (sizeof(T) == 8) {
    spop_lds_go<T, EPI, W, MR, double, double, double, DG>(g, op, batch, s);
  } else if constexpr (EPI == EPI_NEGDIV || EPI == EPI_RK) {
    spop_lds_go<T, EPI, W, MR, float, float, double, DG>(g, op, batch, s);
  } else if constexpr (EPI == EPI_GRADT) {
    spop_lds_go<T, EPI, W, MR, float, double, float, DG>(g, op, batch, s);
  } else {
    if (!g.b1_f32) spop_lds_go<T, EPI, W, MR, double, double, float, DG>(g, op, batch, s);
    else if (!g.b2_f32) spop_lds_go<T, EPI, W, MR, float, double, float, DG>(g, op, batch, s);
    else spop_lds_go<T, EPI, W, MR, float, float, float, DG>(g, op, batch, s);
  }
}

template <typename T, int EPI, int W, int DG>
hipError_t spop_lds_rows(const GemmArgs &g, const StagedOp &op, int batch, hipStream_t s) {
  const int nslot = EPI == EPI_GRADT ? g.Nu : g.M;
  const int need = (nslot + 3) / 4;
#define FR_R(MR_)                                                              \
  if (need <= MR_) {                                                           \
    if constexpr (EPI == EPI_GRADT && MR_ > FR_LDS_GRADT_ROWS_MAX)             \
      return hipErrorInvalidValue;                                             \
    else {                                                                     \
      spop_lds_types<T, EPI, W, MR_, DG>(g, op, batch, s);                     \
      return hipGetLastError();                                                \
    }                                                                          \
  }
  FR_LDS_ROWS(FR_R)
#undef FR_R
  return hipErrorInvalidValue;
}

template <typename T, int EPI, int DG>
hipError_t spop_lds_width_t(const GemmArgs &g, const StagedOp &op, int batch, hipStream_t s) {
  switch (op.width) {
#define FR_W(W_) \
  case W_: return spop_lds_rows<T, EPI, W_, DG>(g, op, batch, s);
    FR_LDS_WIDTHS(FR_W)
#undef FR_W
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t spop_lds_prec(int epi, const GemmArgs &g, const StagedOp &op, int batch, hipStream_t s) {
  if (g.N <= 0) return hipSuccess;
  if (op.kc < 1 || op.nchunk < 1 || !op.cstart || !op.cwidth ||
      (int64_t)op.kc * 64 * sizeof(T) > 65536)
    return hipErrorInvalidValue;
  switch (epi) {
    case EPI_STORE: return spop_lds_width_t<T, EPI_STORE, 0>(g, op, batch, s);
    case EPI_NEGDIV: return spop_lds_width_t<T, EPI_NEGDIV, 0>(g, op, batch, s);
    case EPI_RK: return spop_lds_width_t<T, EPI_RK, 0>(g, op, batch, s);
    case EPI_ADD:
      if constexpr (sizeof(T) == 8) return spop_lds_width_t<T, EPI_ADD, 0>(g, op, batch, s);
      return hipErrorInvalidValue;
    case EPI_GRADT:
      if (batch != 1 || !g.smat || g.Nu * g.D != g.M) return hipErrorInvalidValue;
      if (sizeof(T) == 4 && (!g.b1_f32 || g.b2_f32 || !g.c_f32)) return hipErrorInvalidValue;
      if (g.D == 2) return spop_lds_width_t<T, EPI_GRADT, 2>(g, op, batch, s);
      if (g.D == 3) return spop_lds_width_t<T, EPI_GRADT, 3>(g, op, batch, s);
      return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
}

}  // namespace fr
