// LDS-staged sparse operator product: C = A [B1; B2] for a structurally
// sparse A (kernel template; instantiated in spop_lds_f64.hip and
// spop_lds_f32.hip).
//
// A workgroup owns 64 state columns (one per lane) and all M rows of the
// output.  The K rows of B are streamed through LDS in chunks of at most kc
// (<= kStagedRows) rows.  Each wavefront loads every fourth row of a chunk into registers
// with all its loads in flight at once (buffer loads whose range is empty
// past the chunk's last row or the last column: no branches, no memory
// access there), and the loads of chunk c + 1 are issued before chunk c is
// used, so they overlap its arithmetic.  Each wavefront then accumulates its
// quarter of the output rows (rows w, w + 4, ...) in registers from LDS,
// using the chunk's ELL entries (wave-uniform, scalar loads; padding entries
// have value 0 and a column inside the chunk).  HBM sees each input once and
// each output once: no B row is fetched twice from outside the workgroup,
// however many operator rows use it.
#pragma once

#include "buffer.h"
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
  // rows of one chunk a wavefront loads: chunks hold at most kStagedRows
  // rows (checked by the launcher), 64 KB of FP64 or 32 KB of FP32 values
  constexpr int KCW = kStagedRows / 4;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t col = (int64_t)blockIdx.x * 64 + lane;
  const bool cvalid = col < g.N;
  const char *B1 = (const char *)g.B1 + (int64_t)blockIdx.y * g.sB1 * (int64_t)sizeof(TB1);
  const char *B2 = (const char *)g.B2;
  const int K1 = g.K1;
  // a row of B: its N live columns in bytes (N <= ldb < 2^29, checked by the
  // launcher), this lane's byte offset in it
  const int nb1 = (int)(g.N * (int64_t)sizeof(TB1)), nb2 = (int)(g.N * (int64_t)sizeof(TB2));
  const uint32_t off1 = (uint32_t)(col * (int64_t)sizeof(TB1));
  const uint32_t off2 = (uint32_t)(col * (int64_t)sizeof(TB2));
  const int64_t rs1 = g.ldb1 * (int64_t)sizeof(TB1), rs2 = g.ldb2 * (int64_t)sizeof(TB2);
  // output slots: operator rows, or (gradient transform) points whose DG
  // rows d Nu + rho are accumulated together
  constexpr int RPS = EPI == EPI_GRADT ? DG : 1;
  const int nslot = EPI == EPI_GRADT ? g.Nu : g.M;
  T acc[MR][RPS];
#pragma unroll
  for (int m = 0; m < MR; ++m)
#pragma unroll
    for (int d = 0; d < RPS; ++d) acc[m][d] = 0;

  // rows w + 4 j of chunk c into v[j] (0 past the chunk and past column N)
  auto load_chunk = [&](int c, T(&v)[KCW]) {
    const int k0 = cstart[c], kn = cstart[c + 1] - k0;
#pragma unroll
    for (int j = 0; j < KCW; ++j) {
      const int i = w + 4 * j;
      const int k = k0 + i;
      const bool in = i < kn;
      if constexpr (sizeof(TB1) == sizeof(TB2)) {
        const char *row = k < K1 ? B1 + (int64_t)k * rs1 : B2 + (int64_t)(k - K1) * rs2;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)row, 0, __builtin_amdgcn_readfirstlane(in ? nb1 : 0), kRawBufferWord3);
        v[j] = (T)load_row<TB1>(rs, off1);
      } else {
        // panels of two element types: one of the two loads has an empty range
        const __amdgpu_buffer_rsrc_t r1 = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(B1 + (int64_t)k * rs1), 0,
            __builtin_amdgcn_readfirstlane(in && k < K1 ? nb1 : 0), kRawBufferWord3);
        const __amdgpu_buffer_rsrc_t r2 = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(B2 + (int64_t)(k - K1) * rs2), 0,
            __builtin_amdgcn_readfirstlane(in && k >= K1 ? nb2 : 0), kRawBufferWord3);
        v[j] = (T)load_row<TB1>(r1, off1) + (T)load_row<TB2>(r2, off2);
      }
    }
  };
  auto store_chunk = [&](int c, const T(&v)[KCW]) {
    const int kn = cstart[c + 1] - cstart[c];
#pragma unroll
    for (int j = 0; j < KCW; ++j) {
      const int i = w + 4 * j;
      if (i < kn) lds[i * 64 + lane] = v[j];
    }
  };
  // The ELL entries this wavefront uses in a chunk (its MR slots x RPS rows
  // x W entries) are held across the lanes of a few registers, one entry
  // per lane, loaded with vector loads (prefetched with the chunk's rows);
  // the product reads each back with v_readlane at a compile-time lane.
  // No scalar memory access sits between the LDS reads, which therefore
  // stay in flight together.
  constexpr int NE = MR * RPS * W;
  constexpr int NEV = (NE + 63) / 64;
  auto load_ell = [&](int c, uint32_t(&ec)[NEV], uint32_t(&el)[NEV], uint32_t(&eh)[NEV]) {
#pragma unroll
    for (int q = 0; q < NEV; ++q) {
      const int j = lane + 64 * q;
      const int m = j / (RPS * W), d = (j / W) % RPS, e = j % W;
      const int slot = w + 4 * m;
      const bool ok = j < NE && slot < nslot;
      const int row = EPI == EPI_GRADT ? d * g.Nu + slot : slot;
      const int64_t at = ok ? ((int64_t)c * g.M + row) * W + e : 0;
      const uint64_t bits = __builtin_bit_cast(uint64_t, vals[at]);
      ec[q] = ok ? (uint32_t)colidx[at] : 0u;
      el[q] = ok ? (uint32_t)bits : 0u;
      eh[q] = ok ? (uint32_t)(bits >> 32) : 0u;
    }
  };
  auto compute = [&](const uint32_t(&ec)[NEV], const uint32_t(&el)[NEV],
                     const uint32_t(&eh)[NEV]) {
    // (slots past the last row hold zero entries: they are computed, with
    // no branch between the rows, and never stored)
#pragma unroll
    for (int m = 0; m < MR; ++m) {
#pragma unroll
      for (int d = 0; d < RPS; ++d) {
        T s = 0;
#pragma unroll
        for (int e = 0; e < W; ++e) {
          const int j = (m * RPS + d) * W + e;
          const int k = __builtin_amdgcn_readlane((int)ec[j / 64], j % 64);
          const uint64_t bits =
              ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)eh[j / 64], j % 64) << 32) |
              (uint32_t)__builtin_amdgcn_readlane((int)el[j / 64], j % 64);
          s += (T)__builtin_bit_cast(double, bits) * lds[k * 64 + lane];
        }
        acc[m][d] += s;
      }
    }
  };

  T v[KCW];
  uint32_t ec[NEV], el[NEV], eh[NEV], nc_[NEV], nl[NEV], nh[NEV];
  load_ell(0, ec, el, eh);
  load_chunk(0, v);
  for (int c = 0; c < nchunk; ++c) {
    if (c > 0) __syncthreads();  // every wavefront is done with chunk c - 1
    store_chunk(c, v);
    __syncthreads();
    if (c + 1 < nchunk) {  // in flight while chunk c is used
      load_ell(c + 1, nc_, nl, nh);
      load_chunk(c + 1, v);
    }
    compute(ec, el, eh);
#pragma unroll
    for (int q = 0; q < NEV; ++q) {
      ec[q] = nc_[q];
      el[q] = nl[q];
      eh[q] = nh[q];
    }
  }
  if (!cvalid) return;

  int64_t n = 0;
  if (EPI == EPI_NEGDIV || EPI == EPI_RK || EPI == EPI_GRADT) n = col % g.ld;
  const bool live = n < g.nelem;
  double dtv = 0;
  if (EPI == EPI_RK && live) dtv = g.dt[g.prob ? g.prob[n] : 0];
  if constexpr (EPI == EPI_GRADT) {
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      const int slot = w + 4 * m;
      if (slot >= nslot) break;
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
    }
    return;
  }
  // Outputs eight rows at a time, with every load they need (1/J; for the
  // RK4 update the state, read unless this is the last stage, and the
  // register, read unless this is a first stage that is not also the last)
  // issued before the first is used: buffer loads whose range is empty
  // where nothing is read, so no branch makes them wait one by one.
  const bool scaled = EPI == EPI_NEGDIV || EPI == EPI_RK;
  const int nrj = scaled ? (int)(g.nelem * (int64_t)sizeof(double)) : 0;
  const int nro = EPI == EPI_RK && !g.rk.last ? -1 : 0;
  const int nra = EPI == EPI_RK && !(g.rk.first && !g.rk.last) ? -1 : 0;
  const uint32_t offc = (uint32_t)(col * (int64_t)sizeof(double));
  const uint32_t offn = (uint32_t)(n * (int64_t)sizeof(double));
  constexpr int G = MR < 8 ? MR : 8;
  static_assert(MR % G == 0, "rows per wavefront in groups of eight");
#pragma unroll
  for (int m0 = 0; m0 < MR; m0 += G) {
    if (w + 4 * m0 >= nslot) break;
    double rjv[G], u0v[G], accv[G];
    if constexpr (scaled) {
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const int64_t r = w + 4 * (m0 + q);
        rjv[q] = load_row<double>(uniform_rsrc(g.rcpdjac + r * g.ld, r < nslot ? nrj : 0), offn);
        if constexpr (EPI == EPI_RK) {
          u0v[q] = load_row<double>(uniform_rsrc(g.out + r * g.ldc, r < nslot ? nro : 0), offc);
          accv[q] = load_row<double>(uniform_rsrc(g.acc + r * g.ldc, r < nslot ? nra : 0), offc);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int m = m0 + q;
      const int slot = w + 4 * m;
      if (slot >= nslot) break;
      const int64_t idx = (int64_t)slot * g.ldc + col;
      if (EPI == EPI_STORE) {
        ((TC *)g.C)[(int64_t)blockIdx.y * g.sC + idx] = (TC)acc[m][0];
      } else if (EPI == EPI_ADD) {
        TC *cp = (TC *)g.C + (int64_t)blockIdx.y * g.sC + idx;
        *cp = (TC)((double)*cp + (double)acc[m][0]);
      } else {
        // padding columns: exactly 0 whatever they hold (even NaN)
        const double kk = live ? -rjv[q] * (double)acc[m][0] : 0.0;
        if (EPI == EPI_NEGDIV) {
          g.out[idx] = kk;
        } else {
          const double bdt = g.rk.b * dtv * kk;
          if (g.rk.last) {
            g.out[idx] = accv[q] + bdt;
          } else {
            const double u0 = u0v[q];
            g.acc[idx] = (g.rk.first ? u0 : accv[q]) + bdt;
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
    // C^f and the state's deviation (deviation form), both FP32
    spop_lds_go<T, EPI, W, MR, float, float, float, DG>(g, op, batch, s);
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
  if (op.kc < 1 || op.kc > kStagedRows || op.nchunk < 1 || !op.cstart || !op.cwidth)
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
      if (sizeof(T) == 4 && (!g.b1_f32 || !g.b2_f32 || !g.c_f32)) return hipErrorInvalidValue;
      if (g.D == 2) return spop_lds_width_t<T, EPI_GRADT, 2>(g, op, batch, s);
      if (g.D == 3) return spop_lds_width_t<T, EPI_GRADT, 3>(g, op, batch, s);
      return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
}

}  // namespace fr
