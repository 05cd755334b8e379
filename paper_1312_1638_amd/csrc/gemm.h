// Operator GEMM on the matrix cores (Appendix A products C <- A B).
//
// One wavefront computes MBW 16-row blocks x NC 16-column strips of C.  The
// operator A is pre-packed on the host in fragment order ([row group][k
// step][row block][64 lanes], lane l holding A[16 m + l % 16][4 ks + l / 16])
// so each fragment is one 512-byte contiguous read that stays in L2; each
// fragment feeds NC MFMAs and each B fragment (4 rows x 16 columns of the
// SoA state, 128 contiguous bytes per row) feeds MBW.  The k loop runs in
// chunks of KC k-steps whose fragments are loaded one chunk ahead.  WM
// wavefronts split the rows of one column tile when the tile count alone
// would not fill the GPU.
#pragma once

#include "kernels.h"

namespace fr {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// Output lane layouts differ: register r of lane l holds row 4 r + l / 16 for
// v_mfma_f64_16x16x4f64 and row 4 (l / 16) + r for v_mfma_f32_16x16x4f32
// (column l % 16 in both; inputs A[l % 16][l / 16], B[l / 16][l % 16]).
template <typename T> struct Mma;
template <> struct Mma<double> {
  typedef dbl4 acc_t;
  static __device__ __forceinline__ int row(int kq, int r) { return 4 * r + kq; }
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mma<float> {
  typedef flt4 acc_t;
  static __device__ __forceinline__ int row(int kq, int r) { return 4 * kq + r; }
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

template <typename T, typename TB>
__device__ __forceinline__ T load_b(const TB *__restrict__ B, int64_t ldb, int K, int ks, int kq,
                                    int64_t col) {
  const int k = ks * 4 + kq;
  return k < K ? (T)B[(int64_t)k * ldb + col] : (T)0;
}

template <int MBW, int NC> struct Chunk {
  static constexpr int L = MBW + NC;
  static constexpr int KC = L >= 12 ? 1 : (16 / L > 4 ? 4 : 16 / L);
};

// MULTI: a multi-block launch that reads each workgroup's block from g.slots
// (a separate instantiation: slot loads through a generic pointer count as
// divergent and would spread to the single-block kernel's addressing).
template <typename T, int MBW, int NC, int EPI, typename TB1, typename TB2, typename TC,
          bool MULTI = false>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  typedef typename Mma<T>::acc_t acc_t;
  constexpr int KC = Chunk<MBW, NC>::KC;
  const int lane = threadIdx.x & 63;
  // multi-block launch: this workgroup's block and its index within it
  int64_t wg = blockIdx.x;
  if constexpr (MULTI) wg = take_slot(g, wg, sizeof(TB1), sizeof(TB2), sizeof(TC));
  const int64_t gw = wg * 4 + (threadIdx.x >> 6);
  const int rg = (int)(gw % g.WM);
  const int64_t n0 = (gw / g.WM) * (16 * NC);
  if (n0 >= g.N) return;
  const int col = lane & 15, kq = lane >> 4;
  const int KS1 = g.KS1, KS = g.KS1 + g.KS2;
  const TB1 *__restrict__ B1 = (const TB1 *)g.B1 + (int64_t)blockIdx.y * g.sB1;
  const TB2 *__restrict__ B2 = (const TB2 *)g.B2;
  const T *__restrict__ A = (const T *)g.Apack + (int64_t)rg * KS * MBW * 64 + lane;
  bool live_strip[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) live_strip[c] = n0 + 16 * c < g.N;

  acc_t acc[MBW][NC];
#pragma unroll
  for (int m = 0; m < MBW; ++m)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[m][c] = acc_t{0, 0, 0, 0};

  T b0[KC][NC], b1[KC][NC], a0[KC][MBW], a1[KC][MBW];
  auto load = [&](int ch, T (&b)[KC][NC], T (&a)[KC][MBW]) {
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int ks = ch * KC + kk;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int64_t bc = n0 + 16 * c + col;
        if (!live_strip[c]) b[kk][c] = 0;
        else if (ks < KS1) b[kk][c] = load_b<T>(B1, g.ldb1, g.K1, ks, kq, bc);
        else if (ks < KS) b[kk][c] = load_b<T>(B2, g.ldb2, g.K2, ks - KS1, kq, bc);
        else b[kk][c] = 0;
      }
#pragma unroll
      for (int m = 0; m < MBW; ++m) a[kk][m] = ks < KS ? A[((int64_t)ks * MBW + m) * 64] : (T)0;
    }
  };
  auto compute = [&](const T (&b)[KC][NC], const T (&a)[KC][MBW]) {
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
#pragma unroll
      for (int m = 0; m < MBW; ++m)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[m][c] = Mma<T>::run(a[kk][m], b[kk][c], acc[m][c]);
  };
  const int nch = (KS + KC - 1) / KC;
  load(0, b0, a0);
  for (int ch = 0; ch < nch; ch += 2) {
    if (ch + 1 < nch) load(ch + 1, b1, a1);
    compute(b0, a0);
    if (ch + 1 >= nch) break;
    if (ch + 2 < nch) load(ch + 2, b0, a0);
    compute(b1, a1);
  }

  // epilogue: lane holds rows 16 m + Mma<T>::row(kq, r) of column n0 + 16 c + col
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (!live_strip[c]) continue;
    const int64_t s0 = n0 + 16 * c;
    const int64_t colg = s0 + col;
    int64_t n = 0;
    if (EPI == EPI_NEGDIV || EPI == EPI_RK) n = colg - (s0 / g.ld) * g.ld;
    const bool live = n < g.nelem;
    double dtv = 0;
    if (EPI == EPI_RK && live) dtv = g.dt[g.prob ? g.prob[n] : 0];
#pragma unroll
    for (int m = 0; m < MBW; ++m) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = (rg * MBW + m) * 16 + Mma<T>::row(kq, r);
        if (row >= g.M) continue;
        const double v = (double)acc[m][c][r];
        const int64_t idx = (int64_t)row * g.ldc + colg;
        if (EPI == EPI_STORE) {
          ((TC *)g.C)[(int64_t)blockIdx.y * g.sC + idx] = (TC)v;
        } else if (EPI == EPI_ADD) {
          TC *cp = (TC *)g.C + (int64_t)blockIdx.y * g.sC + idx;
          *cp = (TC)((double)*cp + v);
        } else {
          const double k = live ? -g.rcpdjac[(int64_t)row * g.ld + n] * v : 0.0;
          if (EPI == EPI_NEGDIV) {
            g.out[idx] = k;
          } else {
            const double bdt = g.rk.b * dtv * k;
            if (g.rk.last) {
              g.out[idx] = g.acc[idx] + bdt;
            } else {
              const double u0 = g.out[idx];
              g.acc[idx] = (g.rk.first ? u0 : g.acc[idx]) + bdt;
              g.stage[idx] = u0 + g.rk.a_next * dtv * k;
            }
          }
        }
      }
    }
  }
}

// Instantiated (MBW, NC) shapes; the dispatcher maps a runtime plan to one.
#define FR_GEMM_SHAPES(X)                                                                 \
  X(1, 1) X(1, 2) X(1, 4) X(2, 1) X(2, 2) X(2, 4) X(3, 1) X(3, 2) X(3, 4) X(4, 1)       \
  X(4, 2) X(4, 4) X(6, 1) X(6, 2) X(6, 4) X(8, 1) X(8, 2) X(12, 1) X(12, 2)

template <typename T, int MBW, int NC, int EPI, bool MULTI>
void launch_gemm_kind(const GemmArgs &g, dim3 grid, hipStream_t s) {
  if constexpr (sizeof(T) == 8) {
    gemm_kernel<T, MBW, NC, EPI, double, double, double, MULTI><<<grid, 256, 0, s>>>(g);
  } else if constexpr (EPI == EPI_NEGDIV || EPI == EPI_RK) {
    gemm_kernel<T, MBW, NC, EPI, float, float, double, MULTI><<<grid, 256, 0, s>>>(g);
  } else {
    if (!g.b1_f32)
      gemm_kernel<T, MBW, NC, EPI, double, double, float, MULTI><<<grid, 256, 0, s>>>(g);
    else if (!g.b2_f32)
      gemm_kernel<T, MBW, NC, EPI, float, double, float, MULTI><<<grid, 256, 0, s>>>(g);
    else
      gemm_kernel<T, MBW, NC, EPI, float, float, float, MULTI><<<grid, 256, 0, s>>>(g);
  }
}

template <typename T, int MBW, int NC, int EPI>
hipError_t launch_gemm_shape(const GemmArgs &g, int batch, hipStream_t s) {
  if (g.slots) {
    // multi-block launch: every slot's workgroups (the -1/J and RK4
    // epilogues write through out and the RK registers)
    if ((EPI == EPI_NEGDIV || EPI == EPI_RK) && !g.out) return hipErrorInvalidValue;
    if (EPI == EPI_RK && (!g.acc || !g.dt || (!g.rk.last && !g.stage))) return hipErrorInvalidValue;
    if (EPI == EPI_STORE && !g.C) return hipErrorInvalidValue;
    launch_gemm_kind<T, MBW, NC, EPI, true>(g, dim3((unsigned)g.nwg, batch), s);
  } else {
    const int64_t wgs = gemm_workgroups(g.N, NC, g.WM);
    launch_gemm_kind<T, MBW, NC, EPI, false>(g, dim3((unsigned)wgs, batch), s);
  }
  return hipGetLastError();
}

template <typename T, int EPI>
hipError_t launch_gemm_epi(const GemmArgs &g, int batch, hipStream_t s) {
#define FR_CASE(MB_, NC_) \
  if (g.MBW == MB_ && g.NC == NC_) return launch_gemm_shape<T, MB_, NC_, EPI>(g, batch, s);
  FR_GEMM_SHAPES(FR_CASE)
#undef FR_CASE
  return hipErrorInvalidValue;
}

}  // namespace fr
