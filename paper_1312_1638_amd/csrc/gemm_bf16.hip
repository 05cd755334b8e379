// BF16x3 operator GEMMs: split-precision products on the bf16 matrix cores.
//
// A (the constant operator, FP64 on the host) is split once into
// A_hi = bf16(A) and A_lo = bf16(A - A_hi); each B element (FP32 scratch or
// the FP64 state) is split on the fly the same way, and
// C = A_hi B_hi + A_hi B_lo + A_lo B_hi is accumulated in FP32 with
// v_mfma_f32_16x16x32_bf16 (Henry, Tang & Heinecke's bf16x3 scheme; the
// dropped A_lo B_lo term is ~2^-16 of the product).  Rounding to bf16 is
// round-to-nearest-even on the FP32 bit pattern.
#include "gemm.h"

namespace fr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_value(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}

template <typename TB>
__device__ __forceinline__ float load_bf(const TB *__restrict__ B, int64_t ldb, int K, int k,
                                         int64_t col) {
  return k < K ? (float)B[(int64_t)k * ldb + col] : 0.0f;
}

// Fragment layout of A: [rg][k-step of 32][row block m][hi/lo][64 lanes][8],
// lane l of fragment (m, ks) holding A[16 m + l % 16][32 ks + 8 (l / 16) + j].
template <int MBW, int NC, int EPI, typename TB1, typename TB2, typename TC>
__global__ __launch_bounds__(256) void gemm_bf16x3_kernel(GemmArgs g) {
  typedef flt4 acc_t;
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int rg = (int)(gw % g.WM);
  const int64_t n0 = (gw / g.WM) * (16 * NC);
  if (n0 >= g.N) return;
  const int col = lane & 15, kq = lane >> 4;
  const int KS1 = g.KS1, KS = g.KS1 + g.KS2;
  const TB1 *__restrict__ B1 = (const TB1 *)g.B1 + (int64_t)blockIdx.y * g.sB1;
  const TB2 *__restrict__ B2 = (const TB2 *)g.B2;
  const u16x8 *__restrict__ A =
      (const u16x8 *)g.Apack + (int64_t)rg * KS * MBW * 2 * 64 + lane;
  bool live_strip[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) live_strip[c] = n0 + 16 * c < g.N;
  acc_t acc[MBW][NC];
#pragma unroll
  for (int m = 0; m < MBW; ++m)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[m][c] = acc_t{0, 0, 0, 0};

  for (int ks = 0; ks < KS; ++ks) {
    bf16x8 bh[NC], bl[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int64_t bc = n0 + 16 * c + col;
      u16x8 h, l;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        float v = 0.0f;
        if (live_strip[c]) {
          if (ks < KS1) v = load_bf(B1, g.ldb1, g.K1, ks * 32 + kq * 8 + j, bc);
          else v = load_bf(B2, g.ldb2, g.K2, (ks - KS1) * 32 + kq * 8 + j, bc);
        }
        const unsigned short hb = bf16_bits(v);
        h[j] = hb;
        l[j] = bf16_bits(v - bf16_value(hb));
      }
      bh[c] = __builtin_bit_cast(bf16x8, h);
      bl[c] = __builtin_bit_cast(bf16x8, l);
    }
#pragma unroll
    for (int m = 0; m < MBW; ++m) {
      const bf16x8 ah = __builtin_bit_cast(bf16x8, A[(((int64_t)ks * MBW + m) * 2 + 0) * 64]);
      const bf16x8 al = __builtin_bit_cast(bf16x8, A[(((int64_t)ks * MBW + m) * 2 + 1) * 64]);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[c], acc[m][c], 0, 0, 0);
        acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[c], acc[m][c], 0, 0, 0);
        acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[c], acc[m][c], 0, 0, 0);
      }
    }
  }

  // epilogue (output layout of the 16x16 f32 accumulators: row 4 (l/16) + r)
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
        const int row = (rg * MBW + m) * 16 + 4 * kq + r;
        if (row >= g.M) continue;
        const double v = (double)acc[m][c][r];
        const int64_t idx = (int64_t)row * g.ldc + colg;
        if (EPI == EPI_STORE) {
          ((TC *)g.C)[(int64_t)blockIdx.y * g.sC + idx] = (TC)v;
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

// Epilogue of one 16 x 16 FP32 accumulator block (rows 4 (l / 16) + r of
// row block `rb`, column colg of strip s0): store, -1/J, or the RK update.
template <int EPI, typename TC>
__device__ __forceinline__ void bf16_epilogue(const GemmArgs &g, const flt4 &acc, int rb, int kq,
                                              int64_t s0, int64_t colg, int64_t n, bool live,
                                              double dtv) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = rb * 16 + 4 * kq + r;
    if (row >= g.M) continue;
    const double v = (double)acc[r];
    const int64_t idx = (int64_t)row * g.ldc + colg;
    if (EPI == EPI_STORE) {
      ((TC *)g.C)[(int64_t)blockIdx.y * g.sC + idx] = (TC)v;
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

// LDS-staged form.  A workgroup of four wavefronts owns TW = 16 NCT columns
// and every row of C.  Per stage of G k-steps (32 k each) the workgroup
// loads its B tile once -- each lane 8 consecutive k of one column, so a
// wavefront load covers 64 (or 128) consecutive columns of one row --
// splits every value into bf16 hi and lo once, and stores both in LDS in
// MFMA operand order ([strip][k quarter][column], 16 bytes each).  The
// wavefronts then split the rows (WM row groups of MBW blocks) and the
// column strips (NCT WM / 4 each) and read each operand with one 16-byte
// LDS read.  Against the direct kernel, B is fetched once per workgroup
// instead of once per wavefront, with coalesced row segments instead of
// 8 strided values per lane, and split once instead of once per row group.
template <int MBW, int WM, int NCT, int EPI, typename TB1, typename TB2, typename TC>
__global__ __launch_bounds__(256) void gemm_bf16x3_lds_kernel(GemmArgs g) {
  constexpr int G = 2;                    // k-steps per LDS stage
  constexpr int TW = 16 * NCT;            // columns per workgroup
  constexpr int NCW = NCT * WM / 4;       // strips per wavefront
  constexpr int PPT = NCT / 4;            // (column, k quarter) pairs per thread per k-step
  static_assert(NCW >= 1 && NCT % 4 == 0, "strips per wavefront");
  __shared__ u16x8 sh[G][2][NCT * 64];    // [stage step][hi, lo][(strip * 4 + kq) * 16 + col]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rg = w % WM, sg = w / WM;
  const int64_t n0 = (int64_t)blockIdx.x * TW;
  const int col = lane & 15, kq = lane >> 4;
  const int KS1 = g.KS1, KS = g.KS1 + g.KS2;
  const TB1 *__restrict__ B1 = (const TB1 *)g.B1 + (int64_t)blockIdx.y * g.sB1;
  const TB2 *__restrict__ B2 = (const TB2 *)g.B2;
  const u16x8 *__restrict__ A =
      (const u16x8 *)g.Apack + (int64_t)rg * KS * MBW * 2 * 64 + lane;
  flt4 acc[MBW][NCW];
#pragma unroll
  for (int m = 0; m < MBW; ++m)
#pragma unroll
    for (int c = 0; c < NCW; ++c) acc[m][c] = flt4{0, 0, 0, 0};

  for (int ks0 = 0; ks0 < KS; ks0 += G) {
    // load the stage's B tile: all loads first, then split and store
    float v[G][PPT][8];
#pragma unroll
    for (int st = 0; st < G; ++st)
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        const int pr = (int)threadIdx.x + 256 * i;
        const int64_t bc = n0 + pr % TW;
        const int q = pr / TW;
        const int ks = ks0 + st;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          float x = 0.0f;
          if (bc < g.N && ks < KS) {
            if (ks < KS1) x = load_bf(B1, g.ldb1, g.K1, ks * 32 + q * 8 + j, bc);
            else x = load_bf(B2, g.ldb2, g.K2, (ks - KS1) * 32 + q * 8 + j, bc);
          }
          v[st][i][j] = x;
        }
      }
#pragma unroll
    for (int st = 0; st < G; ++st)
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        const int pr = (int)threadIdx.x + 256 * i;
        const int cw = pr % TW, q = pr / TW;
        u16x8 h, l;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const unsigned short hb = bf16_bits(v[st][i][j]);
          h[j] = hb;
          l[j] = bf16_bits(v[st][i][j] - bf16_value(hb));
        }
        const int at = ((cw >> 4) * 4 + q) * 16 + (cw & 15);
        sh[st][0][at] = h;
        sh[st][1][at] = l;
      }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < G; ++st) {
      const int ks = ks0 + st;
      if (ks < KS) {
        bf16x8 bh[NCW], bl[NCW];
#pragma unroll
        for (int c = 0; c < NCW; ++c) {
          const int at = ((sg * NCW + c) * 4 + kq) * 16 + col;
          bh[c] = __builtin_bit_cast(bf16x8, sh[st][0][at]);
          bl[c] = __builtin_bit_cast(bf16x8, sh[st][1][at]);
        }
#pragma unroll
        for (int m = 0; m < MBW; ++m) {
          const bf16x8 ah = __builtin_bit_cast(bf16x8, A[(((int64_t)ks * MBW + m) * 2 + 0) * 64]);
          const bf16x8 al = __builtin_bit_cast(bf16x8, A[(((int64_t)ks * MBW + m) * 2 + 1) * 64]);
#pragma unroll
          for (int c = 0; c < NCW; ++c) {
            acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[c], acc[m][c], 0, 0, 0);
            acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[c], acc[m][c], 0, 0, 0);
            acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[c], acc[m][c], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int c = 0; c < NCW; ++c) {
    const int64_t s0 = n0 + 16 * (sg * NCW + c);
    if (s0 >= g.N) continue;
    const int64_t colg = s0 + col;
    int64_t n = 0;
    if (EPI == EPI_NEGDIV || EPI == EPI_RK) n = colg - (s0 / g.ld) * g.ld;
    const bool live = n < g.nelem;
    double dtv = 0;
    if (EPI == EPI_RK && live) dtv = g.dt[g.prob ? g.prob[n] : 0];
#pragma unroll
    for (int m = 0; m < MBW; ++m)
      bf16_epilogue<EPI, TC>(g, acc[m][c], rg * MBW + m, kq, s0, colg, n, live, dtv);
  }
}

template <int MBW, int WM, int NCT, int EPI>
static hipError_t launch_bf16_lds_shape(const GemmArgs &g, int batch, hipStream_t s) {
  const int64_t tiles = (g.N + 16 * NCT - 1) / (16 * NCT);
  dim3 grid((unsigned)tiles, batch), block(256);
  if constexpr (EPI == EPI_NEGDIV || EPI == EPI_RK) {
    gemm_bf16x3_lds_kernel<MBW, WM, NCT, EPI, float, float, double><<<grid, block, 0, s>>>(g);
  } else {
    if (!g.b1_f32)
      gemm_bf16x3_lds_kernel<MBW, WM, NCT, EPI, double, double, float><<<grid, block, 0, s>>>(g);
    else if (!g.b2_f32)
      gemm_bf16x3_lds_kernel<MBW, WM, NCT, EPI, float, double, float><<<grid, block, 0, s>>>(g);
    else
      gemm_bf16x3_lds_kernel<MBW, WM, NCT, EPI, float, float, float><<<grid, block, 0, s>>>(g);
  }
  return hipGetLastError();
}

template <int MBW, int NC, int EPI>
static hipError_t launch_bf16_shape(const GemmArgs &g, int batch, hipStream_t s) {
  const int64_t tiles = (g.N + 16 * NC - 1) / (16 * NC);
  const int64_t waves = tiles * g.WM;
  dim3 grid((unsigned)((waves + 3) / 4), batch), block(256);
  if constexpr (EPI == EPI_NEGDIV || EPI == EPI_RK) {
    gemm_bf16x3_kernel<MBW, NC, EPI, float, float, double><<<grid, block, 0, s>>>(g);
  } else {
    if (!g.b1_f32)
      gemm_bf16x3_kernel<MBW, NC, EPI, double, double, float><<<grid, block, 0, s>>>(g);
    else if (!g.b2_f32)
      gemm_bf16x3_kernel<MBW, NC, EPI, float, double, float><<<grid, block, 0, s>>>(g);
    else
      gemm_bf16x3_kernel<MBW, NC, EPI, float, float, float><<<grid, block, 0, s>>>(g);
  }
  return hipGetLastError();
}

template <int EPI>
static hipError_t launch_bf16_epi(const GemmArgs &g, int batch, hipStream_t s) {
  if (g.NC >= 64) {
    // LDS-staged plans: NC is the column tile of a workgroup
#define FR_CASE(MB_, WM_, TW_)                                                \
  if (g.MBW == MB_ && g.WM == WM_ && g.NC == TW_)                             \
    return launch_bf16_lds_shape<MB_, WM_, TW_ / 16, EPI>(g, batch, s);
    FR_BF16_LDS_SHAPES(FR_CASE)
#undef FR_CASE
    return hipErrorInvalidValue;
  }
#define FR_CASE(MB_, NC_) \
  if (g.MBW == MB_ && g.NC == NC_) return launch_bf16_shape<MB_, NC_, EPI>(g, batch, s);
  FR_GEMM_SHAPES(FR_CASE)
#undef FR_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_bf16x3(int epi, const GemmArgs &g, int batch, hipStream_t s) {
  if (epi == EPI_STORE) return launch_bf16_epi<EPI_STORE>(g, batch, s);
  if (epi == EPI_NEGDIV) return launch_bf16_epi<EPI_NEGDIV>(g, batch, s);
  if (epi == EPI_RK) return launch_bf16_epi<EPI_RK>(g, batch, s);
  return hipErrorInvalidValue;
}

}  // namespace fr
