// Host side of the operator GEMM: packing of operators into fragment order,
// plan enumeration (for the autotuner), dispatch by precision.
#include <algorithm>
#include <cstring>

#include "kernels.h"

namespace fr {

static const int kShapes[][2] = {{1, 1}, {1, 2}, {1, 4}, {2, 1}, {2, 2}, {2, 4}, {3, 1},
                                 {3, 2}, {3, 4}, {4, 1}, {4, 2}, {4, 4}, {6, 1}, {6, 2},
                                 {6, 4}, {8, 1}, {8, 2}, {12, 1}, {12, 2}};

bool gemm_plan_valid(int MBW, int NC) {
  for (auto &s : kShapes)
    if (s[0] == MBW && s[1] == NC) return true;
  return false;
}

bool gemm_plan_valid(int MBW, int NC, int WM, int prec) {
  if (NC >= 64) {
    bool ok = false;
#define FR_CASE(MB_, WM_, TW_) ok = ok || (MB_ == MBW && WM_ == WM && TW_ == NC);
    FR_BF16_LDS_SHAPES(FR_CASE)
#undef FR_CASE
    return ok && prec == PREC_BF16X3;
  }
  return gemm_plan_valid(MBW, NC);
}

static int round_mbw(int need) {
  const int vals[] = {1, 2, 3, 4, 6, 8, 12};
  for (int v : vals)
    if (v >= need) return v;
  return -1;
}

GemmPlan gemm_plan(int M, int64_t N, int prec) {
  (void)prec;
  const int MB = (M + 15) / 16;
  const int64_t ntile = (N + 15) / 16;
  int wm = (MB + 11) / 12;
  while (wm < MB && wm * ntile < 4096) ++wm;
  int mbw = round_mbw((MB + wm - 1) / wm);
  wm = (MB + mbw - 1) / mbw;
  return GemmPlan{mbw, 1, wm};
}

std::vector<GemmPlan> gemm_candidates(int M, int64_t N, int prec) {
  std::vector<GemmPlan> out;
  const int MB = (M + 15) / 16;
  if (prec == PREC_BF16X3) {
    // LDS-staged plans: for each row split WM and column tile TW, the
    // smallest instantiated MBW that covers the rows
    for (int wm : {1, 2, 4})
      for (int tw : {64, 128}) {
        int best = 0;
#define FR_CASE(MB_, WM_, TW_) \
  if (WM_ == wm && TW_ == tw && MB_ * WM_ >= MB && (best == 0 || MB_ < best)) best = MB_;
        FR_BF16_LDS_SHAPES(FR_CASE)
#undef FR_CASE
        if (best && N >= tw) out.push_back(GemmPlan{best, tw, wm});
      }
  }
  for (int wm = 1; wm <= std::min(MB, 12); ++wm) {
    const int mbw = round_mbw((MB + wm - 1) / wm);
    if (mbw < 0) continue;
    const int wmr = (MB + mbw - 1) / mbw;
    if (wmr != wm) continue;  // same plan as a smaller wm
    for (int nc : {1, 2, 4}) {
      if (!gemm_plan_valid(mbw, nc)) continue;
      if (16 * nc > N) continue;
      out.push_back(GemmPlan{mbw, nc, wm});
    }
  }
  return out;
}

int64_t gemm_pack_size(int M, int K1, int K2, int MBW, int WM, int kstep) {
  (void)M;
  const int KS = (K1 + kstep - 1) / kstep + (K2 + kstep - 1) / kstep;
  return (int64_t)WM * KS * MBW * 64;
}

template <typename T>
static void gemm_pack(const double *A, int M, int K1, int K2, int MBW, int WM, T *dst) {
  const int KS1 = (K1 + 3) / 4, KS2 = (K2 + 3) / 4, KS = KS1 + KS2, K = K1 + K2;
  for (int rg = 0; rg < WM; ++rg)
    for (int ks = 0; ks < KS; ++ks)
      for (int m = 0; m < MBW; ++m)
        for (int l = 0; l < 64; ++l) {
          const int row = (rg * MBW + m) * 16 + (l & 15);
          const int kk = ks < KS1 ? ks * 4 + (l >> 4) : (ks - KS1) * 4 + (l >> 4);
          const bool ok = ks < KS1 ? kk < K1 : kk < K2;
          const int acol = ks < KS1 ? kk : K1 + kk;
          const double v = (row < M && ok) ? A[(int64_t)row * K + acol] : 0.0;
          dst[(((int64_t)rg * KS + ks) * MBW + m) * 64 + l] = (T)v;
        }
}

void gemm_pack_f64(const double *A, int M, int K1, int K2, int MBW, int WM, double *dst) {
  gemm_pack<double>(A, M, K1, K2, MBW, WM, dst);
}
void gemm_pack_f32(const double *A, int M, int K1, int K2, int MBW, int WM, float *dst) {
  gemm_pack<float>(A, M, K1, K2, MBW, WM, dst);
}

hipError_t launch_gemm(int prec, int epi, const GemmArgs &g, int batch, hipStream_t s) {
  if (g.N <= 0) return hipSuccess;
  if (prec == PREC_F64) return launch_gemm_f64(epi, g, batch, s);
  if (prec == PREC_F32) return launch_gemm_f32(epi, g, batch, s);
  if (prec == PREC_BF16X3) return launch_gemm_bf16x3(epi, g, batch, s);
  return hipErrorInvalidValue;
}

// round-to-nearest-even of an FP32 value to bf16 (bit pattern)
static uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static double bf16_to_double(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

int64_t gemm_pack_size_bf16(int M, int K1, int K2, int MBW, int WM) {
  (void)M;
  const int KS = (K1 + 31) / 32 + (K2 + 31) / 32;
  return (int64_t)WM * KS * MBW * 2 * 64 * 8;
}

void gemm_pack_bf16x3(const double *A, int M, int K1, int K2, int MBW, int WM, uint16_t *dst) {
  const int KS1 = (K1 + 31) / 32, KS2 = (K2 + 31) / 32, KS = KS1 + KS2, K = K1 + K2;
  for (int rg = 0; rg < WM; ++rg)
    for (int ks = 0; ks < KS; ++ks)
      for (int m = 0; m < MBW; ++m)
        for (int l = 0; l < 64; ++l)
          for (int j = 0; j < 8; ++j) {
            const int row = (rg * MBW + m) * 16 + (l & 15);
            const int kk = (ks < KS1 ? ks : ks - KS1) * 32 + 8 * (l >> 4) + j;
            const bool ok = ks < KS1 ? kk < K1 : kk < K2;
            const int acol = ks < KS1 ? kk : K1 + kk;
            const double v = (row < M && ok) ? A[(int64_t)row * K + acol] : 0.0;
            const uint16_t hi = bf16_rne((float)v);
            const uint16_t lo = bf16_rne((float)(v - bf16_to_double(hi)));
            const int64_t base = (((int64_t)rg * KS + ks) * MBW + m) * 2;
            dst[((base + 0) * 64 + l) * 8 + j] = hi;
            dst[((base + 1) * 64 + l) * 8 + j] = lo;
          }
}

}  // namespace fr
