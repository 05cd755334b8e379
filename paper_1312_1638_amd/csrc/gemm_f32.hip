// FP32 operator GEMMs (v_mfma_f32_16x16x4f32), every instantiated shape.
#include "gemm.h"

namespace fr {

hipError_t launch_gemm_f32(int epi, const GemmArgs &g, int batch, hipStream_t s) {
  if (epi == EPI_STORE) return launch_gemm_epi<float, EPI_STORE>(g, batch, s);
  if (epi == EPI_NEGDIV) return launch_gemm_epi<float, EPI_NEGDIV>(g, batch, s);
  if (epi == EPI_ADD) return hipErrorInvalidValue;
  return launch_gemm_epi<float, EPI_RK>(g, batch, s);
}

}  // namespace fr
