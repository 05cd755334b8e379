// FP64 operator GEMMs (v_mfma_f64_16x16x4f64), every instantiated shape.
#include "gemm.h"

namespace fr {

hipError_t launch_gemm_f64(int epi, const GemmArgs &g, int batch, hipStream_t s) {
  if (epi == EPI_STORE) return launch_gemm_epi<double, EPI_STORE>(g, batch, s);
  if (epi == EPI_NEGDIV) return launch_gemm_epi<double, EPI_NEGDIV>(g, batch, s);
  if (epi == EPI_ADD) return launch_gemm_epi<double, EPI_ADD>(g, batch, s);
  return launch_gemm_epi<double, EPI_RK>(g, batch, s);
}

}  // namespace fr
