// LDS-staged sparse operator kernel, FP32 contexts (kernel in spop_lds.h).
#include "spop_lds.h"

namespace fr {

hipError_t launch_spop_lds_f32(int epi, const GemmArgs &g, const StagedOp &op, int batch,
                               hipStream_t s) {
  return spop_lds_prec<float>(epi, g, op, batch, s);
}

}  // namespace fr
