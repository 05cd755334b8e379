// Sparse-row operator kernel with every field of an element in one thread
// (4 fields in 2-D, 5 in 3-D); kernel in spop.h.
#include "spop.h"

namespace fr {

hipError_t launch_spop_fields4(int prec, int epi, const GemmArgs &g, const SparseOp &sp,
                               int batch, hipStream_t s) {
  return launch_spop_f<4>(prec, epi, g, sp, batch, s);
}

hipError_t launch_spop_fields5(int prec, int epi, const GemmArgs &g, const SparseOp &sp,
                               int batch, hipStream_t s) {
  return launch_spop_f<5>(prec, epi, g, sp, batch, s);
}

hipError_t launch_spop_multi_fields(int prec, int epi, const GemmArgs &g, int width, int fields,
                                    int batch, hipStream_t s) {
  if (fields == 4) return launch_spop_multi_f<4>(prec, epi, g, width, batch, s);
  if (fields == 5) return launch_spop_multi_f<5>(prec, epi, g, width, batch, s);
  return hipErrorInvalidValue;
}

}  // namespace fr
