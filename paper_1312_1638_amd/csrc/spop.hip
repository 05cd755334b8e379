// Sparse-row operator kernel: one field per thread, the dispatchers over the
// fields-per-thread and LDS-staged variants, and the ELL width tables
// (kernels in spop.h and spop_lds.h).
#include "spop.h"

namespace fr {

hipError_t launch_spop(int prec, int epi, const GemmArgs &g, const SparseOp &sp, int batch,
                       hipStream_t s) {
  if (g.N <= 0) return hipSuccess;
  if (sp.rpg < 1) return hipErrorInvalidValue;
  // one row stride for both panels, and the N columns within one row of B
  // (ldb FP64 values, under 4 GiB): a column's byte offset fits 32 bits
  if (g.ldb1 <= 0 || g.ldb1 >= ((int64_t)1 << 29) || g.N > g.ldb1 ||
      (g.K2 > 0 && g.ldb2 != g.ldb1))
    return hipErrorInvalidValue;
  if (sp.fields == 1) return launch_spop_f<1>(prec, epi, g, sp, batch, s);
  if (sp.fields == 4) return launch_spop_fields4(prec, epi, g, sp, batch, s);
  if (sp.fields == 5) return launch_spop_fields5(prec, epi, g, sp, batch, s);
  return hipErrorInvalidValue;
}

hipError_t launch_spop_multi(int prec, int epi, const GemmArgs &g, int width, int fields,
                             int batch, hipStream_t s) {
  if (fields == 1) return launch_spop_multi_f<1>(prec, epi, g, width, batch, s);
  return launch_spop_multi_fields(prec, epi, g, width, fields, batch, s);
}

hipError_t launch_spop_lds(int prec, int epi, const GemmArgs &g, const StagedOp &op, int batch,
                           hipStream_t s) {
  if (prec == PREC_F64) return launch_spop_lds_f64(epi, g, op, batch, s);
  if (prec == PREC_F32) return launch_spop_lds_f32(epi, g, op, batch, s);
  return hipErrorInvalidValue;
}

int spop_lds_width(int nnz_max) {
  int best = 0;
#define FR_W(W_) \
  if (best == 0 && W_ >= nnz_max) best = W_;
  FR_LDS_WIDTHS(FR_W)
#undef FR_W
  return best;
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
