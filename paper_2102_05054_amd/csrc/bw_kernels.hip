// Brickwork random-circuit passes (Sec. 2, Eq. (U), Eq. (unitary)).
#include "op.h"

namespace fq {

struct BwProgram {};

fq_status bw_create(floquet_op*) {
  set_error("brickwork model: kernels not built in this version");
  return FQ_EINVAL;
}
void bw_destroy(floquet_op*) {}
fq_status bw_apply_U(floquet_op*, fq_dtype, const void*, void*, hipStream_t) { return FQ_EINVAL; }
fq_status bw_filter(floquet_op*, int, double, const zd*, fq_dtype, const void*, void*, hipStream_t) {
  return FQ_EINVAL;
}

}  // namespace fq
