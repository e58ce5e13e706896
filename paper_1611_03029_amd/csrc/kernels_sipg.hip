// Symmetric interior penalty DG Laplacian (Sec. 2.2): element-centric face and cell kernel.
#include "device_common.h"

namespace mfl {

hipError_t launch_sipg_apply(const Context &c, const Level &L, int dtype, const void *src, void *dst,
                             hipStream_t s) {
  (void)c; (void)L; (void)dtype; (void)src; (void)dst; (void)s;
  return hipErrorNotSupported;
}

}  // namespace mfl
