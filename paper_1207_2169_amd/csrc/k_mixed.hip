// int8 digit-plane MFMA kernels of the mixed-precision path (placeholder).
#include "common.cuh"

namespace clak {

hipError_t launch_rotate_snps_mixed(const Plan& p, int64_t m_blk) { return hipErrorNotSupported; }

hipError_t launch_grid_mixed(const Plan& p, int64_t m_blk, void* d_b, void* d_se, int out_dtype, int64_t ldo,
                             uint8_t* d_flags) {
  return hipErrorNotSupported;
}

}  // namespace clak
