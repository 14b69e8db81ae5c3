// spmv_truncarnoldi solve instances with two grid barriers per step (the
// halo mode of arnoldi_kernel), FP32 arithmetic, bfloat16 basis.
#include "arnoldi_kernel.hpp"

namespace sg {

const void* arnoldi_pick_halo_bf16(int block, int R, int KW) {
    return arnoldi_detail::arnoldi_pick<false, float, bf16_t, true>(block, R, KW);
}

}  // namespace sg
