// spmv_truncarnoldi solve instances with two grid barriers per step (the
// halo mode of arnoldi_kernel), FP32 arithmetic and basis.
#include "arnoldi_kernel.hpp"

namespace sg {

const void* arnoldi_pick_halo_f32(int block, int R, int KW) {
    return arnoldi_detail::arnoldi_pick<false, float, float, true>(block, R, KW);
}

}  // namespace sg
