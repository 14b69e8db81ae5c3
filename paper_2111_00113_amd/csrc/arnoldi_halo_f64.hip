// spmv_truncarnoldi solve instances with two grid barriers per step (the
// halo mode of arnoldi_kernel), FP64.
#include "arnoldi_kernel.hpp"

namespace sg {

const void* arnoldi_pick_halo_f64(int block, int R, int KW) {
    return arnoldi_detail::arnoldi_pick<false, double, double, true>(block, R, KW);
}

}  // namespace sg
