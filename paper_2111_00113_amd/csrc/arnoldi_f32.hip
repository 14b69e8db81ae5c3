// spmv_truncarnoldi instances with FP32 arithmetic and an FP32 basis (the
// inner cycles of the mixed-precision solve; sums of partials stay FP64).
#include "arnoldi_kernel.hpp"

namespace sg {

const void* arnoldi_pick_f32(int block, int R, int KW) {
    return arnoldi_detail::arnoldi_pick<false, float, float>(block, R, KW);
}

}  // namespace sg
