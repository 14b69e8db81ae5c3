// spmv_truncarnoldi instances with FP32 arithmetic and the basis stored in
// bfloat16 (mixed-precision solve; sums of partials stay FP64).
#include "arnoldi_kernel.hpp"

namespace sg {

const void* arnoldi_pick_bf16(int block, int R, int KW) {
    return arnoldi_detail::arnoldi_pick<false, float, bf16_t>(block, R, KW);
}

}  // namespace sg
