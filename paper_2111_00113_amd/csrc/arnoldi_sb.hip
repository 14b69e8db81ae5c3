// spmv_truncarnoldi instances that also form S b_j (the SB output of
// sgmres_arnoldi_cycle); compiled apart from the solve-path instances.
#include "arnoldi_kernel.hpp"

namespace sg {

const void* arnoldi_pick_sb(int block, int R, int KW) {
    return arnoldi_detail::arnoldi_pick<true, double, double>(block, R, KW);
}

}  // namespace sg
