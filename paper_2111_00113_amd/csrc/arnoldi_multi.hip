// Several independent systems per truncated-Arnoldi basis launch (the batched
// solve): instances, launch shape and launch of arnoldi_multi_kernel
// (arnoldi_kernel.hpp).  Each system's cycle is the one of sgmres_solve
// (Algorithm 1 basis loop), run by its own group of workgroups.
#include "arnoldi_kernel.hpp"

namespace sg {

namespace {

// Window registers: two columns for k <= 2, else four.  The SpMV's column
// look-ahead is on wherever it costs no register spill: every instance but
// FP64 arithmetic with a four-column window (which spilled 24 VGPRs with it
// at four rows per thread and measured slower).
template <typename TC, typename TS, int KW>
const void* pick_rows_multi(int R) {
    constexpr bool look = KW <= 2 || sizeof(TC) == 4;
    switch (R) {
        case 2: return reinterpret_cast<const void*>(arnoldi_detail::arnoldi_multi_kernel<2, KW, 1024, TC, TS, look>);
        case 4: return reinterpret_cast<const void*>(arnoldi_detail::arnoldi_multi_kernel<4, KW, 1024, TC, TS, look>);
        default: return nullptr;
    }
}

template <typename TC, typename TS>
const void* pick_window_multi(int R, int k) {
    return k <= 2 ? pick_rows_multi<TC, TS, 2>(R) : pick_rows_multi<TC, TS, 4>(R);
}

const void* pick_multi(int R, int k, int precision) {
    if (precision == SGMRES_PREC_FP64) return pick_window_multi<double, double>(R, k);
    if (precision == SGMRES_PREC_FP32) return pick_window_multi<float, float>(R, k);
    if (precision == SGMRES_PREC_BF16_BASIS) return pick_window_multi<float, bf16_t>(R, k);
    return nullptr;
}

}  // namespace

hipError_t arnoldi_multi_configure(int R, int k, int s, int zeta, int precision, MultiLaunch* out) {
    if (k < 1 || k > kMultiMaxK) return hipErrorInvalidValue;
    const void* fn = pick_multi(R, k, precision);
    if (!fn) return hipErrorInvalidValue;
    int device = 0;
    hipError_t err = hipGetDevice(&device);
    if (err != hipSuccess) return err;
    int cus = 0, lds_max = 0;
    err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (err != hipSuccess) return err;
    err = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (err != hipSuccess) return err;
    const size_t lds = arnoldi_lds_bytes(kMultiBlock, R, s, k, zeta);
    if (lds > static_cast<size_t>(lds_max)) return hipErrorInvalidValue;
    err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (err != hipSuccess) return err;
    int per_cu = 0;
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kMultiBlock, lds);
    if (err != hipSuccess) return err;
    if (per_cu < 1) return hipErrorInvalidValue;
    out->fn = fn;
    out->R = R;
    out->rows = static_cast<int64_t>(R) * kMultiBlock;
    out->capacity = per_cu * cus;
    out->lds = lds;
    return hipSuccess;
}

hipError_t arnoldi_multi_launch(const MultiLaunch& L, int grid, const ArnoldiParams* ps, const int* grp,
                                hipStream_t stream) {
    if (grid < 1 || grid > L.capacity) return hipErrorInvalidValue;
    void* args[] = {&ps, &grp};
    return hipLaunchCooperativeKernel(L.fn, dim3(grid), dim3(kMultiBlock), args, static_cast<unsigned>(L.lds),
                                      stream);
}

}  // namespace sg
