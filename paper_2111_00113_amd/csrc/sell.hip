// Sliced ELL copy of A for the basis kernels (SELL with slices of 64 rows, one
// wavefront's rows).  Slice i holds rows 64 i .. 64 i + 63; every row of the
// slice is padded to the slice's longest row, and entry k of lane l sits at
// sp[i] + 64 k + l, so a wavefront reads the k-th nonzero of its 64 rows with
// one contiguous load.  Padding entries have value 0 and a column inside the
// row's own block (the row itself, or row n-1 past the end), so they add an
// exact zero.  Each row keeps its nonzeros in CSR order.
#include "common.hpp"
#include "internal.hpp"

namespace sg {

namespace {

__global__ void sell_width_kernel(int64_t n, const int32_t* __restrict__ rp, int64_t nsl, int* __restrict__ K) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t sl = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; sl < nsl; sl += stride) {
        int k = 0;
        for (int l = 0; l < kWave; ++l) {
            const int64_t row = sl * kWave + l;
            if (row < n) k = max(k, rp[row + 1] - rp[row]);
        }
        K[sl] = k;
    }
}

template <typename TC>
__global__ void sell_fill_kernel(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                 const double* __restrict__ val, int64_t nsl, const int64_t* __restrict__ sp,
                                 int32_t* __restrict__ scol, TC* __restrict__ sval) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t row = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; row < nsl * kWave; row += stride) {
        const int64_t sl = row / kWave;
        const int64_t base = sp[sl] + (row - sl * kWave);
        const int K = static_cast<int>((sp[sl + 1] - sp[sl]) / kWave);
        const int rb = row < n ? rp[row] : 0;
        const int rl = row < n ? rp[row + 1] - rb : 0;
        const int32_t pad = static_cast<int32_t>(row < n ? row : n - 1);
        for (int k = 0; k < K; ++k) {
            const int64_t e = base + static_cast<int64_t>(k) * kWave;
            scol[e] = k < rl ? ci[rb + k] : pad;
            sval[e] = k < rl ? static_cast<TC>(val[rb + k]) : TC(0);
        }
    }
}

int grid_for(int64_t items) {
    int64_t g = (items + 255) / 256;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return static_cast<int>(g);
}

}  // namespace

hipError_t launch_sell_width(int64_t n, const int32_t* rp, int* K, hipStream_t stream) {
    const int64_t nsl = (n + kWave - 1) / kWave;
    sell_width_kernel<<<grid_for(nsl), 256, 0, stream>>>(n, rp, nsl, K);
    return hipGetLastError();
}

hipError_t launch_sell_fill(int64_t n, const int32_t* rp, const int32_t* ci, const double* val, const int64_t* sp,
                            int32_t* scol, void* sval, int precision, hipStream_t stream) {
    const int64_t nsl = (n + kWave - 1) / kWave;
    const int g = grid_for(nsl * kWave);
    if (precision == SGMRES_PREC_FP64)
        sell_fill_kernel<double><<<g, 256, 0, stream>>>(n, rp, ci, val, nsl, sp, scol, static_cast<double*>(sval));
    else
        sell_fill_kernel<float><<<g, 256, 0, stream>>>(n, rp, ci, val, nsl, sp, scol, static_cast<float*>(sval));
    return hipGetLastError();
}

}  // namespace sg
