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

// block blk of nblk of one matrix's width pass: slice widths into K
__device__ __forceinline__ void sell_width_body(int blk, int nblk, int64_t n, const int32_t* __restrict__ rp,
                                                int64_t nsl, int* __restrict__ K) {
    const int64_t stride = static_cast<int64_t>(nblk) * blockDim.x;
    for (int64_t sl = static_cast<int64_t>(blk) * blockDim.x + threadIdx.x; sl < nsl; sl += stride) {
        int k = 0;
        for (int l = 0; l < kWave; ++l) {
            const int64_t row = sl * kWave + l;
            if (row < n) k = max(k, rp[row + 1] - rp[row]);
        }
        K[sl] = k;
    }
}

__global__ void sell_width_kernel(int64_t n, const int32_t* __restrict__ rp, int64_t nsl, int* __restrict__ K) {
    sell_width_body(blockIdx.x, gridDim.x, n, rp, nsl, K);
}

// block blk of nblk of one matrix's fill pass
template <typename TC>
__device__ __forceinline__ void sell_fill_body(int blk, int nblk, int64_t n, const int32_t* __restrict__ rp,
                                               const int32_t* __restrict__ ci, const double* __restrict__ val,
                                               int64_t nsl, const int64_t* __restrict__ sp, int32_t* __restrict__ scol,
                                               TC* __restrict__ sval) {
    const int64_t stride = static_cast<int64_t>(nblk) * blockDim.x;
    for (int64_t row = static_cast<int64_t>(blk) * blockDim.x + threadIdx.x; row < nsl * kWave; row += stride) {
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

template <typename TC>
__global__ void sell_fill_kernel(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                 const double* __restrict__ val, int64_t nsl, const int64_t* __restrict__ sp,
                                 int32_t* __restrict__ scol, TC* __restrict__ sval) {
    sell_fill_body<TC>(blockIdx.x, gridDim.x, n, rp, ci, val, nsl, sp, scol, sval);
}

// several matrices per launch: the job whose blocks hold block b (jobs in
// block order; first block blk0 of each pass)
__device__ __forceinline__ int sell_job_of(const SellJob* __restrict__ jobs, int njobs, int b, bool fill) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if ((fill ? jobs[mid].fblk0 : jobs[mid].wblk0) <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void sell_width_jobs_kernel(const SellJob* __restrict__ jobs, int njobs) {
    __shared__ int sj;
    if (threadIdx.x == 0) sj = sell_job_of(jobs, njobs, blockIdx.x, false);
    __syncthreads();
    const SellJob& J = jobs[sj];
    sell_width_body(blockIdx.x - J.wblk0, J.wnblk, J.n, J.rp, (J.n + kWave - 1) / kWave, J.K);
}

template <typename TC>
__global__ void sell_fill_jobs_kernel(const SellJob* __restrict__ jobs, int njobs) {
    __shared__ int sj;
    if (threadIdx.x == 0) sj = sell_job_of(jobs, njobs, blockIdx.x, true);
    __syncthreads();
    const SellJob& J = jobs[sj];
    sell_fill_body<TC>(blockIdx.x - J.fblk0, J.fnblk, J.n, J.rp, J.ci, J.val, (J.n + kWave - 1) / kWave, J.sp,
                       J.scol, static_cast<TC*>(J.sval));
}

int grid_for(int64_t items) {
    int64_t g = (items + 255) / 256;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return static_cast<int>(g);
}

}  // namespace

int sell_width_blocks(int64_t n) { return grid_for((n + kWave - 1) / kWave); }
int sell_fill_blocks(int64_t n) { return grid_for((n + kWave - 1) / kWave * kWave); }

hipError_t launch_sell_jobs(const SellJob* jobs, int njobs, int blocks, bool fill, int precision,
                            hipStream_t stream) {
    if (njobs <= 0 || blocks <= 0) return hipSuccess;
    if (!fill)
        sell_width_jobs_kernel<<<blocks, 256, 0, stream>>>(jobs, njobs);
    else if (precision == SGMRES_PREC_FP64)
        sell_fill_jobs_kernel<double><<<blocks, 256, 0, stream>>>(jobs, njobs);
    else
        sell_fill_jobs_kernel<float><<<blocks, 256, 0, stream>>>(jobs, njobs);
    return hipGetLastError();
}

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
