// Vector kernels for a block of NR right-hand sides sharing one matrix, kept
// interleaved (entry i of right-hand side r at i * NR + r), as the streaming
// basis kernel reads them (arXiv:2111.00113 Algorithm 1 residual and solution
// steps, per right-hand side):
//   pack / unpack   the callers' separate vectors <-> the interleaved block
//   residual        R = F - A X (X may be absent) and per right-hand side
//                   partial sums of |r|^2, one slot per workgroup
//   norm finish     |r| per right-hand side: the workgroup slots in order
//   combine         X += B[:, :d_eff(r)] y(r), columns in order
#include "common.hpp"
#include "internal.hpp"

namespace sg {

namespace {

constexpr int kMBlock = 256;

__device__ __forceinline__ double to_d(double v) { return v; }
__device__ __forceinline__ double to_d(float v) { return static_cast<double>(v); }
__device__ __forceinline__ double to_d(bf16_t v) { return static_cast<double>(from_basis<float>(v)); }

__global__ __launch_bounds__(kMBlock) void pack_kernel(int64_t n, int nr, const double* const* __restrict__ src,
                                                       double* __restrict__ dst) {
    const int64_t total = n * nr;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * kMBlock + threadIdx.x; q < total;
         q += static_cast<int64_t>(gridDim.x) * kMBlock) {
        const int r = static_cast<int>(q % nr);
        const double* s = src[r];
        dst[q] = s ? s[q / nr] : 0.0;
    }
}

__global__ __launch_bounds__(kMBlock) void unpack_kernel(int64_t n, int nr, const double* __restrict__ src,
                                                         double* const* __restrict__ dst) {
    const int64_t total = n * nr;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * kMBlock + threadIdx.x; q < total;
         q += static_cast<int64_t>(gridDim.x) * kMBlock) {
        double* d = dst[q % nr];
        if (d) d[q / nr] = src[q];
    }
}

// R = F - A X (or R = F when X is null); part[blk * NR + r] = this workgroup's
// sum of r_i^2 over its pairs (lanes of one right-hand side by an xor
// butterfly, then the wavefronts in order).  Pairs of a thread: q = tid + k *
// stride, each row summed in CSR order.
template <int NR>
__global__ __launch_bounds__(kMBlock) void residual_multi_kernel(int64_t n, const int32_t* __restrict__ rp,
                                                                 const int32_t* __restrict__ ci,
                                                                 const double* __restrict__ val,
                                                                 const double* __restrict__ F,
                                                                 const double* __restrict__ X,
                                                                 double* __restrict__ R, double* __restrict__ part) {
    __shared__ double red[(kMBlock / kWave) * NR];
    const int64_t total = n * NR;
    const int rhs = threadIdx.x % NR;
    double acc = 0.0;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * kMBlock + threadIdx.x; q < total;
         q += static_cast<int64_t>(gridDim.x) * kMBlock) {
        const int64_t i = q / NR;
        double t = F[q];
        if (X) {
            double ax = 0.0;
            for (int e = rp[i]; e < rp[i + 1]; ++e) ax = madd(val[e], X[static_cast<int64_t>(ci[e]) * NR + rhs], ax);
            t -= ax;
        }
        R[q] = t;
        acc = madd(t, t, acc);
    }
    for (int off = NR; off < kWave; off <<= 1) acc += __shfl_xor(acc, off, kWave);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane < NR) red[lane * (kMBlock / kWave) + wid] = acc;
    __syncthreads();
    if (threadIdx.x < NR) {
        double t = 0.0;
        for (int w = 0; w < kMBlock / kWave; ++w) t += red[threadIdx.x * (kMBlock / kWave) + w];
        part[static_cast<int64_t>(blockIdx.x) * NR + threadIdx.x] = t;
    }
}

// out[r] = sqrt(sum_g part[g * nr + r]) in g order; rel[r] = out[r] / nf[r]
// (0 when nf[r] = 0) when nf is given
__global__ void norm_multi_kernel(const double* __restrict__ part, int G, int nr, const double* __restrict__ nf,
                                  double* __restrict__ out, double* __restrict__ rel) {
    const int r = threadIdx.x;
    if (r >= nr) return;
    double t = 0.0;
    for (int g = 0; g < G; ++g) t += part[static_cast<int64_t>(g) * nr + r];
    const double v = sqrt(t);
    out[r] = v;
    if (nf) rel[r] = nf[r] > 0.0 ? v / nf[r] : 0.0;
}

// X[q] += sum_{j < d_eff(r)} B[j ldb + q] y[r d + j], j ascending
template <typename TS, int NR>
__global__ __launch_bounds__(kMBlock) void combine_multi_kernel(int64_t n, int d, const int* __restrict__ d_eff,
                                                                int dstride,
                                                                const TS* __restrict__ B, int64_t ldb,
                                                                const double* __restrict__ y,
                                                                double* __restrict__ X) {
    const int64_t total = n * NR;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * kMBlock + threadIdx.x; q < total;
         q += static_cast<int64_t>(gridDim.x) * kMBlock) {
        const int r = static_cast<int>(q % NR);
        const int de = d_eff[r * dstride];
        const double* yr = y + static_cast<int64_t>(r) * d;
        double t = X[q];
        for (int j = 0; j < de; ++j)
            t = madd(to_d(B[static_cast<int64_t>(j) * ldb + q]), yr[j], t);
        X[q] = t;
    }
}

int grid_pairs(int64_t total) {
    int64_t g = (total + kMBlock - 1) / kMBlock;
    if (g > kMultiMaxGrid) g = kMultiMaxGrid;
    return static_cast<int>(g < 1 ? 1 : g);
}

}  // namespace

int multi_grid(int64_t n, int nr) { return grid_pairs(n * nr); }

hipError_t launch_pack(int64_t n, int nr, const double* const* src, double* dst, hipStream_t stream) {
    pack_kernel<<<grid_pairs(n * nr), kMBlock, 0, stream>>>(n, nr, src, dst);
    return hipGetLastError();
}

hipError_t launch_unpack(int64_t n, int nr, const double* src, double* const* dst, hipStream_t stream) {
    unpack_kernel<<<grid_pairs(n * nr), kMBlock, 0, stream>>>(n, nr, src, dst);
    return hipGetLastError();
}

hipError_t launch_residual_multi(int64_t n, int nr, const int32_t* rp, const int32_t* ci, const double* val,
                                 const double* F, const double* X, double* R, double* part, const double* nf,
                                 double* out, double* rel, hipStream_t stream) {
    const int G = grid_pairs(n * nr);
    if (nr != 32) return hipErrorInvalidValue;
    residual_multi_kernel<32><<<G, kMBlock, 0, stream>>>(n, rp, ci, val, F, X, R, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    norm_multi_kernel<<<1, 64, 0, stream>>>(part, G, nr, nf, out, rel);
    return hipGetLastError();
}

hipError_t launch_combine_multi(int64_t n, int nr, int d, const int* d_eff, int dstride, const void* B, int64_t ldb,
                                const double* y, double* X, int precision, hipStream_t stream) {
    const int G = grid_pairs(n * nr);
    if (nr != 32) return hipErrorInvalidValue;
    if (precision == SGMRES_PREC_FP64)
        combine_multi_kernel<double, 32><<<G, kMBlock, 0, stream>>>(n, d, d_eff, dstride, static_cast<const double*>(B), ldb, y, X);
    else if (precision == SGMRES_PREC_FP32)
        combine_multi_kernel<float, 32><<<G, kMBlock, 0, stream>>>(n, d, d_eff, dstride, static_cast<const float*>(B), ldb, y, X);
    else if (precision == SGMRES_PREC_BF16_BASIS)
        combine_multi_kernel<bf16_t, 32><<<G, kMBlock, 0, stream>>>(n, d, d_eff, dstride, static_cast<const bf16_t*>(B), ldb, y, X);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace sg
