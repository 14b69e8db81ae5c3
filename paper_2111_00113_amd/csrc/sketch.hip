// Sparse sign embedding kernels (arXiv:2111.00113 Section 2.3.2):
//   pattern export: rows and signs of a range of sketch columns
//   sketch apply:   g = S v, with block-private LDS accumulators, block partials
//                   and a fixed-order cross-block sum.
#include "common.hpp"
#include "internal.hpp"

namespace sg {

namespace {

constexpr int kPatBlock = 256;

__global__ __launch_bounds__(kPatBlock) void pattern_kernel(uint64_t seed, uint32_t cycle, int64_t i0,
                                                            int64_t count, int s, int zeta,
                                                            int32_t* __restrict__ rows,
                                                            int8_t* __restrict__ signs) {
    __shared__ uint16_t slots[kMaxZeta * kPatBlock];
    const int64_t q = static_cast<int64_t>(blockIdx.x) * kPatBlock + threadIdx.x;
    if (q >= count) return;
    uint16_t* slot = slots + threadIdx.x;
    sketch_column(seed, cycle, i0 + q, s, zeta, slot, kPatBlock);
    for (int t = 0; t < zeta; ++t) {
        const unsigned e = slot[t * kPatBlock];
        rows[q * zeta + t] = static_cast<int32_t>(e >> 1);
        signs[q * zeta + t] = (e & 1u) ? static_cast<int8_t>(-1) : static_cast<int8_t>(1);
    }
}

constexpr int kSkBlock = 256;
constexpr int kSkMaxGrid = 512;

__global__ __launch_bounds__(kSkBlock) void sketch_partial_kernel(int64_t n, const double* __restrict__ v,
                                                                  uint64_t seed, uint32_t cycle, int s,
                                                                  int zeta, double* __restrict__ part) {
    extern __shared__ double acc[];  // s doubles, then zeta * kSkBlock uint16
    uint16_t* slots = reinterpret_cast<uint16_t*>(acc + s);
    for (int e = threadIdx.x; e < s; e += kSkBlock) acc[e] = 0.0;
    __syncthreads();
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kSkBlock;
    uint16_t* slot = slots + threadIdx.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kSkBlock + threadIdx.x; i < n; i += stride) {
        sketch_column(seed, cycle, i, s, zeta, slot, kSkBlock);
        const double x = v[i];
        for (int t = 0; t < zeta; ++t) {
            const unsigned e = slot[t * kSkBlock];
            atomicAdd(&acc[e >> 1], (e & 1u) ? -x : x);
        }
    }
    __syncthreads();
    const int G = gridDim.x;
    for (int e = threadIdx.x; e < s; e += kSkBlock) part[static_cast<int64_t>(e) * G + blockIdx.x] = acc[e];
}

// one wavefront per sketch row: fixed-order sum over the G block partials
__global__ __launch_bounds__(256) void sketch_finish_kernel(const double* __restrict__ part, int G, int s,
                                                            double scale, double* __restrict__ g) {
    const int lane = threadIdx.x & (kWave - 1);
    const int e = blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
    if (e >= s) return;
    double t = 0.0;
    for (int q = lane; q < G; q += kWave) t += part[static_cast<int64_t>(e) * G + q];
    t = wave_sum(t);
    if (lane == 0) g[e] = t * scale;
}

}  // namespace

hipError_t launch_sketch_pattern(uint64_t seed, uint32_t cycle, int64_t i0, int64_t count, int s,
                                 int zeta, int32_t* rows, int8_t* signs, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    const int64_t g = (count + kPatBlock - 1) / kPatBlock;
    pattern_kernel<<<static_cast<int>(g), kPatBlock, 0, stream>>>(seed, cycle, i0, count, s, zeta, rows, signs);
    return hipGetLastError();
}

int sketch_grid(int64_t n) {
    const int64_t g = (n + kSkBlock - 1) / kSkBlock;
    return static_cast<int>(g < 1 ? 1 : (g > kSkMaxGrid ? kSkMaxGrid : g));
}

hipError_t launch_sketch_apply(int64_t n, const double* v, uint64_t seed, uint32_t cycle, int s,
                               int zeta, double* part, double* g, hipStream_t stream) {
    const int G = sketch_grid(n);
    const size_t lds = sizeof(double) * s + sizeof(uint16_t) * zeta * kSkBlock;
    sketch_partial_kernel<<<G, kSkBlock, lds, stream>>>(n, v, seed, cycle, s, zeta, part);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int fb = (s + 3) / 4;
    sketch_finish_kernel<<<fb, 256, 0, stream>>>(part, G, s, 1.0 / sqrt(static_cast<double>(zeta)), g);
    return hipGetLastError();
}

}  // namespace sg
