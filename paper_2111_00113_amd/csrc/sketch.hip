// Sparse sign embedding kernels (arXiv:2111.00113 Section 2.3.2):
//   pattern export: rows and signs of a range of sketch columns
//   sketch apply:   g = S v from block-local sketch lists summed in a fixed
//                   order, block partials and a fixed-order cross-block sum.
#include <algorithm>
#include <mutex>

#include "../../include/sgmres.h"
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

// g = S v in a fixed order.  Rows are taken in chunks of kSkChunk; block b
// takes chunks b, b + G, ...  For each chunk the block regroups the chunk's
// sparse sign columns by sketch row (ascending row inside each list, the same
// lists as the basis kernels) and sums every list in a fixed order into its
// LDS accumulator, which only one lane group touches per chunk.  The block's
// totals go to part[e * G + b]; sketch_finish_kernel adds them in block order.
// No atomics touch a floating-point value, so the bits do not vary from run
// to run.
constexpr int kSkBlock = 256;
constexpr int kSkRows = 2;                      // rows per thread and chunk
constexpr int kSkChunk = kSkBlock * kSkRows;    // rows per chunk
constexpr int kSkMaxGrid = 512;

constexpr size_t align8(size_t b) { return (b + 7) & ~static_cast<size_t>(7); }

struct SketchLds {
    size_t acc, vals, lstart, lcount, raw, lists, total;
};

SketchLds sketch_lds_layout(int s, int zeta) {
    SketchLds L{};
    const size_t raw_bytes = std::max(sizeof(uint16_t) * zeta * kSkChunk,
                                      static_cast<size_t>(kSkBlock) * kSkChunk / 256);
    L.acc = 0;
    L.vals = L.acc + align8(sizeof(double) * s);
    L.lstart = L.vals + sizeof(double) * kSkChunk;
    L.lcount = L.lstart + sizeof(int) * (s + 1);
    L.raw = align8(L.lcount + sizeof(int) * s);
    L.lists = L.raw + align8(raw_bytes);
    L.total = L.lists + align8(sizeof(uint16_t) * sketch_lists_len(zeta * kSkChunk, s, true));
    return L;
}

__global__ __launch_bounds__(kSkBlock) void sketch_partial_kernel(int64_t n, const double* __restrict__ v,
                                                                  uint64_t seed, uint32_t cycle, int s,
                                                                  int zeta, SketchLds lay,
                                                                  double* __restrict__ part) {
    extern __shared__ __align__(16) unsigned char lds[];
    double* acc = reinterpret_cast<double*>(lds + lay.acc);
    double* vals = reinterpret_cast<double*>(lds + lay.vals);
    int* lstart = reinterpret_cast<int*>(lds + lay.lstart);
    int* lcount = reinterpret_cast<int*>(lds + lay.lcount);
    uint16_t* raw = reinterpret_cast<uint16_t*>(lds + lay.raw);
    uint16_t* lists = reinterpret_cast<uint16_t*>(lds + lay.lists);
    const int tid = threadIdx.x;
    const int first = (tid & (kWave - 1)) & ~(kSketchParts - 1);
    for (int e = tid; e < s; e += kSkBlock) acc[e] = 0.0;
    const int G = gridDim.x;
    const int64_t nch = (n + kSkChunk - 1) / kSkChunk;
    for (int64_t c = blockIdx.x; c < nch; c += G) {
        const int64_t c0 = c * kSkChunk;
#pragma unroll
        for (int r = 0; r < kSkRows; ++r) {
            const int64_t i = c0 + r * kSkBlock + tid;
            vals[r * kSkBlock + tid] = i < n ? v[i] : 0.0;
        }
        // ends with a block synchronisation, which also publishes vals
        sketch_lists_build<kSkRows, kSkBlock, true>(seed, cycle, c0 + tid, n, s, zeta, raw, lstart, lcount, lists);
        // the kSketchParts pieces of list e are summed by consecutive lanes
        // (all active together: 4 s tasks, BLOCK a multiple of 4) and added in
        // piece order by the first of them
        for (int t = tid; t < kSketchParts * s; t += kSkBlock) {
            const int pc = t % kSketchParts;
            const int e = t / kSketchParts;
            const double piece = sketch_piece4(vals, lstart, lcount, lists, e, pc);
            double a = 0.0;
#pragma unroll
            for (int u = 0; u < kSketchParts; ++u) a += __shfl(piece, first + u, kWave);
            if (pc == 0) acc[e] += a;
        }
        __syncthreads();  // the next chunk rewrites vals and the lists
    }
    for (int e = tid; e < s; e += kSkBlock) part[static_cast<int64_t>(e) * G + blockIdx.x] = acc[e];
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
    const int64_t g = (n + kSkChunk - 1) / kSkChunk;
    return static_cast<int>(g < 1 ? 1 : (g > kSkMaxGrid ? kSkMaxGrid : g));
}

size_t sketch_apply_lds_bytes(int s, int zeta) { return sketch_lds_layout(s, zeta).total; }

hipError_t launch_sketch_apply(int64_t n, const double* v, uint64_t seed, uint32_t cycle, int s,
                               int zeta, double* part, double* g, hipStream_t stream) {
    const int G = sketch_grid(n);
    const SketchLds lay = sketch_lds_layout(s, zeta);
    if (lay.total > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(sketch_partial_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(lay.total));
        if (e != hipSuccess) return e;
    }
    sketch_partial_kernel<<<G, kSkBlock, lay.total, stream>>>(n, v, seed, cycle, s, zeta, lay, part);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int fb = (s + 3) / 4;
    sketch_finish_kernel<<<fb, 256, 0, stream>>>(part, G, s, 1.0 / sqrt(static_cast<double>(zeta)), g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Allocation-free g = S v for callers that cannot allocate device memory
// (code under stream capture, serving loops, harnesses that forbid it).  The
// block partials live in a fixed device array instead of the workspace.
// ---------------------------------------------------------------------------
namespace {

// s x G block partials, s <= 4096 and G <= 512 (16 MiB per device, held for
// the life of the process).  In host code this name is a stand-in for the
// device array, never its address: kernels receive the address that
// hipGetSymbolAddress returned for the current device.
constexpr size_t kScratchDoubles = static_cast<size_t>(4096) * 512;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's copy of scratch, looked up once per device (with
// that device current).
int scratch_for_device(double** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SGMRES_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return SGMRES_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SGMRES_EHIP;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return SGMRES_OK;
}

}  // namespace
}  // namespace sg

extern "C" int sgmres_sketch_apply_noalloc(int64_t n, const double* v, uint64_t seed, uint32_t cycle, int s,
                                           int zeta, double* g, void* stream) {
    using namespace sg;
    if (n < 0 || (n > 0 && !v) || !g || s < 1 || s > 4096 || zeta < 1 || zeta > s || zeta > kMaxZeta)
        return SGMRES_EINVAL;
    const int G = sketch_grid(n);
    if (static_cast<size_t>(s) * static_cast<size_t>(G) > kScratchDoubles) return SGMRES_EINVAL;
    double* part = nullptr;
    const int rc = scratch_for_device(&part);
    if (rc) return rc;
    // every partial is written before it is read: nothing to clear
    const hipError_t e = launch_sketch_apply(n, v, seed, cycle, s, zeta, part, g, static_cast<hipStream_t>(stream));
    if (e == hipSuccess) return SGMRES_OK;
    return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? SGMRES_ENOMEM : SGMRES_EHIP;
}
