// Sketch of a finished basis, S B, and S A B from it through the Arnoldi
// relation (arXiv:2111.00113 Section 2.3.2 sparse sign embedding; Section
// 1.2.2 truncated-Arnoldi recurrence), for the streaming basis kernel.
//
//   lists    the sparse sign pattern of the cycle, regrouped per 512-row chunk
//            by sketch row (ascending row inside each list, as in the basis
//            kernels), written once per cycle to HBM
//   vectors  per workgroup and group of 16 vectors: each chunk's tile of the
//            16 vectors (512 rows, staged in LDS row-major, so a row's 16
//            entries are one conflict-free read) is summed list by list into
//            per-lane accumulators: lane group g (16 lanes, one per vector)
//            owns sketch rows g, g + 64, ...; chunks in order, each list in
//            order, so the block partial of every (vector, sketch row) has a
//            fixed order of additions
//   finish   SB = (sum of the block partials in block order) / sqrt(zeta)
//   relation S A b_j = sum_a H[a, j] S b_{j-a} + nu_j S b_{j+1}
//
// Vector v of a basis with NR interleaved right-hand sides is right-hand side
// v % NR of column v / NR: entry i at B[(v / NR) * ldb + i * NR + v % NR].
#include "common.hpp"
#include "internal.hpp"

namespace sg {

namespace {

constexpr int kLsBlock = 256;
constexpr int kLsRows = 2;
constexpr int kChunk = kLsBlock * kLsRows;  // rows per chunk (512)
constexpr int kVecBlock2 = 1024;
constexpr int kCG = 16;                     // vectors per group (lanes per lane group)
constexpr int kLaneGroups = kVecBlock2 / kCG;
constexpr int kMaxU = 16;                   // sketch rows per lane group: s <= 1024
constexpr int kTileStride = kCG + 1;        // doubles per staged row (padding against bank conflicts)

__device__ __forceinline__ double as_double(double v) { return v; }
__device__ __forceinline__ double as_double(float v) { return static_cast<double>(v); }
__device__ __forceinline__ double as_double(bf16_t v) { return static_cast<double>(from_basis<float>(v)); }

// per-chunk record in 32-bit words: lstart (s + 1), lcount (s), then the lists
// (uint16, zeta * 512 + 3 s entries, groups of four)
__host__ __device__ inline int64_t list_words(int s, int zeta) {
    const int64_t w = (2 * static_cast<int64_t>(s) + 1) + (static_cast<int64_t>(zeta) * kChunk + 3 * s + 1) / 2;
    return (w + 63) / 64 * 64;
}

__global__ __launch_bounds__(kLsBlock) void lists_kernel(int64_t n, uint64_t seed, uint32_t cycle, int s, int zeta,
                                                        uint32_t* __restrict__ out) {
    extern __shared__ __align__(16) unsigned char lds[];
    int* lstart = reinterpret_cast<int*>(lds);
    int* lcount = lstart + (s + 1);
    uint16_t* raw = reinterpret_cast<uint16_t*>(lds + ((sizeof(int) * (2 * s + 1) + 15) & ~static_cast<size_t>(15)));
    const size_t raw_bytes = ((sizeof(uint16_t) * zeta * kChunk > static_cast<size_t>(kLsBlock) * kChunk / 256
                                   ? sizeof(uint16_t) * zeta * kChunk
                                   : static_cast<size_t>(kLsBlock) * kChunk / 256) + 15) & ~static_cast<size_t>(15);
    uint16_t* lists = reinterpret_cast<uint16_t*>(reinterpret_cast<unsigned char*>(raw) + raw_bytes);
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * kChunk;
    sketch_lists_build<kLsRows, kLsBlock, true>(seed, cycle, c0 + threadIdx.x, n, s, zeta, raw, lstart, lcount,
                                                lists);
    uint32_t* rec = out + static_cast<int64_t>(blockIdx.x) * list_words(s, zeta);
    for (int q = threadIdx.x; q < 2 * s + 1; q += kLsBlock) rec[q] = static_cast<uint32_t>(lstart[q]);
    const int len = lstart[s];  // padded to groups of four
    const uint32_t* lw = reinterpret_cast<const uint32_t*>(lists);
    for (int q = threadIdx.x; q < (len + 1) / 2; q += kLsBlock) rec[2 * s + 1 + q] = lw[q];
}

template <typename TS, int NR>
__global__ __launch_bounds__(kVecBlock2) void vectors_kernel(int64_t n, const TS* __restrict__ B, int64_t ldb,
                                                             int nvec, int s, int zeta,
                                                             const uint32_t* __restrict__ recs,
                                                             double* __restrict__ part) {
    extern __shared__ __align__(16) unsigned char lds[];
    double* tile = reinterpret_cast<double*>(lds);  // kChunk rows x kTileStride
    uint32_t* rec = reinterpret_cast<uint32_t*>(tile + kChunk * kTileStride);
    const int tid = threadIdx.x;
    const int lg = tid / kCG;
    const int c = tid % kCG;
    const int G = gridDim.x;
    const int blk = blockIdx.x;
    const int64_t nch = (n + kChunk - 1) / kChunk;
    const int64_t ch0 = (static_cast<int64_t>(blk) * nch) / G;
    const int64_t ch1 = (static_cast<int64_t>(blk + 1) * nch) / G;
    const int64_t lw = list_words(s, zeta);
    const int U = (s + kLaneGroups - 1) / kLaneGroups;
    const int64_t E = static_cast<int64_t>(nvec) * s;
    for (int v0 = 0; v0 < nvec; v0 += kCG) {
        double acc[kMaxU];
#pragma unroll
        for (int u = 0; u < kMaxU; ++u) acc[u] = 0.0;
        for (int64_t ch = ch0; ch < ch1; ++ch) {
            __syncthreads();  // the previous chunk's tile and lists are consumed
            const uint32_t* src = recs + ch * lw;
            const int used = 2 * s + 1 + (static_cast<int>(src[s]) + 1) / 2;  // lstart[s]: padded length
            for (int q = tid; q < used; q += kVecBlock2) rec[q] = src[q];
            const int64_t r0 = ch * kChunk;
            for (int idx = tid; idx < kChunk * kCG; idx += kVecBlock2) {
                int cc, l;
                if constexpr (NR == 1) {
                    cc = idx / kChunk;
                    l = idx % kChunk;
                } else {
                    cc = idx % kCG;
                    l = idx / kCG;
                }
                const int v = v0 + cc;
                const int64_t i = r0 + l;
                double x = 0.0;
                if (v < nvec && i < n)
                    x = as_double(B[static_cast<int64_t>(v / NR) * ldb + i * NR + (v % NR)]);
                tile[l * kTileStride + cc] = x;
            }
            __syncthreads();
            const int* lstart = reinterpret_cast<const int*>(rec);
            const int* lcount = lstart + (s + 1);
            const uint16_t* lists = reinterpret_cast<const uint16_t*>(rec + 2 * s + 1);
#pragma unroll
            for (int u = 0; u < kMaxU; ++u) {
                const int e = lg + kLaneGroups * u;
                if (u < U && e < s) {
                    const int len = lcount[e];
                    const uint16_t* L = lists + lstart[e];
                    double a = acc[u];
                    for (int q = 0; q < len; ++q) {
                        const unsigned key = L[q];
                        const double x = tile[(key >> 1) * kTileStride + c];
                        a += (key & 1u) ? -x : x;
                    }
                    acc[u] = a;
                }
            }
        }
        const int v = v0 + c;
        if (v < nvec) {
#pragma unroll
            for (int u = 0; u < kMaxU; ++u) {
                const int e = lg + kLaneGroups * u;
                if (u < U && e < s) part[static_cast<int64_t>(blk) * E + static_cast<int64_t>(v) * s + e] = acc[u];
            }
        }
    }
}

// SB[q] = scale * sum_g part[g * E + q], g in order
__global__ __launch_bounds__(256) void vectors_finish_kernel(const double* __restrict__ part, int G, int64_t E,
                                                             double scale, double* __restrict__ SB) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (q >= E) return;
    double t = 0.0;
    for (int g = 0; g < G; ++g) t += part[static_cast<int64_t>(g) * E + q];
    SB[q] = t * scale;
}

// S A b_j of right-hand side r from the sketched basis (vectors v = col * NR + r):
// SAB[(r d + j) s + e] = sum_{a < kw} H[a, j] SB[v(j - a)] + nu_j SB[v(j + 1)],
// kw = min(j + 1, k), for j < dc (the column of a breakdown has nu_j = 0 and
// no b_{j+1}); columns j >= dc are left alone
__global__ __launch_bounds__(256) void relation_kernel(int nr, int d, int k, int s, const double* __restrict__ H,
                                                       const double* __restrict__ SB, const int* __restrict__ dc_dev,
                                                       double* __restrict__ SAB) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t total = static_cast<int64_t>(nr) * d * s;
    if (q >= total) return;
    const int e = static_cast<int>(q % s);
    const int j = static_cast<int>((q / s) % d);
    const int r = static_cast<int>(q / (static_cast<int64_t>(s) * d));
    const int dc = dc_dev[nr > 1 ? r : 0];
    if (j >= dc) return;
    const int kw = j + 1 < k ? j + 1 : k;
    const double* Hj = H + (static_cast<int64_t>(r) * d + j) * (k + 1);
    double t = 0.0;
    for (int a = 0; a < kw; ++a) t += Hj[a] * SB[(static_cast<int64_t>(j - a) * nr + r) * s + e];
    const double nu = Hj[k];
    if (nu != 0.0) t += nu * SB[(static_cast<int64_t>(j + 1) * nr + r) * s + e];
    SAB[q] = t;
}

}  // namespace

int64_t basis_lists_words(int64_t n, int s, int zeta) { return ((n + kChunk - 1) / kChunk) * list_words(s, zeta); }

int basis_sketch_grid(int64_t n) {
    const int64_t nch = (n + kChunk - 1) / kChunk;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t g = nch < cus ? nch : cus;
    return static_cast<int>(g < 1 ? 1 : g);
}

hipError_t launch_basis_lists(int64_t n, uint64_t seed, uint32_t cycle, int s, int zeta, uint32_t* lists,
                              hipStream_t stream) {
    const int64_t nch = (n + kChunk - 1) / kChunk;
    const size_t raw_bytes = sizeof(uint16_t) * zeta * kChunk > static_cast<size_t>(kLsBlock) * kChunk / 256
                                 ? sizeof(uint16_t) * zeta * kChunk
                                 : static_cast<size_t>(kLsBlock) * kChunk / 256;
    const size_t lds = ((sizeof(int) * (2 * s + 1) + 15) & ~static_cast<size_t>(15)) + ((raw_bytes + 15) & ~static_cast<size_t>(15)) +
                       sizeof(uint16_t) * sketch_lists_len(zeta * kChunk, s, true);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(lists_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    lists_kernel<<<static_cast<unsigned>(nch), kLsBlock, lds, stream>>>(n, seed, cycle, s, zeta, lists);
    return hipGetLastError();
}

template <typename TS, int NR>
hipError_t launch_vectors(int64_t n, const TS* B, int64_t ldb, int nvec, int s, int zeta, const uint32_t* lists,
                          double* part, double* SB, hipStream_t stream) {
    const int G = basis_sketch_grid(n);
    const size_t lds = sizeof(double) * kChunk * kTileStride + sizeof(uint32_t) * list_words(s, zeta);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(vectors_kernel<TS, NR>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    vectors_kernel<TS, NR><<<G, kVecBlock2, lds, stream>>>(n, B, ldb, nvec, s, zeta, lists, part);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t E = static_cast<int64_t>(nvec) * s;
    vectors_finish_kernel<<<static_cast<unsigned>((E + 255) / 256), 256, 0, stream>>>(
        part, G, E, 1.0 / sqrt(static_cast<double>(zeta)), SB);
    return hipGetLastError();
}

bool basis_sketch_fits(int s, int zeta) {
    return s >= 1 && s <= kLaneGroups * kMaxU &&
           sizeof(double) * kChunk * kTileStride + sizeof(uint32_t) * list_words(s, zeta) <= 160 * 1024;
}

hipError_t launch_basis_sketch(int64_t n, const void* B, int64_t ldb, int nr, int precision, int nvec, int s,
                               int zeta, const uint32_t* lists, double* part, double* SB, hipStream_t stream) {
    if (nr == 1) {
        if (precision == SGMRES_PREC_FP64)
            return launch_vectors<double, 1>(n, static_cast<const double*>(B), ldb, nvec, s, zeta, lists, part, SB, stream);
        if (precision == SGMRES_PREC_FP32)
            return launch_vectors<float, 1>(n, static_cast<const float*>(B), ldb, nvec, s, zeta, lists, part, SB, stream);
        if (precision == SGMRES_PREC_BF16_BASIS)
            return launch_vectors<bf16_t, 1>(n, static_cast<const bf16_t*>(B), ldb, nvec, s, zeta, lists, part, SB,
                                             stream);
    } else if (nr == 32) {
        if (precision == SGMRES_PREC_FP64)
            return launch_vectors<double, 32>(n, static_cast<const double*>(B), ldb, nvec, s, zeta, lists, part, SB,
                                              stream);
        if (precision == SGMRES_PREC_FP32)
            return launch_vectors<float, 32>(n, static_cast<const float*>(B), ldb, nvec, s, zeta, lists, part, SB, stream);
        if (precision == SGMRES_PREC_BF16_BASIS)
            return launch_vectors<bf16_t, 32>(n, static_cast<const bf16_t*>(B), ldb, nvec, s, zeta, lists, part, SB,
                                              stream);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_relation(int nr, int d, int k, int s, const double* H, const double* SB, const int* dc_dev,
                           double* SAB, hipStream_t stream) {
    const int64_t total = static_cast<int64_t>(nr) * d * s;
    relation_kernel<<<static_cast<unsigned>((total + 255) / 256), 256, 0, stream>>>(nr, d, k, s, H, SB, dc_dev, SAB);
    return hipGetLastError();
}

}  // namespace sg
