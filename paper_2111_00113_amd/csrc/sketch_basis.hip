// Sketch of a finished basis, S B, and S A B from it through the Arnoldi
// relation (arXiv:2111.00113 Section 2.3.2 sparse sign embedding; Section
// 1.2.2 truncated-Arnoldi recurrence), for the streaming basis kernel.
//
//   lists    the sparse sign pattern of the cycle, regrouped per 512-row chunk
//            by sketch row (ascending row inside each list, as in the basis
//            kernels), written once per cycle to HBM
//   vectors  per workgroup and group of 16 vectors: each chunk's tile of the
//            16 vectors (512 rows, staged in LDS row-major as doubles) is
//            summed list by list: thread e owns sketch row e and adds the rows
//            of list e (16 values each, eight 16-byte LDS reads) into its 16
//            accumulators; chunks in order, each list in order, so the block
//            partial of every (vector, sketch row) has a fixed order of
//            additions.  List entries carry the row's tile offset and the sign
//            bit, and list padding points at a zero row, so an entry costs one
//            decode for 16 values
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
constexpr int kMaxS = 1024;  // sketch rows: one thread each

// A chunk's tile of one group of kCG vectors is staged in LDS as doubles,
// row-major with kTileStride entries per row (rows start on 16-byte
// boundaries), plus one row of zeros (row kChunk) that list padding points at.
// Thread e owns sketch row e (s <= 1024) and keeps one accumulator per vector
// of the group.
constexpr int kCG = 16;                          // vectors per group
constexpr int kTileStride = kCG + 2;             // doubles per staged row (16-byte aligned rows)
constexpr int kTileRows = kChunk + 1;
constexpr int kRowUnits = kTileStride / 2;       // 16-byte units per staged row
constexpr uint32_t kSignBit = 0x8000u;

__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ double widen(float v) { return static_cast<double>(v); }
__device__ __forceinline__ double widen(bf16_t v) { return static_cast<double>(from_basis<float>(v)); }

// Per-chunk record in 32-bit words: lstart (s + 1 entries, list starts in
// uint16 entries, multiples of four), a spare word when s + 1 is odd, then the
// lists: 16-bit entries in groups of four (each group one aligned 8-byte
// word), entry = the row's offset in the tile in 16-byte units
// (row * kRowUnits) | kSignBit when the sign is -1; the padding of a list's
// last group points at the zero row.
__host__ __device__ inline int64_t lists_offset(int s) { return (static_cast<int64_t>(s) + 2) & ~int64_t(1); }
__host__ __device__ inline int64_t list_words(int s, int zeta) {
    const int64_t w = lists_offset(s) + (static_cast<int64_t>(zeta) * kChunk + 3 * s + 1) / 2;
    return (w + 63) / 64 * 64;
}
constexpr int kRecRegs = 12;  // record words per thread while the next chunk is fetched

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
    for (int q = threadIdx.x; q <= s; q += kLsBlock) rec[q] = static_cast<uint32_t>(lstart[q]);
    // one thread per list rewrites its entries (list order kept) and padding
    uint16_t* dst = reinterpret_cast<uint16_t*>(rec + lists_offset(s));
    for (int e = threadIdx.x; e < s; e += kLsBlock) {
        const int a = lstart[e], b = lstart[e + 1], len = lcount[e];
        for (int q = a; q < b; ++q) {
            uint32_t t = static_cast<uint32_t>(kChunk * kRowUnits);  // zero row
            if (q - a < len) {
                const uint32_t key = lists[q];
                t = (key >> 1) * kRowUnits | ((key & 1u) ? kSignBit : 0u);
            }
            dst[q] = static_cast<uint16_t>(t);
        }
    }
}

// TS: basis type.  Block blk takes a contiguous range of chunks; for each group
// of kCG vectors (outer) and chunk (inner) it stages the chunk's tile and list
// record, and thread e adds the tile rows of list e, each with its sign, into
// its kCG accumulators (one 16-byte LDS read per two vectors, one FMA per
// vector and entry, entries in list order).
template <typename TS, int NR>
__global__ __launch_bounds__(kVecBlock2) void vectors_kernel(int64_t n, const TS* __restrict__ B, int64_t ldb,
                                                             int nvec, int s, int zeta,
                                                             const uint32_t* __restrict__ recs,
                                                             double* __restrict__ part) {
    static_assert(NR == 1 || NR % kCG == 0, "a group's vectors share one basis column");
    extern __shared__ __align__(16) unsigned char lds[];
    double* tile = reinterpret_cast<double*>(lds);  // kTileRows x kTileStride
    uint32_t* rec = reinterpret_cast<uint32_t*>(tile + kTileRows * kTileStride);
    constexpr int kTileRegs = kChunk * kCG / kVecBlock2;
    const int tid = threadIdx.x;
    const int G = gridDim.x;
    const int blk = blockIdx.x;
    const int64_t nch = (n + kChunk - 1) / kChunk;
    const int64_t ch0 = (static_cast<int64_t>(blk) * nch) / G;
    const int64_t nchb = (static_cast<int64_t>(blk + 1) * nch) / G - ch0;  // chunks of this block
    const int lw = static_cast<int>(list_words(s, zeta));
    const int64_t E = static_cast<int64_t>(nvec) * s;
    const int nvg = (nvec + kCG - 1) / kCG;
    const int64_t nitems = static_cast<int64_t>(nvg) * nchb;  // (vector group, chunk), chunks fastest
    for (int q = tid; q < kTileStride; q += kVecBlock2) tile[kChunk * kTileStride + q] = 0.0;

    // the next item's tile and list record are fetched into registers while
    // the current one is summed
    TS treg[kTileRegs];
    uint32_t rreg[kRecRegs];
    auto fetch = [&](int64_t it) {
        const int v0 = static_cast<int>(it / nchb) * kCG;
        const int64_t ch = ch0 + it % nchb;
        const int64_t r0 = ch * kChunk;
#pragma unroll
        for (int u = 0; u < kTileRegs; ++u) {
            const int idx = tid + u * kVecBlock2;
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
            treg[u] = (v < nvec && i < n) ? B[static_cast<int64_t>(v / NR) * ldb + i * NR + (v % NR)] : TS{};
        }
        const uint32_t* src = recs + ch * lw;
#pragma unroll
        for (int u = 0; u < kRecRegs; ++u) {
            const int q = tid + u * kVecBlock2;
            rreg[u] = q < lw ? src[q] : 0u;
        }
    };
    auto stage = [&](int64_t it) {
        const int v0 = static_cast<int>(it / nchb) * kCG;
        const int64_t r0 = (ch0 + it % nchb) * kChunk;
#pragma unroll
        for (int u = 0; u < kTileRegs; ++u) {
            const int idx = tid + u * kVecBlock2;
            int cc, l;
            if constexpr (NR == 1) {
                cc = idx / kChunk;
                l = idx % kChunk;
            } else {
                cc = idx % kCG;
                l = idx / kCG;
            }
            tile[l * kTileStride + cc] = (v0 + cc < nvec && r0 + l < n) ? widen(treg[u]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kRecRegs; ++u) {
            const int q = tid + u * kVecBlock2;
            if (q < lw) rec[q] = rreg[u];
        }
    };
    const double2* tile2 = reinterpret_cast<const double2*>(tile);
    double acc[kCG];
#pragma unroll
    for (int c = 0; c < kCG; ++c) acc[c] = 0.0;
    auto add_row = [&](uint32_t key) {
        const double sg = (key & kSignBit) ? -1.0 : 1.0;
        const double2* row = tile2 + (key & (kSignBit - 1u));
#pragma unroll
        for (int h = 0; h < kCG / 2; ++h) {
            const double2 x = row[h];
            acc[2 * h] = __builtin_fma(sg, x.x, acc[2 * h]);
            acc[2 * h + 1] = __builtin_fma(sg, x.y, acc[2 * h + 1]);
        }
    };
    if (nitems > 0) fetch(0);
    for (int64_t it = 0; it < nitems; ++it) {
        __syncthreads();  // the previous item's tile and lists are consumed
        stage(it);
        __syncthreads();
        if (it + 1 < nitems) fetch(it + 1);
        if (tid < s) {
            const int* lstart = reinterpret_cast<const int*>(rec);
            const uint2* L4 = reinterpret_cast<const uint2*>(rec + lists_offset(s));
            const int g0 = lstart[tid] / 4, g1 = lstart[tid + 1] / 4;
            for (int g = g0; g < g1; ++g) {  // groups of four entries, in list order
                const uint2 w = L4[g];
                add_row(w.x & 0xffffu);
                add_row(w.x >> 16);
                add_row(w.y & 0xffffu);
                add_row(w.y >> 16);
            }
        }
        if (it % nchb == nchb - 1) {
            const int v0 = static_cast<int>(it / nchb) * kCG;
#pragma unroll
            for (int c = 0; c < kCG; ++c) {
                if (tid < s && v0 + c < nvec)
                    part[static_cast<int64_t>(blk) * E + static_cast<int64_t>(v0 + c) * s + tid] = acc[c];
                acc[c] = 0.0;
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
    for (int a = 0; a < kw; ++a) t = madd(Hj[a], SB[(static_cast<int64_t>(j - a) * nr + r) * s + e], t);
    const double nu = Hj[k];
    if (nu != 0.0) t = madd(nu, SB[(static_cast<int64_t>(j + 1) * nr + r) * s + e], t);
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
    const size_t lds = sizeof(double) * kTileRows * kTileStride + sizeof(uint32_t) * list_words(s, zeta);
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

bool basis_sketch_fits(int64_t n, int s, int zeta) {
    return n < (int64_t(1) << 26) && s >= 1 && s <= kMaxS &&
           list_words(s, zeta) <= static_cast<int64_t>(kRecRegs) * kVecBlock2 &&
           sizeof(double) * kTileRows * kTileStride + sizeof(uint32_t) * list_words(s, zeta) <= 160 * 1024;
}

hipError_t launch_basis_sketch(int64_t n, const void* B, int64_t ldb, int nr, int precision, int nvec, int s,
                               int zeta, const uint32_t* lists, double* part, double* SB, hipStream_t stream) {
    if (nr == 1) {
        if (precision == SGMRES_PREC_FP64)
            return launch_vectors<double, 1>(n, static_cast<const double*>(B), ldb, nvec, s, zeta, lists, part, SB,
                                             stream);
        if (precision == SGMRES_PREC_FP32)
            return launch_vectors<float, 1>(n, static_cast<const float*>(B), ldb, nvec, s, zeta, lists, part, SB,
                                            stream);
        if (precision == SGMRES_PREC_BF16_BASIS)
            return launch_vectors<bf16_t, 1>(n, static_cast<const bf16_t*>(B), ldb, nvec, s, zeta, lists, part, SB,
                                             stream);
    } else if (nr == 32) {
        if (precision == SGMRES_PREC_FP64)
            return launch_vectors<double, 32>(n, static_cast<const double*>(B), ldb, nvec, s, zeta, lists, part, SB,
                                              stream);
        if (precision == SGMRES_PREC_FP32)
            return launch_vectors<float, 32>(n, static_cast<const float*>(B), ldb, nvec, s, zeta, lists, part, SB,
                                             stream);
        if (precision == SGMRES_PREC_BF16_BASIS)
            return launch_vectors<bf16_t, 32>(n, static_cast<const bf16_t*>(B), ldb, nvec, s, zeta, lists, part, SB,
                                              stream);
    }
    return hipErrorInvalidValue;
}

// g = S r for nr interleaved FP64 residuals (one column), with the cycle's lists
hipError_t launch_residual_sketch(int64_t n, const double* r, int nr, int s, int zeta, const uint32_t* lists,
                                  double* part, double* g, hipStream_t stream) {
    if (nr == 1) return launch_vectors<double, 1>(n, r, n, 1, s, zeta, lists, part, g, stream);
    if (nr == 32) return launch_vectors<double, 32>(n, r, n * 32, 32, s, zeta, lists, part, g, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_relation(int nr, int d, int k, int s, const double* H, const double* SB, const int* dc_dev,
                           double* SAB, hipStream_t stream) {
    const int64_t total = static_cast<int64_t>(nr) * d * s;
    relation_kernel<<<static_cast<unsigned>((total + 255) / 256), 256, 0, stream>>>(nr, d, k, s, H, SB, dc_dev, SAB);
    return hipGetLastError();
}

}  // namespace sg
