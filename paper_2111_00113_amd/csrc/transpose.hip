// CSR transpose on the device, for the transposed solve A^T x = b:
// column histogram -> inclusive scan -> scatter -> per-row sort (so the output
// is deterministic: each row of A^T lists its columns in ascending order).
#include "common.hpp"
#include "internal.hpp"

namespace sg {

namespace {

constexpr int kScanBlock = 1024;
constexpr int kScanItems = 4;
constexpr int kTile = kScanBlock * kScanItems;

__global__ void zero_i32(int32_t* x, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = 0;
}

__global__ void count_cols(int64_t nnz, const int32_t* __restrict__ ci, int32_t* __restrict__ cnt) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < nnz; q += stride)
        atomicAdd(&cnt[ci[q] + 1], 1);
}

// inclusive scan of one tile per block; tile totals to aux
__device__ int32_t block_inclusive_scan(int32_t v, int32_t* lds_wave) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int32_t t = __shfl_up(v, off, kWave);
        if (lane >= off) v += t;
    }
    if (lane == kWave - 1) lds_wave[wid] = v;
    __syncthreads();
    if (wid == 0) {
        int32_t w = (lane < kScanBlock / kWave) ? lds_wave[lane] : 0;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int32_t t = __shfl_up(w, off, kWave);
            if (lane >= off) w += t;
        }
        if (lane < kScanBlock / kWave) lds_wave[lane] = w;
    }
    __syncthreads();
    if (wid > 0) v += lds_wave[wid - 1];
    return v;
}

__global__ __launch_bounds__(kScanBlock) void scan_tiles(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                         int64_t m, int32_t* __restrict__ aux) {
    __shared__ int32_t lds_wave[kScanBlock / kWave];
    __shared__ int32_t total;
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kTile + static_cast<int64_t>(threadIdx.x) * kScanItems;
    int32_t loc[kScanItems];
    int32_t run = 0;
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        const int64_t i = t0 + u;
        run += (i < m) ? in[i] : 0;
        loc[u] = run;
    }
    const int32_t incl = block_inclusive_scan(run, lds_wave);
    const int32_t excl = incl - run;
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        const int64_t i = t0 + u;
        if (i < m) out[i] = loc[u] + excl;
    }
    if (threadIdx.x == kScanBlock - 1) total = incl;
    __syncthreads();
    if (threadIdx.x == 0) aux[blockIdx.x] = total;
}

// single block: exclusive scan of the tile totals, in place
__global__ __launch_bounds__(kScanBlock) void scan_aux(int32_t* aux, int64_t tiles) {
    __shared__ int32_t lds_wave[kScanBlock / kWave];
    __shared__ int32_t carry_s;
    int32_t carry = 0;
    for (int64_t b = 0; b < tiles; b += kScanBlock) {
        const int64_t i = b + threadIdx.x;
        const int32_t v = (i < tiles) ? aux[i] : 0;
        const int32_t incl = block_inclusive_scan(v, lds_wave);
        if (i < tiles) aux[i] = carry + incl - v;
        if (threadIdx.x == kScanBlock - 1) carry_s = carry + incl;
        __syncthreads();
        carry = carry_s;
        __syncthreads();
    }
}

__global__ void add_tile_offsets(int32_t* out, int64_t m, const int32_t* __restrict__ aux) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m) out[i] += aux[i / kTile];
}

__global__ void scatter_rows(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                             const double* __restrict__ val, const int32_t* __restrict__ trp,
                             int32_t* __restrict__ fill, int32_t* __restrict__ tci, double* __restrict__ tval) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int q1 = rp[i + 1];
        for (int q = rp[i]; q < q1; ++q) {
            const int32_t c = ci[q];
            const int32_t dst = trp[c] + atomicAdd(&fill[c], 1);
            tci[dst] = static_cast<int32_t>(i);
            tval[dst] = val[q];
        }
    }
}

__global__ void sort_rows(int64_t n, const int32_t* __restrict__ trp, int32_t* __restrict__ tci,
                          double* __restrict__ tval) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int q0 = trp[i], q1 = trp[i + 1];
        for (int q = q0 + 1; q < q1; ++q) {  // insertion sort: rows of A^T are short
            const int32_t key = tci[q];
            const double kv = tval[q];
            int z = q - 1;
            while (z >= q0 && tci[z] > key) {
                tci[z + 1] = tci[z];
                tval[z + 1] = tval[z];
                --z;
            }
            tci[z + 1] = key;
            tval[z + 1] = kv;
        }
    }
}

int grid_for(int64_t n, int block, int cap) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<int>(g);
}

}  // namespace

int64_t transpose_scratch_ints(int64_t n) { return 2 * (n + 1) + (n + 1 + kTile - 1) / kTile + 1; }

hipError_t launch_csr_transpose(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci,
                                const double* val, int32_t* trp, int32_t* tci, double* tval,
                                int32_t* scratch, hipStream_t stream) {
    // scratch layout: [0, n+1) counts, then fill counters [n+1, 2n+2), then tile sums
    int32_t* cnt = scratch;
    int32_t* fill = scratch + (n + 1);
    int32_t* aux = scratch + 2 * (n + 1);
    const int64_t m = n + 1;
    zero_i32<<<grid_for(2 * m, 256, 4096), 256, 0, stream>>>(scratch, 2 * m);
    count_cols<<<grid_for(nnz, 256, 4096), 256, 0, stream>>>(nnz, ci, cnt);
    const int64_t tiles = (m + kTile - 1) / kTile;
    scan_tiles<<<static_cast<int>(tiles), kScanBlock, 0, stream>>>(cnt, trp, m, aux);
    scan_aux<<<1, kScanBlock, 0, stream>>>(aux, tiles);
    add_tile_offsets<<<grid_for(m, 256, 1 << 30), 256, 0, stream>>>(trp, m, aux);
    scatter_rows<<<grid_for(n, 256, 4096), 256, 0, stream>>>(n, rp, ci, val, trp, fill, tci, tval);
    sort_rows<<<grid_for(n, 256, 4096), 256, 0, stream>>>(n, trp, tci, tval);
    return hipGetLastError();
}

}  // namespace sg
