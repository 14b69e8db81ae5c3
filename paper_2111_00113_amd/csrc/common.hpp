// Device-side building blocks shared by the sGMRES kernels (gfx950 / CDNA4).
//
// Contents: Philox4x32-10 (Salmon et al., SC'11), the sparse-sign column
// generator of the sketch (arXiv:2111.00113 Section 2.3.2), deterministic
// wavefront / workgroup / grid reductions, and a grid barrier with a bounded
// wait for cooperative (all-resident) launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sgmres.h"
#include "internal.hpp"

namespace sg {

constexpr int kWave = 64;
constexpr double kUnitRoundoff = 0x1.0p-53;

// --------------------------------------------------------------------------
// Philox4x32-10: ten rounds of the 4x32 Philox bijection.  Each round takes the
// 32x32->64 products of words 0 and 2 with two odd multipliers, swaps halves
// and mixes in the key; the key is advanced by two Weyl constants per round.
// --------------------------------------------------------------------------
struct U32x4 {
    uint32_t v0, v1, v2, v3;
};

__device__ __forceinline__ U32x4 philox10(U32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t prod_a = static_cast<uint64_t>(0xD2511F53u) * c.v0;
        const uint64_t prod_b = static_cast<uint64_t>(0xCD9E8D57u) * c.v2;
        U32x4 nx;
        nx.v0 = static_cast<uint32_t>(prod_b >> 32) ^ c.v1 ^ k0;
        nx.v1 = static_cast<uint32_t>(prod_b);
        nx.v2 = static_cast<uint32_t>(prod_a >> 32) ^ c.v3 ^ k1;
        nx.v3 = static_cast<uint32_t>(prod_a);
        c = nx;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Sparse sign column i of the sketch (see sgmres_sketch_pattern in sgmres.h).
// Accepted entries are written to slot[t * stride], t < zeta, each packed as
// (row << 1) | negative.  `slot` may live in LDS or global memory; it also
// serves as the list of rows taken so far for the duplicate test.
__device__ __forceinline__ void sketch_column(uint64_t seed, uint32_t cycle, int64_t i, int s,
                                              int zeta, uint16_t* slot, int stride) {
    const uint32_t k0 = static_cast<uint32_t>(seed);
    const uint32_t k1 = static_cast<uint32_t>(seed >> 32);
    const uint32_t c0 = static_cast<uint32_t>(static_cast<uint64_t>(i));
    const uint32_t c1 = static_cast<uint32_t>(static_cast<uint64_t>(i) >> 32);
    int taken = 0;
    for (uint32_t blk = 0; taken < zeta; ++blk) {
        const U32x4 w = philox10(U32x4{c0, c1, cycle, blk}, k0, k1);
        const uint32_t words[4] = {w.v0, w.v1, w.v2, w.v3};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (taken < zeta) {
                const uint32_t u = words[q];
                const uint32_t row = __umulhi(u, static_cast<uint32_t>(s));
                bool dup = false;
                for (int a = 0; a < taken; ++a) dup |= (slot[a * stride] >> 1) == row;
                if (!dup) {
                    slot[taken * stride] = static_cast<uint16_t>((row << 1) | (u & 1u));
                    ++taken;
                }
            }
        }
    }
}

// --------------------------------------------------------------------------
// Deterministic reductions.  The butterfly leaves the same bits in every lane,
// and every block that reduces the same data in the same order gets the same
// bits, which keeps grid-wide decisions (breakdown, kappa) consistent.
// --------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Sum over the workgroup of nv per-thread values; result in lds_out[0..nv).
// lds_tmp needs (blockDim.x / 64) * nv doubles.  Ends with a __syncthreads().
template <int NV>
__device__ __forceinline__ void block_sum(const double (&vals)[NV], int nv, double* lds_tmp,
                                          double* lds_out) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (v < nv) {
            const double t = wave_sum(vals[v]);
            if (lane == 0) lds_tmp[v * nw + wid] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        double acc = 0.0;
        for (int q = 0; q < nw; ++q) acc += lds_tmp[threadIdx.x * nw + q];
        lds_out[threadIdx.x] = acc;
    }
    __syncthreads();
}

// Every block sums partial[v * G + g] over g (fixed order) for v < nv; result
// in lds_out[0..nv).  One wavefront per value, lanes stride over g.
__device__ __forceinline__ void grid_sum(const double* partial, int G, int nv, double* lds_out) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    for (int v = wid; v < nv; v += nw) {
        double acc = 0.0;
        for (int g = lane; g < G; g += kWave) acc += partial[static_cast<int64_t>(v) * G + g];
        acc = wave_sum(acc);
        if (lane == 0) lds_out[v] = acc;
    }
    __syncthreads();
}

// --------------------------------------------------------------------------
// Grid barrier for a cooperative launch (all blocks resident).  The counter is
// monotone within a launch: barrier number q waits for q * G arrivals.  The
// release by thread 0 after __syncthreads() publishes the block's global writes
// at agent scope; the acquire makes every other block's writes visible.  The
// wait is bounded: after `limit` ticks of the 100 MHz real-time counter the
// block raises abort[0] and every later barrier returns at once, so the kernel
// always drains; the host reports SGMRES_ETIMEOUT.
// --------------------------------------------------------------------------
struct GridBarrier {
    unsigned* count;
    int* abort;
    unsigned G;
    unsigned seq;
    uint64_t limit;

    __device__ __forceinline__ void sync() {
        ++seq;
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned target = seq * G;
            __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
            while (__hip_atomic_load(count, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
                if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
                    __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
    }
};

// Blocks of a launch are dealt round-robin to the 8 XCDs; give each XCD a
// contiguous range of logical blocks so that neighbouring rows share an L2.
__device__ __forceinline__ int xcd_logical_block(int phys, int G) {
    if ((G & 7) != 0) return phys;
    return (phys & 7) * (G >> 3) + (phys >> 3);
}

}  // namespace sg
