// Device-side building blocks shared by the sGMRES kernels (gfx950 / CDNA4).
//
// Contents: Philox4x32-10 (Salmon et al., SC'11), the sparse-sign column
// generator of the sketch (arXiv:2111.00113 Section 2.3.2), deterministic
// wavefront / workgroup / grid reductions, and a grid barrier with a bounded
// wait for cooperative (all-resident) launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/sgmres.h"
#include "internal.hpp"

namespace sg {

constexpr int kWave = 64;
constexpr double kUnitRoundoff = 0x1.0p-53;

// --------------------------------------------------------------------------
// Basis precisions.  TC is the type of the per-row arithmetic (SpMV, Gram-
// Schmidt updates, recurrences), TS the storage type of the basis in HBM.  A
// basis vector is rounded to TS once, when it is formed, and the rounded value
// is what every later use sees (SpMV gathers, the register window, the
// combine), so S A B is always formed for the B that is stored.
// --------------------------------------------------------------------------
struct bf16_t {
    uint16_t bits;
};

template <typename TC>
struct BasisPrec;
template <>
struct BasisPrec<double> {
    static constexpr double unit_roundoff = 0x1.0p-53;
};
template <>
struct BasisPrec<float> {
    static constexpr double unit_roundoff = 0x1.0p-24;
};

// TC -> TS; bfloat16 by round-to-nearest-even on the float bits (NaN stays NaN)
template <typename TS, typename TC>
__device__ __forceinline__ TS to_basis(TC x) {
    if constexpr (std::is_same<TS, bf16_t>::value) {
        const uint32_t u = __float_as_uint(static_cast<float>(x));
        if ((u & 0x7fffffffu) > 0x7f800000u) return bf16_t{static_cast<uint16_t>((u >> 16) | 0x40u)};
        return bf16_t{static_cast<uint16_t>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16)};
    } else {
        return static_cast<TS>(x);
    }
}

template <typename TC, typename TS>
__device__ __forceinline__ TC from_basis(TS v) {
    if constexpr (std::is_same<TS, bf16_t>::value) {
        return static_cast<TC>(__uint_as_float(static_cast<uint32_t>(v.bits) << 16));
    } else {
        return static_cast<TC>(v);
    }
}

// a * b + c rounded once.  The library is compiled without floating-point
// contraction, so every fused multiply-add is written out: two instances of a
// kernel (or two kernels) that must give the same bits do the same operations
// whatever the compiler's scheduling.
__device__ __forceinline__ double madd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float madd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// acc + a * b for an FP64 accumulator: fused when the product is FP64, else
// the product rounded in the arithmetic type and added in FP64
__device__ __forceinline__ double dot_acc(double acc, double a, double b) { return __builtin_fma(a, b, acc); }
__device__ __forceinline__ double dot_acc(double acc, float a, float b) { return acc + static_cast<double>(a * b); }

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
// One DPP step on a double: each lane adds the value the DPP pattern `CTRL`
// reads from another lane (lanes outside ROW_MASK, or with no source, add 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double x) {
    const int lo = __double2loint(x);
    const int hi = __double2hiint(x);
    const int lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, true);
    const int hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, true);
    return x + __hiloint2double(hi2, lo2);
}

__device__ __forceinline__ double readlane_d(double x, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront with DPP (pairs, quads, half rows, rows,
// then the row broadcasts of lanes 15 and 31); the total forms in lane 63 and
// is broadcast.  The addition order is fixed, so the result is reproducible
// and identical in every lane.  All lanes must be active.
__device__ __forceinline__ double wave_sum(double v) {
    v = dpp_add<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
    v = dpp_add<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
    v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
    v = dpp_add<0x140, 0xf>(v);  // row_mirror
    v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return readlane_d(v, kWave - 1);
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

// block_sum whose thread v hands sum v to put(v, sum) itself (same order of
// additions), without the closing synchronisation: lds_tmp must not be
// rewritten before the caller's next __syncthreads().
template <int NV, typename Put>
__device__ __forceinline__ void block_sum_put(const double (&vals)[NV], int nv, double* lds_tmp, Put put) {
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
        put(static_cast<int>(threadIdx.x), acc);
    }
}

// Loads of values that other workgroups stored before the last grid barrier.
// They are device-coherent (relaxed agent-scope atomic loads, which bypass the
// CU's L1 and a stale copy in this XCD's L2), so a barrier whose readers use
// them needs no acquire fence: the cache invalidation that fence performs costs
// about 1.7 us per barrier on this chip.  A workgroup's own earlier stores are
// visible to it through the ordinary path.
__device__ __forceinline__ double load_coherent(const double* p) {
    return __longlong_as_double(static_cast<long long>(__hip_atomic_load(
        reinterpret_cast<unsigned long long*>(const_cast<double*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
}
__device__ __forceinline__ float load_coherent(const float* p) {
    return __uint_as_float(
        __hip_atomic_load(reinterpret_cast<unsigned*>(const_cast<float*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ bf16_t load_coherent(const bf16_t* p) {
    // the aligned 32-bit word holding the value
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    const unsigned w = __hip_atomic_load(reinterpret_cast<unsigned*>(a & ~static_cast<uintptr_t>(3)), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return bf16_t{static_cast<uint16_t>((a & 2) ? (w >> 16) : (w & 0xffffu))};
}

// Stores of streamed outputs (basis columns, the halo buffer): non-temporal,
// so they do not linger as dirty L2 lines that the next grid barrier's
// release has to write back.
__device__ __forceinline__ void store_stream(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_stream(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_stream(bf16_t* p, bf16_t v) {
    __builtin_nontemporal_store(v.bits, reinterpret_cast<uint16_t*>(p));
}

// This lane's share of sum_g col[g]: g = lane, lane + 64, ... < G, added in g
// order.  The partials were stored by other workgroups before a grid barrier
// and are read device-coherently.  The loads are issued four at a time before
// the adds, so the sum waits for one memory round trip per 256 entries rather
// than one per 64.
__device__ __forceinline__ double lane_strided_sum(const double* col, int G, int lane) {
    double acc = 0.0;
    for (int g0 = lane; g0 < G; g0 += 4 * kWave) {
        double t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) t[u] = (g0 + u * kWave < G) ? load_coherent(col + g0 + u * kWave) : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (g0 + u * kWave < G) acc += t[u];
    }
    return acc;
}

// Every block sums partial[v * G + g] over g (fixed order) for v < nv; result
// in lds_out[0..nv).  One wavefront per value, lanes stride over g.
__device__ __forceinline__ void grid_sum(const double* partial, int G, int nv, double* lds_out) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    for (int v = wid; v < nv; v += nw) {
        double acc = lane_strided_sum(partial + static_cast<int64_t>(v) * G, G, lane);
        acc = wave_sum(acc);
        if (lane == 0) lds_out[v] = acc;
    }
    __syncthreads();
}

// --------------------------------------------------------------------------
// Tagged partial sums.  A double is published without a grid barrier as two
// relaxed 64-bit stores, each holding one 32-bit half of the value in its low
// word and a tag in its high word.  A reader that finds the expected tag in
// both words has the value (each 64-bit access is single-copy atomic).  Where
// nothing but the partials themselves must be ordered, this replaces a grid
// barrier followed by grid_sum: the wait and the loads of the partials are
// the same memory round trip.  Tags must change from one use of a slot to the
// next and must not match the slots' contents at launch (the host clears
// them, tags start at 1).
// --------------------------------------------------------------------------
__device__ __forceinline__ void tagged_store(unsigned long long* slot, double v, unsigned tag) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned long long t = static_cast<unsigned long long>(tag) << 32;
    __hip_atomic_store(slot, t | (b >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(slot + 1, t | (b & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// This lane's share of sum_g of the tagged partials col[2g], col[2g + 1]
// (g = lane, lane + 64, ... < G, in the order of lane_strided_sum).  Each
// group of four partials is reloaded until all carry `tag`; the wait is
// bounded like the grid barrier's (abort[0] raised after `limit` ticks of the
// 100 MHz counter, or already raised: the sum is then meaningless and the
// host reports the time-out).
__device__ __forceinline__ double tagged_lane_sum(const unsigned long long* col, int G, int lane, unsigned tag,
                                                  int* abort, uint64_t limit) {
    const unsigned long long want = static_cast<unsigned long long>(tag);
    double acc = 0.0;
    for (int g0 = lane; g0 < G; g0 += 4 * kWave) {
        unsigned long long hi[4], lo[4];
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        for (;;) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                hi[u] = want << 32;
                lo[u] = want << 32;
                if (g0 + u * kWave < G) {
                    const unsigned long long* q = col + 2 * static_cast<int64_t>(g0 + u * kWave);
                    hi[u] = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    lo[u] = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            bool ok = true;
#pragma unroll
            for (int u = 0; u < 4; ++u) ok = ok && (hi[u] >> 32) == want && (lo[u] >> 32) == want;
            if (ok) break;
            if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
            if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
                __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (g0 + u * kWave < G)
                acc += __longlong_as_double(static_cast<long long>((hi[u] << 32) | (lo[u] & 0xffffffffull)));
    }
    return acc;
}

// grid_sum over tagged partials part[2 (v G + g) + {0, 1}], v < nv, by the
// wavefronts from `first` on (the others, e.g. one polling a barrier, just
// join the closing synchronisation); result in lds_out[0..nv).  Ends with a
// __syncthreads().
__device__ __forceinline__ void grid_sum_tagged(const unsigned long long* part, int G, int nv, unsigned tag,
                                                double* lds_out, int* abort, uint64_t limit, int first = 0) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave - first;
    for (int v = wid - first; v >= 0 && v < nv; v += nw) {
        double acc = tagged_lane_sum(part + 2 * static_cast<int64_t>(v) * G, G, lane, tag, abort, limit);
        acc = wave_sum(acc);
        if (lane == 0) lds_out[v] = acc;
    }
    __syncthreads();
}

// Tagged single floats: a basis entry published by its owner without a grid
// barrier, as one relaxed 64-bit word (tag in the high half, the float's bits
// in the low half), read by other workgroups that wait for its tag.
__device__ __forceinline__ void tagged_put(unsigned long long* slot, float v, unsigned tag) {
    __hip_atomic_store(slot, (static_cast<unsigned long long>(tag) << 32) | __float_as_uint(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Reload until the tag is `tag`; bounded like the other waits (abort[0] raised
// after `limit` ticks, or already raised: the value is then meaningless).
__device__ __forceinline__ float tagged_get(const unsigned long long* slot, unsigned tag, int* abort,
                                            uint64_t limit) {
    const unsigned long long want = static_cast<unsigned long long>(tag);
    unsigned long long wd = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__builtin_expect((wd >> 32) != want, 0)) {
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        for (;;) {
            __builtin_amdgcn_s_sleep(1);
            wd = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((wd >> 32) == want) break;
            if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
            if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
                __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    return __uint_as_float(static_cast<unsigned>(wd & 0xffffffffull));
}

// --------------------------------------------------------------------------
// Split-phase grid barrier for a cooperative launch (all blocks resident).
//
// Arrival is counted per XCD (the chip's 8 L2 domains, read from the XCC_ID
// hardware register): each block adds 1 to its XCD's counter, and the last
// arriver on an XCD -- by then every block of that XCD has finished its stores
// into the shared L2 -- issues one agent-scope release (L2 write-back) for the
// whole XCD and publishes the generation number in its XCD's flag.  Waiters
// poll the flags of the XCDs holding blocks (one lane per XCD) and take an
// agent-scope acquire, or none (wait_relaxed) when they read other blocks'
// data device-coherently.  This replaces G serialised L2 write-backs and G
// contended atomics with 8 of each, and needs no global counter (measured:
// 2.66 us per barrier plus a grid sum, against 2.91 us through a global
// counter and generation word).  In `per_block_release` mode every block
// also releases before arriving (the textbook protocol), which must give
// bit-identical results.
//
// Waits are bounded: after `limit` ticks of the 100 MHz real-time counter the
// block raises abort[0]; later waits return at once, so the kernel drains and
// the host reports SGMRES_ETIMEOUT.  Counters are monotone within a launch and
// must be zero at launch (SyncWords, cleared by the host before each launch).
// --------------------------------------------------------------------------
struct SyncWords {
    unsigned xcnt[16 * 64];  // per-XCD arrivals, 256 B apart
    unsigned reg[16 * 64];   // per-XCD registered blocks, 256 B apart
    unsigned gcount;         // XCD-leader arrivals (+ registrations)
    unsigned pad0[63];
    unsigned gen;            // unused (kept for the layout of the setup counters)
    unsigned pad1[63];
    unsigned xflag[16 * 64]; // per-XCD published generation, 256 B apart
};

__device__ __forceinline__ unsigned xcc_id() {
    // HW_REG_XCC_ID (hardware register 20), bits [3:0]
    return static_cast<unsigned>(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20)) & 0xfu;
}

struct GridSync {
    SyncWords* w;
    int* abort;
    uint64_t limit;
    unsigned G;
    unsigned xcc;
    unsigned my_size;  // blocks on this XCD
    unsigned nx;       // XCDs holding at least one block
    unsigned xmask;    // bit x: XCD x holds at least one block
    unsigned seq;
    bool per_block_release;

    __device__ __forceinline__ bool spin_ge(unsigned* p, unsigned target) {
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
            if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
                __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        return true;
    }

    // Once per launch, by every block: count blocks per XCD (one flat barrier);
    // lds2: 3 unsigned of LDS.
    __device__ void setup(unsigned* lds2) {
        seq = 0;
        xcc = xcc_id();
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(&w->reg[xcc * 64], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&w->gcount, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            spin_ge(&w->gcount, G);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            unsigned k = 0, m = 0;
            for (int i = 0; i < 16; ++i)
                if (__hip_atomic_load(&w->reg[i * 64], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ++k;
                    m |= 1u << i;
                }
            lds2[0] = __hip_atomic_load(&w->reg[xcc * 64], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            lds2[1] = k;
            lds2[2] = m;
        }
        __syncthreads();
        my_size = lds2[0];
        nx = lds2[1];
        xmask = lds2[2];
        __syncthreads();
    }

    // All prior global writes of this block become visible to every block that
    // returns from the matching wait().  Thread `who` does the counting (and
    // the XCD's write-back when last); the other wavefronts go on at once,
    // so work placed between arrive() and wait() can overlap that latency.
    __device__ __forceinline__ void arrive(unsigned who = 0) {
        ++seq;
        __syncthreads();
        if (threadIdx.x == who) {
            if (per_block_release) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const unsigned old =
                __hip_atomic_fetch_add(&w->xcnt[xcc * 64], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (old + 1 == seq * my_size) {
                // the XCD's last arriver: one write-back covers its XCD
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_store(&w->xflag[xcc * 64], seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }

    // wavefront 0 polls the flags of the XCDs holding blocks, lane x for XCD x
    __device__ __forceinline__ void spin_flags() {
        if (threadIdx.x < kWave) {
            const unsigned lane = threadIdx.x;
            const bool mine = lane < 16 && ((xmask >> lane) & 1u);
            const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
            for (;;) {
                const unsigned f =
                    mine ? __hip_atomic_load(&w->xflag[lane * 64], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : seq;
                if (__all(f >= seq)) break;
                if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
                if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
                    if (lane == 0) __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
    }

    __device__ __forceinline__ void wait() {
        spin_flags();
        if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
    }

    // wait() without the acquire fence: afterwards the block may read other
    // blocks' stores from before their arrival only through load_coherent.
    // (The releases are unchanged; loads issued after the flags are seen
    // reach the device-coherent level, where those stores already are.)
    __device__ __forceinline__ void wait_relaxed() {
        spin_flags();
        __syncthreads();
    }

    __device__ __forceinline__ void sync() {
        arrive();
        wait();
    }
};

// --------------------------------------------------------------------------
// Block-local sketch lists.  The sparse sign pattern of the block's own rows
// (RB = R * BLOCK rows; thread t owns local rows r * BLOCK + t) is generated
// once per cycle and regrouped by sketch row: list e holds the local rows
// whose column of S has a nonzero in row e, each packed as
// (local << 1) | negative, in ascending local order.  A block's share of S v
// is then a fixed-order sum over each list: no atomics, reproducible bits.
// --------------------------------------------------------------------------
constexpr int kSketchParts = 4;  // each list is summed in this many pieces

// raw: scratch of at least zeta * RB uint16 and BLOCK * RB / 256 bytes (the
// pattern, then the ordering bitmaps); lstart: s + 1 ints; lcount: s ints (the
// list lengths on return); lists: sketch_lists_len(zeta * RB, s, PAD4) uint16.
// PAD4: every list starts at a multiple of four entries (lists then 8-byte
// aligned) and is followed by zero entries up to the next one, so a group of
// four entries is one 8-byte load.  Ends with a __syncthreads().
__host__ __device__ constexpr int sketch_lists_len(int entries, int s, bool pad4) {
    return pad4 ? entries + 3 * s : entries;
}

template <int R, int BLOCK, bool PAD4 = false>
__device__ __forceinline__ void sketch_lists_build(uint64_t seed, uint32_t cycle, int64_t base, int64_t n, int s, int zeta,
                                   uint16_t* raw, int* lstart, int* lcount, uint16_t* lists) {
    constexpr int RB = R * BLOCK;
    const int tid = threadIdx.x;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
        if (row < n) sketch_column(seed, cycle, row, s, zeta, raw + r * BLOCK + tid, RB);
    }
    for (int e = tid; e < s; e += BLOCK) lcount[e] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
        if (row < n)
            for (int t = 0; t < zeta; ++t) atomicAdd(&lcount[raw[t * RB + r * BLOCK + tid] >> 1], 1);
    }
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int e = 0; e < s; ++e) {
            lstart[e] = run;
            run += PAD4 ? ((lcount[e] + 3) & ~3) : lcount[e];
            lcount[e] = 0;
        }
        lstart[s] = run;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
        if (row < n) {
            const int local = r * BLOCK + tid;
            for (int t = 0; t < zeta; ++t) {
                const unsigned e = raw[t * RB + local];
                const int pos = lstart[e >> 1] + atomicAdd(&lcount[e >> 1], 1);
                lists[pos] = static_cast<uint16_t>((local << 1) | (e & 1u));
            }
        }
    }
    __syncthreads();
    // Fixed order inside each list (ascending local row): wavefront w takes
    // lists w, w + NW, ...  It marks the list's rows in a bitmap of the
    // block's rows (and their signs in a second one), both in the raw scratch,
    // which is no longer needed; then each lane reads one 64-row word, and
    // the words' popcounts, scanned across the lanes in word order, give where
    // its rows go.  A row appears at most once in a list (the zeta rows of a
    // column of S are distinct).
    {
        constexpr int NW = BLOCK / kWave;
        constexpr int NWORDS = (RB + 63) / 64;
        const int lane = tid & (kWave - 1);
        const int wid = tid / kWave;
        unsigned long long* bm = reinterpret_cast<unsigned long long*>(raw) + static_cast<int64_t>(wid) * 2 * NWORDS;
        unsigned long long* sg = bm + NWORDS;
        for (int w = lane; w < 2 * NWORDS; w += kWave) bm[w] = 0ull;
        for (int e = wid; e < s; e += NW) {
            const int q0 = lstart[e];
            const int len = lcount[e];
            for (int i = lane; i < len; i += kWave) {
                const unsigned key = lists[q0 + i];
                const unsigned u = key >> 1;
                atomicOr(&bm[u >> 6], 1ull << (u & 63u));
                if (key & 1u) atomicOr(&sg[u >> 6], 1ull << (u & 63u));
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            int done = 0;
            for (int w0 = 0; w0 < NWORDS; w0 += kWave) {
                const int w = w0 + lane;
                unsigned long long word = 0ull, sgn = 0ull;
                if (w < NWORDS) {
                    word = bm[w];
                    sgn = sg[w];
                    bm[w] = 0ull;
                    sg[w] = 0ull;
                }
                const int c = __popcll(word);
                int incl = c;
#pragma unroll
                for (int o = 1; o < kWave; o <<= 1) {
                    const int t = __shfl_up(incl, o, kWave);
                    if (lane >= o) incl += t;
                }
                int pos = q0 + done + incl - c;
                while (word) {
                    const int b = __ffsll(static_cast<long long>(word)) - 1;
                    lists[pos++] = static_cast<uint16_t>(((w * 64 + b) << 1) | static_cast<int>((sgn >> b) & 1ull));
                    word &= word - 1ull;
                }
                done += __shfl(incl, kWave - 1, kWave);
            }
            if constexpr (PAD4)
                for (int q = q0 + len + lane; q < lstart[e + 1]; q += kWave) lists[q] = 0;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
    }
    __syncthreads();
}

__device__ __forceinline__ double signed_val(const double* v, unsigned u) {
    const double x = v[u >> 1];
    return (u & 1u) ? -x : x;
}

// Piece `part` of list `row` of vector vv: entries [a0, a1) of the list summed
// four at a time (independent loads), the four sums added pairwise.
__device__ __forceinline__ double sketch_piece(const double* vv, const int* lstart, const uint16_t* lists, int row,
                                               int part) {
    const int q0 = lstart[row];
    const int len = lstart[row + 1] - q0;
    const int a0 = q0 + (len * part) / kSketchParts;
    const int a1 = q0 + (len * (part + 1)) / kSketchParts;
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    int q = a0;
    for (; q + 4 <= a1; q += 4) {
        const unsigned u0 = lists[q], u1 = lists[q + 1], u2 = lists[q + 2], u3 = lists[q + 3];
        acc0 += signed_val(vv, u0);
        acc1 += signed_val(vv, u1);
        acc2 += signed_val(vv, u2);
        acc3 += signed_val(vv, u3);
    }
    for (; q < a1; ++q) acc0 += signed_val(vv, lists[q]);
    return (acc0 + acc1) + (acc2 + acc3);
}

// Block share (unscaled) of S v over sketch rows [r0, r1) for vectors
// v = v0 .. v0+nvec-1 staged in vals[v * RB + local].  Each list is cut into
// kSketchParts pieces, each piece summed four entries at a time (independent
// loads), and the pieces added in a fixed order; fin(v, row, value) receives
// each sum once.  sk_tmp: nvec * (r1 - r0) * kSketchParts doubles.  Starts
// after the caller's __syncthreads() that published vals; contains one
// __syncthreads().
template <int BLOCK, typename Fin>
__device__ __forceinline__ void sketch_lists_reduce(int v0, int nvec, int r0, int r1, const double* vals, int RB,
                                                    const int* lstart, const uint16_t* lists, double* sk_tmp,
                                                    Fin fin) {
    const int tid = threadIdx.x;
    const int nrow = r1 - r0;
    const int tasks = nvec * nrow * kSketchParts;
    for (int t = tid; t < tasks; t += BLOCK) {
        const int part = t % kSketchParts;
        const int e = t / kSketchParts;
        const int v = e / nrow;
        sk_tmp[t] = sketch_piece(vals + (v0 + v) * RB, lstart, lists, r0 + (e - v * nrow), part);
    }
    __syncthreads();
    for (int e = tid; e < nvec * nrow; e += BLOCK) {
        double a = 0.0;
#pragma unroll
        for (int part = 0; part < kSketchParts; ++part) a += sk_tmp[e * kSketchParts + part];
        const int v = e / nrow;
        fin(v0 + v, r0 + (e - v * nrow), a);
    }
}

// Piece `part` of a list built with PAD4: the list's groups of four entries
// are dealt to the pieces in order, each group read with one 8-byte load; the
// entries of a group are added to four separate sums (zero entries past the
// list's end skipped), the four sums then added pairwise.
__device__ __forceinline__ double sketch_piece4(const double* vv, const int* lstart, const int* lcount,
                                                const uint16_t* lists, int row, int part) {
    const int len = lcount[row];
    const int ng = (len + 3) >> 2;
    const int g0 = (ng * part) / kSketchParts;
    const int g1 = (ng * (part + 1)) / kSketchParts;
    const uint2* L = reinterpret_cast<const uint2*>(lists + lstart[row]);
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    for (int g = g0; g < g1; ++g) {
        const uint2 w = L[g];
        const int rem = len - 4 * g;  // entries of this group inside the list (>= 1)
        const double x0 = signed_val(vv, w.x & 0xffffu), x1 = signed_val(vv, w.x >> 16);
        const double x2 = signed_val(vv, w.y & 0xffffu), x3 = signed_val(vv, w.y >> 16);
        acc0 += x0;
        if (rem > 1) acc1 += x1;
        if (rem > 2) acc2 += x2;
        if (rem > 3) acc3 += x3;
    }
    return (acc0 + acc1) + (acc2 + acc3);
}

// Block partial of S v written to dst[(v * s + row) * G + blk] over lists
// built with PAD4, without a block-wide synchronisation or LDS scratch: the
// kSketchParts pieces of a list are summed by consecutive lanes of one
// wavefront and added in piece order by the first of them.  Starts after a
// __syncthreads() that published vals; vals must stay unchanged until the
// caller's next block synchronisation.
template <int BLOCK>
__device__ __forceinline__ void sketch_lists_apply_lanes(int v0, int nvec, int r0, int r1, const double* vals,
                                                         int RB, int s, const int* lstart, const int* lcount,
                                                         const uint16_t* lists, double* dst, int G, int blk) {
    static_assert(BLOCK % kWave == 0 && kWave % kSketchParts == 0, "pieces of a list share a wavefront");
    const int tid = threadIdx.x;
    const int first = (tid & (kWave - 1)) & ~(kSketchParts - 1);
    const int nrow = r1 - r0;
    const int tasks = nvec * nrow * kSketchParts;  // a multiple of kSketchParts: the lanes of
    for (int t = tid; t < tasks; t += BLOCK) {     // a list are active together
        const int part = t % kSketchParts;
        const int e = t / kSketchParts;
        const int v = e / nrow;
        const int row = r0 + (e - v * nrow);
        const double piece = sketch_piece4(vals + (v0 + v) * RB, lstart, lcount, lists, row, part);
        double a = 0.0;
#pragma unroll
        for (int u = 0; u < kSketchParts; ++u) a += __shfl(piece, first + u, kWave);
        if (part == 0) dst[static_cast<int64_t>((v0 + v) * s + row) * G + blk] = a;
    }
}

// Blocks of a launch are dealt round-robin to the 8 XCDs; give each XCD a
// contiguous range of logical blocks so that neighbouring rows share an L2.
__device__ __forceinline__ int xcd_logical_block(int phys, int G) {
    if ((G & 7) != 0) return phys;
    return (phys & 7) * (G >> 3) + (phys >> 3);
}

}  // namespace sg
