// Streaming k-truncated Arnoldi basis kernel: one cooperative launch per
// cycle for systems beyond the resident kernels' capacity, and for blocks of
// right-hand sides that share one matrix (arXiv:2111.00113, Algorithm 1 basis
// loop; truncated-Arnoldi recurrence of Section 1.2.2 with two classical
// Gram-Schmidt passes).
//
// Work items are (row, right-hand side) pairs q = i * NR + rhs, which is also
// where the pair's entry sits in a basis column: column j of B holds the NR
// bases' j-th vectors interleaved, so the gathers of one row's NR entries are
// one contiguous run and the NR right-hand sides share every read of A.  A
// tile is P * BLOCK consecutive pairs; thread t of a block takes pairs
// tile * P * BLOCK + p * BLOCK + t, p < P, so its right-hand side is t % NR.
// The window (the last k basis vectors) comes from an LDS ring of the newest
// columns of the block's tile, then from registers (FP32 arithmetic, one
// right-hand side), then from B; A is read through its sliced ELL copy (entry
// e of row i at sp[i / 64] + 64 e + i % 64).
//
// Per step j (two tagged reductions and one grid barrier):
//   phase 1  m = A b_j; per right-hand side partials <m,m>, W^T m  (tagged)
//   phase 2  h = W^T m; w = m - W h; partials <w,w>, W^T w           (tagged)
//            (HBM state: w is not stored; phase 3 forms it again from m)
//   phase 3  h2 = W^T w; nu^2 = <w,w> - |h2|^2 (window orthonormal to
//            rounding); b_{j+1} = (w - W h2) / nu; H column j   -- barrier --
// With REG state (one tile per block) m and w stay in registers for the whole
// step; otherwise (HST) each block walks its tiles and parks them in a state
// buffer between phases.  The sketch is not formed here: S B is formed from
// the finished basis and S A B from it through the Arnoldi relation
// A b_j = sum_a H[a, j] b_{j-a} + nu_j b_{j+1} (so the last step also forms
// b_{d+1}).
#pragma once

#include "common.hpp"
#include "internal.hpp"

namespace sg {
namespace stream_detail {

constexpr int kBlock = kStreamBlock;
constexpr int kNW = kBlock / kWave;
constexpr int kNV = kStreamMaxK + 1;  // values per reduction: a norm and the window dots

__device__ __forceinline__ double gs_sub(double x, double h, double v) { return __builtin_fma(-h, v, x); }
__device__ __forceinline__ float gs_sub(float x, float h, float v) { return __builtin_fmaf(-h, v, x); }

// Block sum per right-hand side of nv per-thread values (thread t holds values
// of right-hand side t % NR), in a fixed order: the lanes of one right-hand
// side inside a wavefront by an xor butterfly (the same bits in each of them),
// then the wavefronts in order.  put(v, rhs, sum) is called once per value by
// one thread.  red: kNW * nv * NR doubles.  Ends with a __syncthreads().
template <int NR, typename Put>
__device__ __forceinline__ void block_sum_rhs(const double (&vals)[kNV], int nv, double* red, Put put) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
#pragma unroll
    for (int v = 0; v < kNV; ++v) {
        if (v < nv) {
            double x = vals[v];
#pragma unroll
            for (int off = NR; off < kWave; off <<= 1) x += __shfl_xor(x, off, kWave);
            if (lane < NR) red[(v * NR + lane) * kNW + wid] = x;
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nv * NR; idx += kBlock) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < kNW; ++q) acc += red[idx * kNW + q];
        put(idx / NR, idx % NR, acc);
    }
    __syncthreads();
}

// LDS ring slots of an instance: as many tile columns (P * 1024 entries of TC)
// as fit in 150 KiB, at most the window length; none with HBM state
template <typename TC, int P, bool HST>
__host__ __device__ constexpr int ring_slots() {
    return HST ? 0 : ((150 * 1024) / (P * kBlock * static_cast<int>(sizeof(TC))) < kStreamMaxK
                          ? (150 * 1024) / (P * kBlock * static_cast<int>(sizeof(TC)))
                          : kStreamMaxK);
}

template <typename TC, typename TS, int NR, int P, bool HST>
__global__ __launch_bounds__(kBlock) void stream_kernel(StreamParams p) {
    constexpr int NL = ring_slots<TC, P, HST>();
    static_assert(kWave % NR == 0, "a wavefront holds whole rows of right-hand sides");
    static_assert(P % 8 == 0 || P <= 8, "pairs are walked in groups");
    constexpr int T = P * kBlock;  // pairs per tile
    // pairs per SpMV group (each nonzero slot issues the group's loads
    // together; wider groups measured slower: 64 -> 73 us per step at
    // n = 2^22 in FP32 with all 16 pairs of a tile)
    constexpr int PG = P < 4 ? P : 4;
    // window entries read from HBM (those not in the LDS ring)
    constexpr int NH = kStreamMaxK - NL;
    // FP32 arithmetic, one right-hand side, register state: the newest KH of
    // them stay in registers (at most 32 a lane) and move down the window
    // there, so no phase reads them from HBM (FP64 and several right-hand
    // sides: the registers spill)
    constexpr int KH0 = 32 / (P * static_cast<int>(sizeof(TC)) / 4);
    constexpr int KH = (sizeof(TC) == 4 && NR == 1 && !HST && NL > 0) ? (NH < KH0 ? NH : KH0) : 0;
    // otherwise the SpMV group's HBM window entries are loaded with its first
    // slot when they take at most 8 registers a lane
    constexpr bool PRE = KH == 0 && NH > 0 && NH * PG * static_cast<int>(sizeof(TC)) <= 32;
    // FP32 arithmetic, one right-hand side: the next slot's column indices
    // and values are loaded while the current slot's gathers are in flight
    constexpr bool LA = sizeof(TC) == 4 && NR == 1;
    // pairs whose window loads are in flight together in the Gram-Schmidt
    // phases
    constexpr int WP = P < 4 ? P : 4;
    __shared__ double red[kNW * kNV * NR];
    __shared__ double coefA[kNV * NR];  // [v * NR + rhs]: v = 0 <m,m>, 1 + a: h_a
    __shared__ double coefB[kNV * NR];  // v = 0 <w,w>, 1 + a: h2_a
    __shared__ double nus[NR];
    __shared__ int dead[NR];
    __shared__ int dcs[NR];
    __shared__ unsigned sync_lds[3];

    const int G = gridDim.x;
    const int blk = xcd_logical_block(blockIdx.x, G);
    const int tid = threadIdx.x;
    const int wid_s = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int rhs = tid % NR;
    const int64_t n = p.n;
    const int64_t npairs = n * NR;
    const int64_t nt = (npairs + T - 1) / T;
    const int64_t t0 = HST ? (static_cast<int64_t>(blk) * nt) / G : blk;
    const int64_t t1 = HST ? (static_cast<int64_t>(blk + 1) * nt) / G : blk + 1;
    const int d = p.d, k = p.k;
    const TC* Av = static_cast<const TC*>(p.val);
    TS* Bs = static_cast<TS*>(p.B);
    TC* state = static_cast<TC*>(p.state);
    const int64_t ldb = p.ldb;
    constexpr double uround = BasisPrec<TC>::unit_roundoff;
    // columns start on 256-byte boundaries and blocks own whole cache lines
    // of them: other blocks' entries of a column written during this launch
    // are read with plain loads (no cache can hold a stale copy), else
    // device-coherently
    const bool fresh = ((reinterpret_cast<uintptr_t>(p.B) | static_cast<uintptr_t>(ldb * sizeof(TS))) & 255u) == 0;
    auto ldB = [&](const TS* q) -> TC { return from_basis<TC>(fresh ? *q : load_coherent(q)); };
    // Register state: the newest nl basis columns of the block's tile also sit
    // in an LDS ring (slot c % nl holds column c, as the rounded stored values),
    // so window entries a < nl and the SpMV's gathers of the tile's own rows
    // (NR = 1) are LDS reads instead of HBM reads
    extern __shared__ __align__(16) unsigned char ring_raw[];
    TC* ring = reinterpret_cast<TC*>(ring_raw);
    const int64_t tbase = t0 * T;  // first pair of the block's (only) tile in register mode

    GridSync bar{static_cast<SyncWords*>(p.sync), p.abort, p.spin_limit, static_cast<unsigned>(G), 0u, 0u, 0u, 0u, 0u,
                 p.per_block_release != 0};
    bar.setup(sync_lds);

    const bool timing = p.phase_ticks != nullptr && blk == 0 && tid == 0;
    uint64_t t_last = timing ? __builtin_amdgcn_s_memrealtime() : 0;
    auto tick = [&](int q) {
        if (timing) {
            const uint64_t t = __builtin_amdgcn_s_memrealtime();
            p.phase_ticks[q] += t - t_last;
            t_last = t;
        }
    };

    // ---- b_1 = r / |r| (a right-hand side with r = 0 is dead from the start)
    if (tid < NR) {
        dead[tid] = !(p.beta[tid] > 0.0);
        dcs[tid] = dead[tid] ? 0 : d;
    }
    __syncthreads();
    {
        const double beta = p.beta[rhs];
        const bool dz = dead[rhs] != 0;
        for (int64_t tl = t0; tl < t1; ++tl) {
#pragma unroll
            for (int pp = 0; pp < P; ++pp) {
                const uint32_t q = static_cast<uint32_t>(tl * T) + static_cast<uint32_t>(pp * kBlock + tid);
                if (q < npairs) {
                    const TS b1 = to_basis<TS>(dz ? TC(0) : static_cast<TC>(p.r[q] / beta));
                    Bs[q] = b1;
                    if constexpr (NL > 0) ring[pp * kBlock + tid] = from_basis<TC>(b1);
                }
            }
        }
    }
    bar.sync();  // b_1 complete everywhere

    // register state, one right-hand side: slot e of the wavefront's slice for
    // pair pp whose column is the row plus the same offset in every lane (a
    // diagonal of A across the slice) keeps that offset in LDS, and the SpMV
    // forms those columns instead of loading them; found once per launch
    constexpr bool kOff = !HST && NR == 1;
    constexpr int kOffSlots = 16;
    constexpr int kIrregular = INT_MIN;
    __shared__ int doff[kOff ? kNW * P * kOffSlots : 1];
    if constexpr (kOff) {
        const int64_t nsl = (n + kWave - 1) / kWave;
#pragma unroll
        for (int pp = 0; pp < P; ++pp) {
            const int64_t row0 = tbase + static_cast<int64_t>(pp) * kBlock + wid_s * kWave;  // the slice's first row
            const int64_t sl = row0 / kWave;
            int64_t a = 0;
            int K = 0;
            if (sl < nsl) {
                a = p.sp[sl];
                K = static_cast<int>((p.sp[sl + 1] - a) / kWave);
            }
            // the slots' column loads all in flight, then one vote per slot
            int cs[kOffSlots];
#pragma unroll
            for (int e = 0; e < kOffSlots; ++e) cs[e] = e < K ? (p.ci + a)[e * kWave + (tid & (kWave - 1))] : 0;
#pragma unroll
            for (int e = 0; e < kOffSlots; ++e) {
                int o = kIrregular;
                if (e < K) {
                    const int d = cs[e] - static_cast<int>(row0 + (tid & (kWave - 1)));
                    const int d0 = __builtin_amdgcn_readfirstlane(d);
                    if (__all(d == d0)) o = d0;
                }
                if ((tid & (kWave - 1)) == 0) doff[(wid_s * P + pp) * kOffSlots + e] = o;
            }
        }
        __syncthreads();
    }

    TC mreg[HST ? 1 : P];
    // kept window entries: wk[h][pp] is entry NL + h of pair pp
    TC wk[KH > 0 ? KH : 1][KH > 0 ? P : 1];
#pragma unroll
    for (int h = 0; h < (KH > 0 ? KH : 1); ++h)
#pragma unroll
        for (int pp = 0; pp < (KH > 0 ? P : 1); ++pp) wk[h][pp] = TC(0);
    int flags = 0;
    int dc = d;
    for (int j = 0; j < d; ++j) {
        const int kw = min(j + 1, k);
        const TS* bj = Bs + static_cast<int64_t>(j) * ldb;
        const unsigned tag = static_cast<unsigned>(j + 1);
        // window entry a (0 = newest; a < min(j + 1, k)) of the thread's pair
        // at local index loc: ring slot (j - a) % NL when a < NL, else B
        int soff[NL > 0 ? NL : 1] = {};
        if constexpr (NL > 0) {
#pragma unroll
            for (int a = 0; a < NL; ++a) soff[a] = (((j - a) % NL + NL) % NL) * T;
        }
        auto ldW = [&](int a, uint32_t q, int loc) -> TC {
            if (a < NL) return ring[soff[a] + loc];
            return from_basis<TC>((Bs + static_cast<int64_t>(j - a) * ldb)[q]);
        };
        // window entry a of register-state pair pp (compile-time a and pp)
        auto wwin = [&](int a, int pp, uint32_t q) -> TC {
            if (a >= NL && a < NL + KH) return wk[a - NL][pp];
            return ldW(a, q, pp * kBlock + tid);
        };
        tick(0);

        // ---- phase 1: m = A b_j, partials <m,m> and W^T m ------------------
        double acc[kNV];
#pragma unroll
        for (int v = 0; v < kNV; ++v) acc[v] = 0.0;
        for (int64_t tl = t0; tl < t1; ++tl) {
#pragma unroll
            for (int g0 = 0; g0 < P; g0 += PG) {
                // the PG pairs' rows, slice positions and widths (one slice per
                // wavefront and pair: uniform, scalar)
                int64_t spos[PG];
                int sK[PG];
                int lrow[PG];
                int kmax = 0;
#pragma unroll
                for (int u = 0; u < PG; ++u) {
                    // the wavefront's first pair; its NR-pair rows lie in one slice
                    const int64_t qw = tl * T + static_cast<int64_t>(g0 + u) * kBlock + wid_s * kWave;
                    lrow[u] = static_cast<int>(((static_cast<uint32_t>((g0 + u) * kBlock + tid)) / NR) & (kWave - 1));
                    spos[u] = 0;
                    sK[u] = 0;
                    if (qw < npairs) {
                        const int64_t sl = (qw / NR) / kWave;
                        const int64_t a = p.sp[sl];
                        spos[u] = a;
                        sK[u] = static_cast<int>((p.sp[sl + 1] - a) / kWave);
                    }
                    kmax = max(kmax, sK[u]);
                }
                TC m[PG];
#pragma unroll
                for (int u = 0; u < PG; ++u) m[u] = TC(0);
                // slot e's column indices and values of the PG pairs
                const int doff0 = wid_s * P * kOffSlots;
                const int row0 = static_cast<int>(tbase) + tid;  // (n < 2^31 in this path)
                auto ld_slot = [&](int e, int (&c)[PG], TC (&v)[PG]) {
#pragma unroll
                    for (int u = 0; u < PG; ++u) {
                        c[u] = 0;
                        v[u] = TC(0);
                        if (e < sK[u]) {
                            const uint32_t a = static_cast<uint32_t>(e * kWave + lrow[u]);
                            int o = kIrregular;
                            if constexpr (kOff)
                                if (e < kOffSlots) o = __builtin_amdgcn_readfirstlane(doff[doff0 + (g0 + u) * kOffSlots + e]);
                            c[u] = o != kIrregular ? row0 + (g0 + u) * kBlock + o : (p.ci + spos[u])[a];
                            v[u] = (Av + spos[u])[a];
                        }
                    }
                };
                // gathers of slot e and the products' sums (each row in slot
                // order)
                auto spmv_slot = [&](int e, const int (&c)[PG], const TC (&v)[PG], TC (&m)[PG]) {
#pragma unroll
                    for (int u = 0; u < PG; ++u)
                        if (e < sK[u]) {
                            TC bv;
                            if constexpr (NR == 1 && NL > 0) {
                                const uint32_t lc = static_cast<uint32_t>(c[u] - tbase);
                                bv = lc < static_cast<uint32_t>(T) ? ring[soff[0] + lc]
                                                                   : ldB(bj + static_cast<uint32_t>(c[u]));
                            } else {
                                bv = ldB(bj + (static_cast<uint32_t>(c[u]) * NR + rhs));
                            }
                            m[u] = madd(v[u], bv, m[u]);
                        }
                };
                int c[PG];
                TC v[PG];
                if constexpr (LA) ld_slot(0, c, v);
                // the group's window entries that live in HBM, in flight
                // with the first slot
                TC wpre[PRE ? PG : 1][NH > 0 ? NH : 1];
                if constexpr (PRE) {
#pragma unroll
                    for (int u = 0; u < PG; ++u) {
                        const uint32_t q =
                            static_cast<uint32_t>(tl * T) + static_cast<uint32_t>((g0 + u) * kBlock + tid);
#pragma unroll
                        for (int h = 0; h < NH; ++h) {
                            const int a = kStreamMaxK - NH + h;
                            wpre[u][h] = (q < npairs && a < kw)
                                             ? from_basis<TC>((Bs + static_cast<int64_t>(j - a) * ldb)[q])
                                             : TC(0);
                        }
                    }
                }
                for (int e = 0; e < kmax; ++e) {
                    if constexpr (LA) {
                        // next slot's loads in flight during this slot's gathers
                        int cn[PG];
                        TC vn[PG];
                        ld_slot(e + 1, cn, vn);
                        spmv_slot(e, c, v, m);
#pragma unroll
                        for (int u = 0; u < PG; ++u) {
                            c[u] = cn[u];
                            v[u] = vn[u];
                        }
                    } else {
                        ld_slot(e, c, v);
                        spmv_slot(e, c, v, m);
                    }
                }
#pragma unroll
                for (int u = 0; u < PG; ++u) {
                    const uint32_t q = static_cast<uint32_t>(tl * T) + static_cast<uint32_t>((g0 + u) * kBlock + tid);
                    if (KH == 0 && q < npairs) {
                        acc[0] = dot_acc(acc[0], m[u], m[u]);
#pragma unroll
                        for (int a = 0; a < kStreamMaxK; ++a)
                            if (a < kw) {
                                TC wa;
                                if constexpr (PRE) {
                                    wa = a >= kStreamMaxK - NH ? wpre[u][a - (kStreamMaxK - NH)]
                                                               : ldW(a, q, (g0 + u) * kBlock + tid);
                                } else {
                                    wa = ldW(a, q, (g0 + u) * kBlock + tid);
                                }
                                acc[1 + a] = dot_acc(acc[1 + a], wa, m[u]);
                            }
                    }
                    if constexpr (HST) {
                        if (q < npairs) state[q] = m[u];
                    } else {
                        mreg[g0 + u] = m[u];
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if constexpr (KH > 0) {
            // the window dots of the tile's pairs, pairs in order
#pragma unroll
            for (int pp = 0; pp < P; ++pp) {
                const uint32_t q = static_cast<uint32_t>(tbase) + static_cast<uint32_t>(pp * kBlock + tid);
                if (q < npairs) {
                    acc[0] = dot_acc(acc[0], mreg[pp], mreg[pp]);
#pragma unroll
                    for (int a = 0; a < kStreamMaxK; ++a)
                        if (a < kw) acc[1 + a] = dot_acc(acc[1 + a], wwin(a, pp, q), mreg[pp]);
                }
                if ((pp + 1) % WP == 0) __builtin_amdgcn_sched_barrier(0);
            }
        }
        block_sum_rhs<NR>(acc, kw + 1, red, [&](int v, int r, double val) {
            tagged_store(p.part_a + 2 * (static_cast<int64_t>(v * NR + r) * G + blk), val, tag);
        });
        tick(1);

        // ---- phase 2: h, w = m - W h, partials <w,w> and W^T w ------------
        grid_sum_tagged(p.part_a, G, (kw + 1) * NR, tag, coefA, p.abort, p.spin_limit);
        tick(2);
#pragma unroll
        for (int v = 0; v < kNV; ++v) acc[v] = 0.0;
        for (int64_t tl = t0; tl < t1; ++tl) {
#pragma unroll
            for (int pp = 0; pp < P; ++pp) {
                const uint32_t q = static_cast<uint32_t>(tl * T) + static_cast<uint32_t>(pp * kBlock + tid);
                if (q < npairs) {
                    TC w;
                    if constexpr (HST) w = state[q];
                    else w = mreg[pp];
                    TC wa[kStreamMaxK];
#pragma unroll
                    for (int a = 0; a < kStreamMaxK; ++a)
                        if (a < kw) wa[a] = HST ? ldW(a, q, pp * kBlock + tid) : wwin(a, pp, q);
#pragma unroll
                    for (int a = 0; a < kStreamMaxK; ++a)
                        if (a < kw) w = gs_sub(w, static_cast<TC>(coefA[(1 + a) * NR + rhs]), wa[a]);
                    acc[0] = dot_acc(acc[0], w, w);
#pragma unroll
                    for (int a = 0; a < kStreamMaxK; ++a)
                        if (a < kw) acc[1 + a] = dot_acc(acc[1 + a], wa[a], w);
                    // HBM state keeps m: phase 3 forms w again from it (the
                    // same operations), which saves writing w back
                    if constexpr (!HST) mreg[pp] = w;
                }
                // WP pairs' window loads in flight at a time: keeps the
                // register state of many pairs from spilling
                if ((pp + 1) % WP == 0) __builtin_amdgcn_sched_barrier(0);
            }
        }
        block_sum_rhs<NR>(acc, kw + 1, red, [&](int v, int r, double val) {
            tagged_store(p.part_b + 2 * (static_cast<int64_t>(v * NR + r) * G + blk), val, tag);
        });
        tick(3);

        // ---- phase 3: h2, nu, b_{j+1} -------------------------------------
        grid_sum_tagged(p.part_b, G, (kw + 1) * NR, tag, coefB, p.abort, p.spin_limit);
        tick(4);
        if (tid < NR) {
            double h2sq = 0.0;
            for (int a = 0; a < kw; ++a) h2sq = madd(coefB[(1 + a) * NR + tid], coefB[(1 + a) * NR + tid], h2sq);
            const double nu2 = coefB[tid] - h2sq;
            const bool brk = !(nu2 > 16.0 * uround * uround * coefA[tid]);
            nus[tid] = brk ? 0.0 : sqrt(nu2);
            if (!dead[tid] && brk) {
                dead[tid] = 1;
                dcs[tid] = j + 1;
            }
        }
        __syncthreads();
        if (blk == 0) {
            for (int idx = tid; idx < NR * (k + 1); idx += kBlock) {
                const int r = idx / (k + 1), a = idx % (k + 1);
                double hv = 0.0;
                if (a == k) hv = nus[r];
                else if (a < kw) hv = coefA[(1 + a) * NR + r] + coefB[(1 + a) * NR + r];
                p.H[(static_cast<int64_t>(r) * d + j) * (k + 1) + a] = hv;
            }
        }
        if constexpr (NR == 1) {
            if (nus[0] == 0.0) {
                dc = j + 1;
                flags |= SGMRES_FLAG_BREAKDOWN;
                break;
            }
        }
        {
            const double nu = nus[rhs];
            const bool dz = !(nu > 0.0);
            const TC nu_t = static_cast<TC>(nu);
            TS* bn = Bs + static_cast<int64_t>(j + 1) * ldb;
            for (int64_t tl = t0; tl < t1; ++tl) {
#pragma unroll
                for (int pp = 0; pp < P; ++pp) {
                    const uint32_t q = static_cast<uint32_t>(tl * T) + static_cast<uint32_t>(pp * kBlock + tid);
                    if (q < npairs) {
                        TC w;
                        if constexpr (HST) w = state[q];
                        else w = mreg[pp];
                        TC wa[kStreamMaxK];
#pragma unroll
                        for (int a = 0; a < kStreamMaxK; ++a)
                            wa[a] = a < kw ? (HST ? ldW(a, q, pp * kBlock + tid) : wwin(a, pp, q)) : TC(0);
                        if constexpr (HST) {
                            // w = m - W h, as in phase 2
#pragma unroll
                            for (int a = 0; a < kStreamMaxK; ++a)
                                if (a < kw) w = gs_sub(w, static_cast<TC>(coefA[(1 + a) * NR + rhs]), wa[a]);
                        }
#pragma unroll
                        for (int a = 0; a < kStreamMaxK; ++a)
                            if (a < kw) w = gs_sub(w, static_cast<TC>(coefB[(1 + a) * NR + rhs]), wa[a]);
                        const TS st = to_basis<TS>(dz ? TC(0) : w / nu_t);
                        bn[q] = st;
                        // (the slot of column j + 1 - nl: window entry nl at the next
                        // step, which then reads it from B)
                        if constexpr (NL > 0) ring[((j + 1) % NL) * T + pp * kBlock + tid] = from_basis<TC>(st);
                        if constexpr (KH > 0) {
                            // the next step's kept entries: entry NL - 1 of
                            // this step (the ring slot just overwritten) and
                            // the kept entries moved one place down
#pragma unroll
                            for (int h = KH - 1; h > 0; --h) wk[h][pp] = wk[h - 1][pp];
                            wk[0][pp] = wa[NL - 1];
                        }
                    }
                    if ((pp + 1) % WP == 0) __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        tick(5);
        bar.arrive(kBlock - kWave);
        bar.wait_relaxed();
        tick(6);
    }
    if (blk == 0 && tid == 0) {
        if constexpr (NR == 1) {
            p.status[0] = dc;
            p.status[1] |= flags;
        }
    }
    if constexpr (NR > 1) {
        if (blk == 0 && tid < NR) {
            p.dc_rhs[tid] = dcs[tid];
            p.flags_rhs[tid] |= (dcs[tid] < d) ? SGMRES_FLAG_BREAKDOWN : 0;
        }
    }
}

}  // namespace stream_detail
}  // namespace sg
