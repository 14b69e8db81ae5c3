// spmv_truncarnoldi: one cycle of k-truncated Arnoldi basis generation fused
// with SpMV and sparse-sign sketching, as a single persistent cooperative
// launch (arXiv:2111.00113, Algorithm 1 basis loop; truncated-Arnoldi
// recurrence of Section 1.2.2; two classical Gram-Schmidt passes).
//
// Work decomposition.  Logical block b owns rows [b*R*BLOCK, (b+1)*R*BLOCK);
// thread t of it owns rows b*R*BLOCK + r*BLOCK + t, r < R, so the 64 rows of a
// wavefront in chunk r are one slice of the sliced ELL copy of A (sell.hip):
// the SpMV reads the k-th nonzero of the wavefront's rows with one contiguous
// load of values and one of columns, and sums each row in CSR order.  What a
// row needs between steps stays on chip for the whole cycle: its slice
// position and the last KW basis entries (registers), m_j = A b_j and w
// (registers).  Per step the kernel moves A's values and columns, the gathered
// b_j and the written b_{j+1} through HBM, plus per-block partial sums.
//
// Sketch.  The pattern of S restricted to the block's rows is generated once
// per cycle and sorted by sketch row into LDS lists.  Each step stages m_j (and
// b_j when S B is wanted) of the block's rows in LDS and forms the block's
// share of S m_j (and S b_j) as fixed-order sums over those lists (no atomics,
// so the result is bitwise reproducible).  The block partials of all steps are
// kept and summed across blocks once, at the end of the cycle.
//
// Per step j (three grid synchronisations, the first two carrying a
// reduction; the block's sketch work fills the waits).  The first is not a
// barrier: its partials are tagged with the step (tagged_store), and each
// block waits for the tags as it loads them.  The others are split-phase grid
// barriers:
//   phase 1  m = A b_j; tagged partials <m,m>, W^T m
//            stage m in LDS; sketch rows [0, s/3)
//   phase 2  h = W^T m (sum of the tagged partials, waiting for them);
//            w = m - W h; partial <w,w>, W^T w
//                                                        -- arrive --
//            sketch rows [s/3, 2s/3)                     -- wait --
//   phase 3  h2 = W^T w; |w - W h2|^2 = <w,w> - |h2|^2 (window orthonormal to
//            rounding); b_{j+1} = (w - W h2)/nu; H column j  -- arrive --
//            sketch rows [2s/3, s)                       -- wait --
// In the halo mode (see the kernel) the third barrier is dropped and the sketch
// is split over the first two waits.
#pragma once

#include "common.hpp"
#include "internal.hpp"

namespace sg {
namespace arnoldi_detail {

constexpr int kChunk = 8;     // reduction values per block_sum pass (global window)
constexpr int kRedSlots = 9;  // max values per block_sum: window of 8 plus a norm

// x - h * v as one fused multiply-add, the same instruction wherever the new
// basis column is formed (its owner, and blocks recomputing it for their halo)
__device__ __forceinline__ double gs_sub(double x, double h, double v) { return __builtin_fma(-h, v, x); }
__device__ __forceinline__ float gs_sub(float x, float h, float v) { return __builtin_fmaf(-h, v, x); }

// SKB: also form S b_j (SB); the solve needs only S m_j.  TC: per-row
// arithmetic type (A's values are read in TC); TS: storage type of B.  Sums of
// block partials, H and the sketch sums are FP64 in every variant.
// HALO: two grid barriers per step instead of three.  The new column b_{j+1}
// is not published by a third barrier: each block keeps its own rows of it in
// LDS, and the entries its SpMV needs from other blocks' rows come
//   - FP32 arithmetic: from their owners, which store each such entry with
//     its column number as tag in one 64-bit word of the halo buffer (rows
//     marked in the xbits bitmap); the reader reloads until the tag matches.
//     The owner cannot overwrite the word before every reader has passed the
//     next second barrier.
//   - FP64 arithmetic: recomputed by the reader as (w - W h2) / nu from w
//     (the halo buffer, written before the second barrier) and the window
//     columns, with the owner's operations in the owner's order, so the
//     values are the owner's bits.  (Publishing a double takes two tagged
//     words; measured slower: 9.84 -> 9.21 solves/s at n = 2^20.)
// Chosen when few nonzeros reach outside their block (requires SKB = false).
// One cycle of one system on the G blocks of its grid (or group of blocks);
// blk: this block's logical index among them.  LOOK: the three-barrier SpMV
// loads the next slot's columns ahead (the multi-system instances, at their
// register limit, do without: measured slower with it).
template <int R, int KW, int BLOCK, bool SKB, typename TC, typename TS, bool HALO, bool LOOK = true>
__device__ __forceinline__ void arnoldi_body(const ArnoldiParams& p, const int G, const int blk) {
    extern __shared__ double smem[];
    constexpr int NW = BLOCK / kWave;
    constexpr int RB = R * BLOCK;  // rows per block
    const int s = p.s;
    const int zeta = p.zeta;
    const int64_t n = p.n;
    // LDS: vals (2 RB doubles; the raw pattern, then the list-ordering bitmaps,
    //      at init) | reduction scratch | coefficients | list starts (s+1) |
    //      list lengths (s, one spare) | lists (zeta RB + 3s, groups of four)
    double* vals = smem;
    double* red_tmp = vals + arnoldi_vals_doubles(RB, zeta);
    double* red_out = red_tmp + NW * kRedSlots;
    double* coef = red_out + kRedSlots;  // [0] <m,m>, [1..k] h ; [k+1] <w,w>, [k+2..2k+1] h2 ; [2k+2] nu
    int* lstart = reinterpret_cast<int*>(coef + 2 * p.k + 3);
    int* lcount = lstart + (s + 1);
    uint16_t* lists = reinterpret_cast<uint16_t*>(lcount + s + 1);  // 8-byte aligned (2s + 2 ints)
    __shared__ unsigned sync_lds[3];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    const int64_t base = static_cast<int64_t>(blk) * RB + tid;
    const double scale = 1.0 / sqrt(static_cast<double>(zeta));
    const int64_t slab = static_cast<int64_t>(2 * s) * G;  // sketch partials of one step
    const TC* Av = static_cast<const TC*>(p.val);
    TS* Bs = static_cast<TS*>(p.B);
    constexpr double uround = BasisPrec<TC>::unit_roundoff;
    static_assert(!HALO || !SKB, "the halo mode keeps b_{j+1} where S b_j would be staged");
    TC* bst = reinterpret_cast<TC*>(vals);  // HALO: own rows of the current column
    constexpr bool kPub = sizeof(TC) == 4;  // HALO: publish (else recompute) halo entries
    TC* wbuf = static_cast<TC*>(p.hbuf);
    unsigned long long* pub = static_cast<unsigned long long*>(p.hbuf);
    const int64_t row_lo = static_cast<int64_t>(blk) * RB;
    const int64_t row_hi = min(n, row_lo + RB);
    // A basis column is written once per cycle, before anything reads it, and
    // the launch begins with an acquire.  When columns start on 256-byte
    // boundaries (and blocks own whole cache lines of them, RB being a multiple
    // of 64 rows), no cache line can hold a stale copy of a column's entries:
    // other blocks' rows of B are then read with plain loads, which hit the
    // XCD's L2.  Otherwise a line may straddle two columns and be cached before
    // the later column is written: such reads are device-coherent.
    const bool fresh =
        ((reinterpret_cast<uintptr_t>(p.B) | static_cast<uintptr_t>(p.ldb * sizeof(TS))) & 255u) == 0;
    auto ldB = [&](const TS* q) -> TS { return fresh ? *q : load_coherent(q); };

    GridSync bar{static_cast<SyncWords*>(p.sync), p.abort, p.spin_limit, static_cast<unsigned>(G), 0u, 0u, 0u, 0u, 0u,
                 p.per_block_release != 0};
    bar.setup(sync_lds);

    // ---- sliced ELL position of own rows, held for the cycle ------------------
    // the 64 rows of this wavefront in chunk r form one slice: entry k of this
    // lane's row is at spos[r] + 64 k + lane, for k < sK[r].  Both are the same
    // for the whole wavefront and live in scalar registers.
    int64_t spos[R];
    int sK[R];
    {
        const int64_t nsl = (n + kWave - 1) / kWave;
        const int wid_s = __builtin_amdgcn_readfirstlane(wid);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t sl = (static_cast<int64_t>(blk) * RB + static_cast<int64_t>(r) * BLOCK) / kWave + wid_s;
            spos[r] = 0;
            sK[r] = 0;
            if (sl < nsl) {
                const int64_t a = p.sp[sl];
                spos[r] = a;
                sK[r] = static_cast<int>((p.sp[sl + 1] - a) / kWave);
            }
        }
    }

    // HALO: bit r set when own row r is gathered by another block
    unsigned xmask = 0;
    if constexpr (HALO) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
            if (row < n && ((p.xbits[row >> 5] >> (row & 31)) & 1u)) xmask |= 1u << r;
        }
    }

    // Halo mode: nonzero slot q of the wavefront's 64 rows of chunk r whose
    // column is the row plus the same offset in every lane (a diagonal of A
    // across the slice, as in banded and grid operators) keeps that offset in
    // LDS, and the SpMV forms those columns instead of loading them; other
    // slots (and q >= 16) read the column index array.  Found once per cycle
    // from the column indices themselves.
    constexpr int kOffSlots = 16;
    constexpr int kIrregular = INT_MIN;
    __shared__ int hoff[HALO ? NW * R * kOffSlots : 1];
    if constexpr (HALO) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
            // the slots' column loads all in flight, then one vote per slot
            int cs[kOffSlots];
#pragma unroll
            for (int q = 0; q < kOffSlots; ++q)
                cs[q] = q < sK[r] ? p.ci[spos[r] + static_cast<int64_t>(q) * kWave + lane] : 0;
#pragma unroll
            for (int q = 0; q < kOffSlots; ++q) {
                int o = kIrregular;
                if (q < sK[r]) {
                    const int d = cs[q] - static_cast<int>(row);
                    const int d0 = __builtin_amdgcn_readfirstlane(d);
                    if (__all(d == d0)) o = d0;
                }
                if (lane == 0) hoff[(wid * R + r) * kOffSlots + q] = o;
            }
        }
    }

    // ---- sketch lists of the block's rows, sorted by sketch row --------------
    sketch_lists_build<R, BLOCK, true>(p.seed, p.cycle, base, n, s, zeta, reinterpret_cast<uint16_t*>(vals), lstart,
                                 lcount, lists);

    // Block partials of S b_j (vector 0, only when SB is wanted) and S m_j
    // (vector 1) over sketch rows [r0, r1), staged in vals.
    constexpr int sk_v0 = SKB ? 0 : 1;
    constexpr int sk_nv = SKB ? 2 : 1;
    // (no block synchronisation inside: the wavefronts of a block finish their
    // pieces independently, the last one first doing the barrier arrival)
    auto block_sketch = [&](int r0, int r1, double* dst) {
        sketch_lists_apply_lanes<BLOCK>(sk_v0, sk_nv, r0, r1, vals, RB, s, lstart, lcount, lists, dst, G, blk);
    };
    // the thread that counts this block's barrier arrivals: one of the last
    // wavefront, which gets no sketch pieces when a window has at most
    // BLOCK - 64 of them, so the arrival's atomic round trip and the XCD
    // write-back are not in front of any sketch work
    constexpr unsigned kArriver = BLOCK - kWave;
    // the sketch of one step is spread over the barrier windows (three, or two
    // in the halo mode)
    const int sk_cut1 = HALO ? s / 2 : s / 3;
    const int sk_cut2 = HALO ? s : (2 * s) / 3;

    // ---- init: g partial (S r), b_1 = r/|r| ----------------------------------
    const double beta = *p.beta;
    // window entries a = 0 .. KW-1 (0 = newest) of the own rows; in the halo
    // mode the newest one is not held in registers: it is the column staged
    // in LDS for the SpMV's gathers (bst), read from there
    TC win[KW > 0 ? KW : 1][R];
    auto Wr = [&](int a, int r) -> TC {
        if constexpr (HALO) {
            if (a == 0) return bst[r * BLOCK + tid];
        }
        return win[a][r];
    };
#pragma unroll
    for (int a = 0; a < (KW > 0 ? KW : 1); ++a)
#pragma unroll
        for (int r = 0; r < R; ++r) win[a][r] = TC(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
        double rv = 0.0;
        if (row < n) {
            rv = p.r[row];
            const TS b1 = to_basis<TS>(static_cast<TC>(rv / beta));
            Bs[row] = b1;
            win[0][r] = from_basis<TC>(b1);
        }
        vals[r * BLOCK + tid] = rv;
    }
    __syncthreads();
    // g partials after the d step slabs
    sketch_lists_apply_lanes<BLOCK>(0, 1, 0, s, vals, RB, s, lstart, lcount, lists,
                                    p.part_sk + static_cast<int64_t>(p.d) * slab, G, blk);
    bar.sync();  // B[:,0] and the g partials are complete
    if constexpr (HALO) {
#pragma unroll
        for (int r = 0; r < R; ++r) bst[r * BLOCK + tid] = win[0][r];
        __syncthreads();
    }

    // window entry a (0 = newest) of own row r at step j
    auto Wg = [&](int j, int a, int r) -> TC {
        const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
        return row < n ? from_basis<TC>(Bs[static_cast<int64_t>(j - a) * p.ldb + row]) : TC(0);
    };

    // partial sums of <x,x> and W^T x over own rows, handed to put(q, value)
    // by thread q: slot q = 0: <x,x>; slot q = 1 + a: <W_a, x>
    auto dots_to_partials = [&](const TC (&x)[R], int j, int kw, auto put) {
        if constexpr (KW > 0) {
            double v[KW + 1];
            TC t = TC(0);
#pragma unroll
            for (int r = 0; r < R; ++r) t = madd(x[r], x[r], t);
            v[0] = static_cast<double>(t);
#pragma unroll
            for (int a = 0; a < KW; ++a) {
                TC u = TC(0);
#pragma unroll
                for (int r = 0; r < R; ++r) u = madd(Wr(a, r), x[r], u);
                v[a + 1] = static_cast<double>(u);
            }
            // (no closing synchronisation: both callers synchronise the block
            // before red_tmp is written again)
            block_sum_put<KW + 1>(v, kw + 1, red_tmp, put);
        } else {
            for (int q0 = 0; q0 < kw + 1; q0 += kChunk) {
                double v[kChunk];
#pragma unroll
                for (int c = 0; c < kChunk; ++c) {
                    const int q = q0 + c;
                    TC u = TC(0);
                    if (q == 0) {
#pragma unroll
                        for (int r = 0; r < R; ++r) u = madd(x[r], x[r], u);
                    } else if (q <= kw) {
#pragma unroll
                        for (int r = 0; r < R; ++r) u = madd(Wg(j, q - 1, r), x[r], u);
                    }
                    v[c] = static_cast<double>(u);
                }
                const int cnt = min(kChunk, kw + 1 - q0);
                block_sum<kChunk>(v, cnt, red_tmp, red_out);
                if (tid < cnt) put(q0 + tid, red_out[tid]);
            }
        }
    };

    // profiling: block 0 accumulates the real-time ticks spent in each phase
    const bool timing = p.phase_ticks != nullptr && blk == 0 && tid == 0;
    uint64_t t_last = timing ? __builtin_amdgcn_s_memrealtime() : 0;
    auto tick = [&](int k) {
        if (timing) {
            const uint64_t t = __builtin_amdgcn_s_memrealtime();
            p.phase_ticks[k] += t - t_last;
            t_last = t;
        }
    };

    int dc = p.d;
    int flags = 0;
    for (int j = 0; j < p.d; ++j) {
        const TS* bj = Bs + static_cast<int64_t>(j) * p.ldb;
        const int kw = min(j + 1, p.k);

        // ---- phase 1: m = A b_j and partial dots ---------------------------
        // SpMV, nonzero slot outermost: slot q of the R rows is fetched with R
        // independent loads, then R independent gathers (each row still sums
        // its nonzeros in CSR order)
        TC m[R];
#pragma unroll
        for (int r = 0; r < R; ++r) m[r] = TC(0);
        int kmax = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) kmax = max(kmax, sK[r]);
        if constexpr (HALO) {
            // own rows from LDS; other blocks' rows of b_j from their owners'
            // tagged words, or recomputed from w and the window of step j-1
            // (b_1 is in HBM, published at init)
            const unsigned tag_b = static_cast<unsigned>(j);
            const int kwp = min(j, p.k);
            const TC nup = static_cast<TC>(coef[2 * p.k + 2]);
            const double* h2p = coef + p.k + 2;
            const TS* Bp = Bs + static_cast<int64_t>(j > 0 ? j - 1 : 0) * p.ldb;
            // slot q + 1's column and value loads are issued before slot q is
            // consumed, so two slots of loads are in flight (the SpMV is bound
            // by the loads in flight, not by bandwidth: 9.2 against 11.0 us per
            // step at cd1024 in FP32)
            int c[R], cn[R];
            TC v[R], vn[R];
            // column of slot q of chunk r: the row plus the slot's offset, or
            // loaded (the offset is wavefront-uniform)
            auto col_of = [&](int r, int q, int64_t e) -> int {
                const int o =
                    q < kOffSlots ? __builtin_amdgcn_readfirstlane(hoff[(wid * R + r) * kOffSlots + q]) : kIrregular;
                if (o != kIrregular) return static_cast<int>(base + static_cast<int64_t>(r) * BLOCK) + o;
                return p.ci[e];
            };
            auto load_slot = [&](int q, int (&cd)[R], TC (&vd)[R]) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    cd[r] = -1;
                    vd[r] = TC(0);
                    if (q < sK[r]) {
                        const int64_t e = spos[r] + static_cast<int64_t>(q) * kWave + lane;
                        cd[r] = col_of(r, q, e);
                        vd[r] = Av[e];
                    }
                }
            };
            // (FP32 arithmetic only: the FP64 kernel is at its register limit
            // and the extra registers spilled, measured slower overall; it
            // loads slot q + 1's columns only, so that slot q's gathers and
            // value loads wait for one round trip instead of two)
            constexpr bool kLook = sizeof(TC) < 8;
            auto load_cols = [&](int q, int (&cd)[R]) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    cd[r] = -1;
                    if (q < sK[r]) cd[r] = col_of(r, q, spos[r] + static_cast<int64_t>(q) * kWave + lane);
                }
            };
            if constexpr (kLook) load_slot(0, c, v);
            else load_cols(0, c);
            for (int q = 0; q < kmax; ++q) {
                if constexpr (kLook) {
                    load_slot(q + 1, cn, vn);
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        v[r] = TC(0);
                        if (q < sK[r]) v[r] = Av[spos[r] + static_cast<int64_t>(q) * kWave + lane];
                    }
                    load_cols(q + 1, cn);
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (q < sK[r]) {
                        const int cc = c[r];
                        TC bv;
                        if (cc >= row_lo && cc < row_hi) {
                            bv = bst[cc - row_lo];
                        } else if (j == 0) {
                            bv = from_basis<TC>(load_coherent(bj + cc));
                        } else if constexpr (kPub) {
                            bv = tagged_get(pub + cc, tag_b, p.abort, p.spin_limit);
                        } else {
                            // w is rewritten every step: read device-coherently; the
                            // window columns as described at ldB.  The first four
                            // window loads are issued together (addresses clamped
                            // into valid columns), then consumed in order.
                            TC t = load_coherent(wbuf + cc);
                            TS wa[4];
#pragma unroll
                            for (int a = 0; a < 4; ++a) wa[a] = ldB(Bp + cc - static_cast<int64_t>(min(a, kwp - 1)) * p.ldb);
#pragma unroll
                            for (int a = 0; a < 4; ++a)
                                if (a < kwp) t = gs_sub(t, static_cast<TC>(h2p[a]), from_basis<TC>(wa[a]));
                            for (int a = 4; a < kwp; ++a)
                                t = gs_sub(t, static_cast<TC>(h2p[a]),
                                           from_basis<TC>(ldB(Bp + cc - static_cast<int64_t>(a) * p.ldb)));
                            bv = from_basis<TC>(to_basis<TS>(t / nup));
                        }
                        m[r] = madd(v[r], bv, m[r]);
                    }
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    c[r] = cn[r];
                    if constexpr (kLook) v[r] = vn[r];
                }
            }
        } else {
            // with LOOK, slot q + 1's columns are loaded while slot q's values
            // and gathers are in flight, so each slot waits for one round trip
            // (its gathers need its columns) instead of two (rd1m FP64:
            // 6.77 -> 6.25 ms per launch)
            int c[R], cn[R];
            auto load_cols = [&](int q, int (&cd)[R]) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    cd[r] = 0;
                    if (q < sK[r]) cd[r] = p.ci[spos[r] + static_cast<int64_t>(q) * kWave + lane];
                }
            };
            if constexpr (LOOK) load_cols(0, c);
            for (int q = 0; q < kmax; ++q) {
                TC v[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if constexpr (!LOOK) c[r] = 0;
                    v[r] = TC(0);
                    if (q < sK[r]) {
                        const int64_t e = spos[r] + static_cast<int64_t>(q) * kWave + lane;
                        if constexpr (!LOOK) c[r] = p.ci[e];
                        v[r] = Av[e];
                    }
                }
                if constexpr (LOOK) load_cols(q + 1, cn);
                // own rows of b_j were stored by this block; other blocks' rows
                // as described at ldB (the per-step barriers take no acquire)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (q < sK[r]) {
                        const int cc = c[r];
                        const TS bv = (cc >= row_lo && cc < row_hi) ? bj[cc] : ldB(bj + cc);
                        m[r] = madd(v[r], from_basis<TC>(bv), m[r]);
                    }
                if constexpr (LOOK) {
#pragma unroll
                    for (int r = 0; r < R; ++r) c[r] = cn[r];
                }
            }
        }
        // the first reduction of the step goes through tagged partials (tag
        // j + 1) instead of a grid barrier: nothing else written before it is
        // read by other blocks before the second barrier
        const unsigned tag_a = static_cast<unsigned>(j + 1);
        dots_to_partials(m, j, kw, [&](int q, double val) {
            tagged_store(p.part_a + 2 * (static_cast<int64_t>(q) * G + blk), val, tag_a);
        });
        // stage b_j and m_j for the sketch
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (SKB) {
                TC bv;
                if constexpr (KW > 0) bv = win[0][r];
                else bv = Wg(j, 0, r);
                vals[r * BLOCK + tid] = static_cast<double>(bv);
            }
            vals[RB + r * BLOCK + tid] = static_cast<double>(m[r]);
        }
        __syncthreads();
        tick(0);
        // block sketch partials of b_j and m_j, first third, while the other
        // blocks' partials arrive
        double* sk_dst = p.part_sk + static_cast<int64_t>(j) * slab;
        block_sketch(0, sk_cut1, sk_dst);
        tick(1);

        // ---- phase 2: h, w = m - W h, partial dots ------------------------
        grid_sum_tagged(p.part_a, G, kw + 1, tag_a, coef, p.abort, p.spin_limit);  // coef[0] = <m,m>, coef[1+a] = h_a
        tick(2);
        if (j == p.d - 1) {
            block_sketch(sk_cut1, s, sk_dst);
            break;
        }
        TC w[R];
#pragma unroll
        for (int r = 0; r < R; ++r) w[r] = m[r];
        if constexpr (KW > 0) {
#pragma unroll
            for (int a = 0; a < KW; ++a) {
                if (a < kw) {
                    const TC h = static_cast<TC>(coef[1 + a]);
#pragma unroll
                    for (int r = 0; r < R; ++r) w[r] = gs_sub(w[r], h, Wr(a, r));
                }
            }
        } else {
            for (int a = 0; a < kw; ++a) {
                const TC h = static_cast<TC>(coef[1 + a]);
#pragma unroll
                for (int r = 0; r < R; ++r) w[r] = gs_sub(w[r], h, Wg(j, a, r));
            }
        }
        if constexpr (HALO && !kPub) {
            // only the rows other blocks gather
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
                if ((xmask >> r) & 1u) store_stream(wbuf + row, w[r]);
            }
        }
        // tagged as well: the second barrier still orders w and the basis
        // columns, but its partials are loaded while the barrier is polled
        dots_to_partials(w, j, kw, [&](int q, double val) {
            tagged_store(p.part_b + 2 * (static_cast<int64_t>(q) * G + blk), val, tag_a);
        });
        tick(3);
        bar.arrive(kArriver);
        block_sketch(sk_cut1, sk_cut2, sk_dst);  // second third
        // wavefront 0 polls the barrier while the others load the partials
        double* c2 = coef + p.k + 1;
        bar.spin_flags();
        grid_sum_tagged(p.part_b, G, kw + 1, tag_a, c2, p.abort, p.spin_limit, 1);  // c2[0] = <w,w>, c2[1+a] = h2_a
        tick(4);

        // ---- phase 3: h2, nu, b_{j+1} -------------------------------------
        double h2sq = 0.0;
        for (int a = 0; a < kw; ++a) h2sq = madd(c2[1 + a], c2[1 + a], h2sq);
        const double nu2 = c2[0] - h2sq;
        const double mm = coef[0];
        const bool breakdown = !(nu2 > 16.0 * uround * uround * mm);
        const double nu = breakdown ? 0.0 : sqrt(nu2);
        if (blk == 0 && tid <= p.k) {
            double hv;
            if (tid == p.k) hv = nu;
            else if (tid < kw) hv = coef[1 + tid] + c2[1 + tid];
            else hv = 0.0;
            p.H[static_cast<int64_t>(j) * (p.k + 1) + tid] = hv;
        }
        if (breakdown) {
            if constexpr (!HALO) block_sketch(sk_cut2, s, sk_dst);
            dc = j + 1;
            flags |= SGMRES_FLAG_BREAKDOWN;
            break;
        }
        TS* bn = Bs + static_cast<int64_t>(j + 1) * p.ldb;
        TC bnew[R];
#pragma unroll
        for (int r = 0; r < R; ++r) bnew[r] = w[r];
        if constexpr (KW > 0) {
#pragma unroll
            for (int a = 0; a < KW; ++a) {
                if (a < kw) {
                    const TC h = static_cast<TC>(c2[1 + a]);
#pragma unroll
                    for (int r = 0; r < R; ++r) bnew[r] = gs_sub(bnew[r], h, Wr(a, r));
                }
            }
        } else {
            for (int a = 0; a < kw; ++a) {
                const TC h = static_cast<TC>(c2[1 + a]);
#pragma unroll
                for (int r = 0; r < R; ++r) bnew[r] = gs_sub(bnew[r], h, Wg(j, a, r));
            }
        }
        const TC nu_t = static_cast<TC>(nu);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
            const TS st = to_basis<TS>(bnew[r] / nu_t);
            bnew[r] = from_basis<TC>(st);
            if (row < n) {
                // the halo mode gathers own rows from LDS and other blocks'
                // through the halo buffer: nothing rereads the column from L2
                // in the next step
                if constexpr (HALO) {
                    store_stream(bn + row, st);
                    if constexpr (kPub)
                        if ((xmask >> r) & 1u) tagged_put(pub + row, bnew[r], static_cast<unsigned>(j + 1));
                } else {
                    bn[row] = st;
                }
            }
        }
        if constexpr (KW > 0) {
#pragma unroll
            for (int a = KW - 1; a > 0; --a)
#pragma unroll
                for (int r = 0; r < R; ++r) win[a][r] = Wr(a - 1, r);
#pragma unroll
            for (int r = 0; r < R; ++r)
                if constexpr (!HALO) win[0][r] = bnew[r];  // the halo mode stages it in LDS below
        }
        tick(5);
        if constexpr (HALO) {
            // no third barrier: stage the own rows of b_{j+1}; keep nu for the
            // recomputation of other blocks' rows in the next step
#pragma unroll
            for (int r = 0; r < R; ++r) bst[r * BLOCK + tid] = bnew[r];
            if (!kPub && tid == 0) coef[2 * p.k + 2] = nu;
            __syncthreads();
        } else {
            bar.arrive(kArriver);
            block_sketch(sk_cut2, s, sk_dst);  // last third
            bar.wait_relaxed();
        }
        tick(6);
    }

    // ---- end of cycle: sum the block sketch partials across blocks ----------
    bar.sync();  // the last step's partials were written after its arrival
    {
        // entries: per step the wanted sketch rows (S b_j then S m_j, or S m_j
        // only), then g
        constexpr int nsl_mul = SKB ? 2 : 1;
        const int nsl = nsl_mul * s;
        const int off = SKB ? 0 : s;
        const int64_t E = static_cast<int64_t>(nsl) * dc + s;
        const int64_t per = (E + G - 1) / G;
        const int64_t e0 = static_cast<int64_t>(blk) * per;
        const int64_t e1 = min(E, e0 + per);
        for (int64_t e = e0 + wid; e < e1; e += NW) {
            const int64_t jj = e / nsl;  // == dc for the g entries
            const int ee = static_cast<int>(e - jj * nsl) + (jj < dc ? off : 0);
            const double* col = (jj < dc) ? p.part_sk + jj * slab + static_cast<int64_t>(ee) * G
                                          : p.part_sk + static_cast<int64_t>(p.d) * slab + static_cast<int64_t>(ee) * G;
            double t = lane_strided_sum(col, G, lane);
            t = wave_sum(t) * scale;
            if (lane == 0) {
                if (jj == dc) p.g[ee] = t;
                else if (ee < s) p.SB[jj * s + ee] = t;
                else p.SAB[jj * s + (ee - s)] = t;
            }
        }
    }
    tick(7);
    if (blk == 0 && tid == 0) {
        p.status[0] = dc;
        p.status[1] |= flags;
    }
}

template <int R, int KW, int BLOCK, bool SKB, typename TC, typename TS, bool HALO = false>
__global__ __launch_bounds__(BLOCK) void arnoldi_kernel(ArnoldiParams p) {
    arnoldi_body<R, KW, BLOCK, SKB, TC, TS, HALO>(p, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
}

// Several independent systems in one cooperative launch (the batched solve):
// logical block lb belongs to group grp[lb] (-1: idle padding), and group g
// runs one cycle of the system described by ps[g] on its ps[g].G blocks, the
// logical blocks [ps[g].blk0, ps[g].blk0 + ps[g].G), which the XCD-aware
// numbering keeps on as few XCDs as possible.  Each group has its own grid
// barrier words, partial sums and status; groups never wait for each other.
// LOOK: the SpMV loads the next slot's columns ahead (where it fits in the
// registers without a spill).
template <int R, int KW, int BLOCK, typename TC, typename TS, bool LOOK>
__global__ __launch_bounds__(BLOCK) void arnoldi_multi_kernel(const ArnoldiParams* __restrict__ ps,
                                                              const int* __restrict__ grp) {
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int g = __builtin_amdgcn_readfirstlane(grp[lb]);
    if (g < 0) return;
    const ArnoldiParams& p = ps[g];
    arnoldi_body<R, KW, BLOCK, false, TC, TS, false, LOOK>(p, p.G, lb - p.blk0);
}

// Kernel instance for (BLOCK, R, KW); (R, KW) = (8, 8) is never selected
// (the register window is capped at 32 doubles per thread).
template <bool SKB, typename TC, typename TS, int BLOCK, bool HALO>
const void* pick_rows(int R, int KW) {
#define SG_CASE(RR, KK) \
    if (R == RR && KW == KK) return reinterpret_cast<const void*>(arnoldi_kernel<RR, KK, BLOCK, SKB, TC, TS, HALO>);
    SG_CASE(1, 0) SG_CASE(1, 4) SG_CASE(1, 8)
    SG_CASE(2, 0) SG_CASE(2, 4) SG_CASE(2, 8)
    SG_CASE(4, 0) SG_CASE(4, 4) SG_CASE(4, 8)
    SG_CASE(8, 0) SG_CASE(8, 4)
#undef SG_CASE
    return nullptr;
}

template <bool SKB, typename TC, typename TS, bool HALO = false>
const void* arnoldi_pick(int block, int R, int KW) {
    switch (block) {
        case 256: return pick_rows<SKB, TC, TS, 256, HALO>(R, KW);
        case 512: return pick_rows<SKB, TC, TS, 512, HALO>(R, KW);
        case 1024: return pick_rows<SKB, TC, TS, 1024, HALO>(R, KW);
        default: return nullptr;
    }
}

}  // namespace arnoldi_detail
}  // namespace sg
