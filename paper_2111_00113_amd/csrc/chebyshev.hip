// Chebyshev basis cycle: the shifted-and-scaled Chebyshev recurrence of
// arXiv:2111.00113 Section 4.4 (equation for b_j, j >= 3, with the starting
// vectors b_1 = r/|r|, b_2 = (A - cI) b_1 / (2 rho)), fused with SpMV (on the
// sliced ELL copy of A, sell.hip) and sparse-sign sketching in one persistent
// cooperative launch.
//
// The recurrence has no inner products, so a step needs one grid barrier (the
// new column must be complete before any block gathers it for the next SpMV)
// and no grid reduction.  The paper rescales every column to unit norm after
// its use in the recurrence; here the norms are accumulated as block partials
// during the cycle and applied to the sketched columns at the end, so B holds
// the raw recurrence vectors and `colnorm` their norms.  The raw vectors are
// bt_j = kappa^(j-1) b_j with kappa = 2 rho / (dx + dy): a constant rescale per
// step (removed again by the normalisation) that keeps |bt_j| near |r|/|r| when
// the box encloses the spectrum, instead of decaying like 2^(1-j) for an
// interval.
//
// Per step j (row state in registers: bt_{j-1}, bt_j):
//   m = A bt_j;  bt_{j+1} = a (m - c bt_j) - q bt_{j-1} -> B[:, j+1];
//   stage m (and bt_j) in LDS, wavefront sums of |bt_j|^2           -- arrive --
//   block partials: |bt_j|^2, S m (and S bt_j when SB is wanted)     -- wait --
// End of cycle: block u reduces column u's norm, then its sketch entries
// scaled by 1/(sqrt(zeta) |bt_u|); the last unit is g = S r.
#include "common.hpp"
#include "internal.hpp"

namespace sg {

namespace {

// TC: per-row arithmetic type; TS: storage type of B (see BasisPrec).
template <int R, int BLOCK, typename TC, typename TS>
__global__ __launch_bounds__(BLOCK) void chebyshev_kernel(ChebParams p) {
    extern __shared__ double smem[];
    constexpr int NW = BLOCK / kWave;
    constexpr int RB = R * BLOCK;
    const int s = p.s;
    const int zeta = p.zeta;
    const int64_t n = p.n;
    // LDS: vals (2 RB doubles; raw pattern and list-ordering bitmaps at init)
    //      | wavefront norm sums (NW) | list starts (s+1) | list lengths (s, one
    //      spare) | lists (zeta RB + 3s, groups of four)
    double* vals = smem;
    double* red_tmp = vals + arnoldi_vals_doubles(RB, zeta);
    int* lstart = reinterpret_cast<int*>(red_tmp + NW);
    int* lcount = lstart + (s + 1);
    uint16_t* lists = reinterpret_cast<uint16_t*>(lcount + s + 1);  // 8-byte aligned (2s + 2 ints)
    __shared__ unsigned sync_lds[3];
    __shared__ double unit_scale;

    const int G = gridDim.x;
    const int blk = xcd_logical_block(blockIdx.x, G);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    const int64_t base = static_cast<int64_t>(blk) * RB + tid;
    const double scale = 1.0 / sqrt(static_cast<double>(zeta));
    const int64_t slab = static_cast<int64_t>(2 * s) * G;
    const TC* Av = static_cast<const TC*>(p.val);
    TS* Bs = static_cast<TS*>(p.B);
    const TC cc = static_cast<TC>(p.c);
    const bool fresh =
        ((reinterpret_cast<uintptr_t>(p.B) | static_cast<uintptr_t>(p.ldb * sizeof(TS))) & 255u) == 0;

    GridSync bar{static_cast<SyncWords*>(p.sync), p.abort, p.spin_limit, static_cast<unsigned>(G), 0u, 0u, 0u, 0u, 0u,
                 p.per_block_release != 0};
    bar.setup(sync_lds);

    // sliced ELL position of own rows (see sell.hip): entry k of this lane's
    // row in chunk r is at spos[r] + 64 k + lane, for k < sK[r]; both are the
    // same for the whole wavefront and live in scalar registers
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
    // nonzero slot q of the wavefront's 64 rows of chunk r whose column is the
    // row plus the same offset in every lane keeps that offset in LDS; the
    // SpMV forms those columns instead of loading them (found once per cycle)
    constexpr int kOffSlots = 16;
    constexpr int kIrregular = INT_MIN;
    __shared__ int soff[NW * R * kOffSlots];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
        for (int q = 0; q < kOffSlots; ++q) {
            int o = kIrregular;
            if (q < sK[r]) {
                const int d = p.ci[spos[r] + static_cast<int64_t>(q) * kWave + lane] - static_cast<int>(row);
                const int d0 = __builtin_amdgcn_readfirstlane(d);
                if (__all(d == d0)) o = d0;
            }
            if (lane == 0) soff[(wid * R + r) * kOffSlots + q] = o;
        }
    }
    sketch_lists_build<R, BLOCK, true>(p.seed, p.cycle, base, n, s, zeta, reinterpret_cast<uint16_t*>(vals), lstart,
                                 lcount, lists);

    const int sk_v0 = p.sketch_basis ? 0 : 1;
    const int sk_nv = p.sketch_basis ? 2 : 1;

    // ---- init: g partial (S r), bt_1 = r/|r| ---------------------------------
    const double beta = *p.beta;
    TC bprev[R], bcur[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
        double rv = 0.0;
        bprev[r] = TC(0);
        bcur[r] = TC(0);
        if (row < n) {
            rv = p.r[row];
            const TS st = to_basis<TS>(static_cast<TC>(rv / beta));
            Bs[row] = st;
            bcur[r] = from_basis<TC>(st);
        }
        vals[r * BLOCK + tid] = rv;
    }
    __syncthreads();
    sketch_lists_apply_lanes<BLOCK>(0, 1, 0, s, vals, RB, s, lstart, lcount, lists, p.part_sk + static_cast<int64_t>(p.d) * slab,
                                    G, blk);
    bar.sync();
    // the thread that counts this block's barrier arrivals (the last
    // wavefront's first lane); the other wavefronts start the step's sketch
    // at once, without waiting for its atomic round trip
    constexpr unsigned kArriver = BLOCK - kWave;
    // When only S m is sketched, the first half of vals is free: it holds the
    // block's own rows of the current column (as TC), and the SpMV gathers
    // those from LDS; other blocks' rows come from B.
    const bool lds_b = !p.sketch_basis;
    TC* bst = reinterpret_cast<TC*>(vals);
    const int64_t row_lo = static_cast<int64_t>(blk) * RB;
    const int64_t row_hi = min(n, row_lo + RB);
    if (lds_b) {
#pragma unroll
        for (int r = 0; r < R; ++r) bst[r * BLOCK + tid] = bcur[r];
    }
    __syncthreads();

    const bool timing = p.phase_ticks != nullptr && blk == 0 && tid == 0;
    uint64_t t_last = timing ? __builtin_amdgcn_s_memrealtime() : 0;
    auto tick = [&](int k) {
        if (timing) {
            const uint64_t t = __builtin_amdgcn_s_memrealtime();
            p.phase_ticks[k] += t - t_last;
            t_last = t;
        }
    };

    for (int j = 0; j < p.d; ++j) {
        const TS* bj = Bs + static_cast<int64_t>(j) * p.ldb;
        // SpMV, nonzero slot outermost (R independent loads, then R gathers per
        // slot; each row sums its nonzeros in CSR order)
        TC m[R];
        int kmax = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            m[r] = TC(0);
            kmax = max(kmax, sK[r]);
        }
        // slot q + 1's column and value loads are issued before slot q is
        // consumed: two slots of loads in flight
        int c[R], cn[R];
        TC v[R], vn[R];
        auto load_slot = [&](int q, int (&cd)[R], TC (&vd)[R]) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cd[r] = 0;
                vd[r] = TC(0);
                if (q < sK[r]) {
                    const int64_t e = spos[r] + static_cast<int64_t>(q) * kWave + lane;
                    const int o = q < kOffSlots ? __builtin_amdgcn_readfirstlane(soff[(wid * R + r) * kOffSlots + q])
                                                : kIrregular;
                    cd[r] = o != kIrregular ? static_cast<int>(base + static_cast<int64_t>(r) * BLOCK) + o : p.ci[e];
                    vd[r] = Av[e];
                }
            }
        };
        load_slot(0, c, v);
        for (int q = 0; q < kmax; ++q) {
            load_slot(q + 1, cn, vn);
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (q < sK[r]) {
                    const int cc = c[r];
                    const TC bv = (lds_b && cc >= row_lo && cc < row_hi) ? bst[cc - row_lo] : from_basis<TC>(bj[cc]);
                    m[r] = madd(v[r], bv, m[r]);
                }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                c[r] = cn[r];
                v[r] = vn[r];
            }
        }
        const bool more = j + 1 < p.d;
        TC bnext[R];
        if (more) {
            const TC a = static_cast<TC>((j == 0) ? p.a1 : p.a);
            const TC q = static_cast<TC>((j == 0) ? 0.0 : p.q);
            TS* bn = Bs + static_cast<int64_t>(j + 1) * p.ldb;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
                const TS st = to_basis<TS>(madd(a, madd(-cc, bcur[r], m[r]), -(q * bprev[r])));
                if (row < n) bn[row] = st;
                bnext[r] = from_basis<TC>(st);
            }
        }
        // partials of this step while the barrier completes: the block's
        // |bt_j|^2 (wavefront sums, then their sum in wavefront order) and
        // the sketch of m_j (and bt_j), staged in LDS before the arrival,
        // whose block synchronisation publishes them
        double nn = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double bc = static_cast<double>(bcur[r]);
            nn = madd(bc, bc, nn);
            if (p.sketch_basis) vals[r * BLOCK + tid] = bc;
            vals[RB + r * BLOCK + tid] = static_cast<double>(m[r]);
        }
        nn = wave_sum(nn);
        if (lane == 0) red_tmp[wid] = nn;
        tick(0);
        if (more) bar.arrive(kArriver);
        else __syncthreads();
        // every SpMV of the block is done with column j: stage column j + 1
        // (published by the wait's block synchronisation)
        if (lds_b && more) {
#pragma unroll
            for (int r = 0; r < R; ++r) bst[r * BLOCK + tid] = bnext[r];
        }
        if (tid == 0) {
            double acc = 0.0;
            for (int q = 0; q < NW; ++q) acc += red_tmp[q];
            p.part_nrm[static_cast<int64_t>(j) * G + blk] = acc;
        }
        sketch_lists_apply_lanes<BLOCK>(sk_v0, sk_nv, 0, s, vals, RB, s, lstart, lcount, lists,
                                        p.part_sk + static_cast<int64_t>(j) * slab, G, blk);
        tick(1);
        if (more) {
            // no acquire when the columns start on 256-byte boundaries: the
            // next SpMV gathers column j + 1, written once per cycle before
            // anything reads it (the launch began with an acquire), and no cache
            // line then spans two columns, so none can hold a stale copy
            if (fresh) bar.wait_relaxed();
            else bar.wait();
            tick(2);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                bprev[r] = bcur[r];
                bcur[r] = bnext[r];
            }
        }
    }

    // ---- end of cycle: normalise and sum the sketch partials across blocks ---
    bar.sync();
    const int nsl = p.sketch_basis ? 2 * s : s;
    const int off = p.sketch_basis ? 0 : s;
    for (int u = blk; u <= p.d; u += G) {
        if (u < p.d) {
            if (wid == 0) {
                const double* col = p.part_nrm + static_cast<int64_t>(u) * G;
                double t = lane_strided_sum(col, G, lane);
                t = wave_sum(t);
                if (lane == 0) {
                    const double nrm = sqrt(t);
                    p.colnorm[u] = nrm;
                    unit_scale = nrm > 0.0 ? scale / nrm : 0.0;
                }
            }
        } else if (tid == 0) {
            unit_scale = scale;
        }
        __syncthreads();
        const double us = unit_scale;
        const int ne = (u < p.d) ? nsl : s;
        for (int e = wid; e < ne; e += NW) {
            const int ee = (u < p.d) ? e + off : e;
            const double* col = p.part_sk + static_cast<int64_t>(u) * slab + static_cast<int64_t>(ee) * G;
            double t = lane_strided_sum(col, G, lane);
            t = wave_sum(t) * us;
            if (lane == 0) {
                if (u == p.d) p.g[ee] = t;
                else if (ee < s) p.SB[static_cast<int64_t>(u) * s + ee] = t;
                else p.SAB[static_cast<int64_t>(u) * s + (ee - s)] = t;
            }
        }
        __syncthreads();
    }
    tick(7);
    if (blk == 0 && tid == 0) p.status[0] = p.d;
}

using KernelFn = void (*)(ChebParams);

template <int BLOCK, typename TC, typename TS>
KernelFn pick(int R) {
    switch (R) {
        case 1: return chebyshev_kernel<1, BLOCK, TC, TS>;
        case 2: return chebyshev_kernel<2, BLOCK, TC, TS>;
        case 4: return chebyshev_kernel<4, BLOCK, TC, TS>;
        case 8: return chebyshev_kernel<8, BLOCK, TC, TS>;
        default: return nullptr;
    }
}

template <typename TC, typename TS>
KernelFn pick_block(int block, int R) {
    switch (block) {
        case 256: return pick<256, TC, TS>(R);
        case 512: return pick<512, TC, TS>(R);
        case 1024: return pick<1024, TC, TS>(R);
        default: return nullptr;
    }
}

KernelFn pick_kernel(int block, int R, int precision) {
    switch (precision) {
        case SGMRES_PREC_FP64: return pick_block<double, double>(block, R);
        case SGMRES_PREC_FP32: return pick_block<float, float>(block, R);
        case SGMRES_PREC_BF16_BASIS: return pick_block<float, bf16_t>(block, R);
        default: return nullptr;
    }
}

}  // namespace

size_t chebyshev_lds_bytes(int block, int R, int s, int zeta) {
    const int nw = block / kWave;
    const int RB = R * block;
    return sizeof(double) * static_cast<size_t>(arnoldi_vals_doubles(RB, zeta) + nw) +
           sizeof(int) * static_cast<size_t>(2 * s + 2) +
           sizeof(uint16_t) * static_cast<size_t>(sketch_lists_len(zeta * RB, s, true));
}

hipError_t chebyshev_configure(const ArnoldiShape& shape, ArnoldiLaunch* out) {
    int device = 0;
    hipError_t err = hipGetDevice(&device);
    if (err != hipSuccess) return err;
    int cus = 0;
    err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (err != hipSuccess) return err;
    int lds_max = 0;
    err = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (err != hipSuccess) return err;
    const int blocks_try[3] = {1024, 512, 256};
    const int rows_try[4] = {1, 2, 4, 8};
    for (int bi = 0; bi < 3; ++bi) {
        const int block = blocks_try[bi];
        if (shape.block && block != shape.block) continue;
        for (int ri = 0; ri < 4; ++ri) {
            const int R = rows_try[ri];
            if (shape.rows_per_thread && R != shape.rows_per_thread) continue;
            const size_t lds = chebyshev_lds_bytes(block, R, shape.s, shape.zeta);
            if (lds > static_cast<size_t>(lds_max)) continue;
            KernelFn fn = pick_kernel(block, R, shape.precision);
            if (!fn) continue;
            err = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      static_cast<int>(lds));
            if (err != hipSuccess) continue;
            int per_cu = 0;
            err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn), block, lds);
            if (err != hipSuccess || per_cu < 1) continue;
            const int64_t need = (shape.n + static_cast<int64_t>(R) * block - 1) / (static_cast<int64_t>(R) * block);
            if (need > static_cast<int64_t>(per_cu) * cus) continue;
            out->fn = reinterpret_cast<const void*>(fn);
            out->block = block;
            out->R = R;
            out->KW = 0;
            out->grid = static_cast<int>(need);
            out->lds = lds;
            return hipSuccess;
        }
    }
    return hipErrorInvalidValue;
}

hipError_t chebyshev_launch(const ArnoldiLaunch& L, ChebParams params, hipStream_t stream) {
    void* args[] = {&params};
    return hipLaunchCooperativeKernel(L.fn, dim3(L.grid), dim3(L.block), args, static_cast<unsigned>(L.lds), stream);
}

}  // namespace sg
