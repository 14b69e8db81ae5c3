// spmv_truncarnoldi: one cycle of k-truncated Arnoldi basis generation fused
// with CSR SpMV and sparse-sign sketching, as a single persistent cooperative
// launch (arXiv:2111.00113, Algorithm 1 basis loop; truncated-Arnoldi
// recurrence of Section 1.2.2; two classical Gram-Schmidt passes).
//
// Work decomposition.  Logical block b owns rows [b*R*BLOCK, (b+1)*R*BLOCK);
// thread t of it owns rows b*R*BLOCK + r*BLOCK + t, r < R (coalesced across
// lanes).  Everything a row needs between steps stays on chip: the last KW
// basis entries of its rows (registers), m_j = A b_j and w (registers) and the
// row's sketch column (LDS, generated once per cycle).  Per step the kernel
// moves A, the gathered b_j and the written b_{j+1} through HBM, plus a few
// kilobytes of per-block partial sums.
//
// Per step j (three grid barriers, each carrying a reduction):
//   phase 1  m = A b_j; scatter S b_j, S m into LDS; partial <m,m>, W^T m
//            -- barrier --
//   phase 2  h = W^T m (grid sum); w = m - W h; partial <w,w>, W^T w;
//            column j of SB / SAB (and g at j = 0) summed from block partials
//            -- barrier --
//   phase 3  h2 = W^T w; |w - W h2|^2 = <w,w> - |h2|^2 (window orthonormal to
//            rounding); b_{j+1} = (w - W h2)/nu; H column j
//            -- barrier --
#include "common.hpp"
#include "internal.hpp"

namespace sg {

namespace {

constexpr int kChunk = 8;     // reduction values per block_sum pass (global window)
constexpr int kRedSlots = 9;  // max values per block_sum: window of 8 plus a norm

template <int R, int KW, int BLOCK>
__global__ __launch_bounds__(BLOCK) void arnoldi_kernel(ArnoldiParams p) {
    extern __shared__ double smem[];
    constexpr int NW = BLOCK / kWave;
    const int s = p.s;
    const int zeta = p.zeta;
    const int64_t n = p.n;
    double* acc = smem;                         // 2s: SB / SAB accumulators (g at init)
    double* red_tmp = acc + 2 * s;              // NW * kRedSlots
    double* red_out = red_tmp + NW * kRedSlots; // kRedSlots
    double* coef = red_out + kRedSlots;         // [0] <m,m>, [1..k] h ; [k+1] <w,w>, [k+2..2k+1] h2
    uint16_t* pat = reinterpret_cast<uint16_t*>(coef + 2 * p.k + 2);  // zeta x (R*BLOCK)
    const int pstride = R * BLOCK;

    const int G = gridDim.x;
    const int blk = xcd_logical_block(blockIdx.x, G);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    const int64_t base = static_cast<int64_t>(blk) * R * BLOCK + tid;
    GridBarrier bar{p.bar_count, p.abort, static_cast<unsigned>(G), 0u, p.spin_limit};
    const double scale = 1.0 / sqrt(static_cast<double>(zeta));

    // ---- init: sketch pattern of own rows, b_1 = r/|r|, g partial ----------
    for (int e = tid; e < 2 * s; e += BLOCK) acc[e] = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
        if (row < n) sketch_column(p.seed, p.cycle, row, s, zeta, pat + r * BLOCK + tid, pstride);
    }
    __syncthreads();

    const double beta = *p.beta;
    double win[KW > 0 ? KW : 1][R];
#pragma unroll
    for (int a = 0; a < (KW > 0 ? KW : 1); ++a)
#pragma unroll
        for (int r = 0; r < R; ++r) win[a][r] = 0.0;

#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
        if (row < n) {
            const double rv = p.r[row];
            const double b1 = rv / beta;
            p.B[row] = b1;
            win[0][r] = b1;
            for (int t = 0; t < zeta; ++t) {
                const unsigned e = pat[t * pstride + r * BLOCK + tid];
                atomicAdd(&acc[e >> 1], (e & 1u) ? -rv : rv);
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < s; e += BLOCK) {
        p.part_sk[static_cast<int64_t>(2 * s + e) * G + blk] = acc[e];
        acc[e] = 0.0;
    }
    bar.sync();

    // window entry a (0 = newest) of own row r at step j
    auto Wg = [&](int j, int a, int r) -> double {
        const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
        return row < n ? p.B[static_cast<int64_t>(j - a) * p.ldb + row] : 0.0;
    };

    // partial sums of <x,x> and W^T x over own rows -> part[q*G + blk]
    // slot q = 0: <x,x>; slot q = 1 + a: <W_a, x>
    auto dots_to_partials = [&](const double (&x)[R], int j, int kw, double* part) {
        if constexpr (KW > 0) {
            double v[KW + 1];
            double t = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) t += x[r] * x[r];
            v[0] = t;
#pragma unroll
            for (int a = 0; a < KW; ++a) {
                double u = 0.0;
#pragma unroll
                for (int r = 0; r < R; ++r) u += win[a][r] * x[r];
                v[a + 1] = u;
            }
            block_sum<KW + 1>(v, kw + 1, red_tmp, red_out);
            if (tid <= kw) part[static_cast<int64_t>(tid) * G + blk] = red_out[tid];
        } else {
            for (int q0 = 0; q0 < kw + 1; q0 += kChunk) {
                double v[kChunk];
#pragma unroll
                for (int c = 0; c < kChunk; ++c) {
                    const int q = q0 + c;
                    double u = 0.0;
                    if (q == 0) {
#pragma unroll
                        for (int r = 0; r < R; ++r) u += x[r] * x[r];
                    } else if (q <= kw) {
#pragma unroll
                        for (int r = 0; r < R; ++r) u += Wg(j, q - 1, r) * x[r];
                    }
                    v[c] = u;
                }
                const int cnt = min(kChunk, kw + 1 - q0);
                block_sum<kChunk>(v, cnt, red_tmp, red_out);
                if (tid < cnt) part[static_cast<int64_t>(q0 + tid) * G + blk] = red_out[tid];
            }
        }
    };

    int dc = p.d;
    int flags = 0;
    for (int j = 0; j < p.d; ++j) {
        const double* bj = p.B + static_cast<int64_t>(j) * p.ldb;
        const int kw = min(j + 1, p.k);

        // ---- phase 1: m = A b_j, sketch b_j and m, partial dots ------------
        double m[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
            double am = 0.0;
            if (row < n) {
                const int q1 = p.rp[row + 1];
                for (int q = p.rp[row]; q < q1; ++q) am += p.val[q] * bj[p.ci[q]];
            }
            m[r] = am;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
            if (row < n) {
                double bv;
                if constexpr (KW > 0) bv = win[0][r];
                else bv = bj[row];
                const double mv = m[r];
                for (int t = 0; t < zeta; ++t) {
                    const unsigned e = pat[t * pstride + r * BLOCK + tid];
                    const bool neg = e & 1u;
                    atomicAdd(&acc[e >> 1], neg ? -bv : bv);
                    atomicAdd(&acc[s + (e >> 1)], neg ? -mv : mv);
                }
            }
        }
        dots_to_partials(m, j, kw, p.part_a);
        __syncthreads();
        for (int e = tid; e < 2 * s; e += BLOCK) {
            p.part_sk[static_cast<int64_t>(e) * G + blk] = acc[e];
            acc[e] = 0.0;
        }
        bar.sync();

        // ---- phase 2: h, w = m - W h, partial dots; sketch column j -------
        grid_sum(p.part_a, G, kw + 1, coef);  // coef[0] = <m,m>, coef[1+a] = h_a
        {
            const int E = (j == 0) ? 3 * s : 2 * s;
            const int per = (E + G - 1) / G;
            const int e0 = blk * per;
            const int e1 = min(E, e0 + per);
            for (int e = e0 + wid; e < e1; e += NW) {
                double t = 0.0;
                for (int g = lane; g < G; g += kWave) t += p.part_sk[static_cast<int64_t>(e) * G + g];
                t = wave_sum(t) * scale;
                if (lane == 0) {
                    if (e < s) p.SB[static_cast<int64_t>(j) * s + e] = t;
                    else if (e < 2 * s) p.SAB[static_cast<int64_t>(j) * s + (e - s)] = t;
                    else p.g[e - 2 * s] = t;
                }
            }
        }
        if (j == p.d - 1) break;

        double w[R];
#pragma unroll
        for (int r = 0; r < R; ++r) w[r] = m[r];
        if constexpr (KW > 0) {
#pragma unroll
            for (int a = 0; a < KW; ++a) {
                if (a < kw) {
                    const double h = coef[1 + a];
#pragma unroll
                    for (int r = 0; r < R; ++r) w[r] -= h * win[a][r];
                }
            }
        } else {
            for (int a = 0; a < kw; ++a) {
                const double h = coef[1 + a];
#pragma unroll
                for (int r = 0; r < R; ++r) w[r] -= h * Wg(j, a, r);
            }
        }
        dots_to_partials(w, j, kw, p.part_b);
        bar.sync();

        // ---- phase 3: h2, nu, b_{j+1} -----------------------------------
        double* c2 = coef + p.k + 1;
        grid_sum(p.part_b, G, kw + 1, c2);  // c2[0] = <w,w>, c2[1+a] = h2_a
        double h2sq = 0.0;
        for (int a = 0; a < kw; ++a) h2sq += c2[1 + a] * c2[1 + a];
        const double nu2 = c2[0] - h2sq;
        const double mm = coef[0];
        const bool breakdown = !(nu2 > 16.0 * kUnitRoundoff * kUnitRoundoff * mm);
        const double nu = breakdown ? 0.0 : sqrt(nu2);
        if (blk == 0 && tid <= p.k) {
            double hv;
            if (tid == p.k) hv = nu;
            else if (tid < kw) hv = coef[1 + tid] + c2[1 + tid];
            else hv = 0.0;
            p.H[static_cast<int64_t>(j) * (p.k + 1) + tid] = hv;
        }
        if (breakdown) {
            dc = j + 1;
            flags |= SGMRES_FLAG_BREAKDOWN;
            break;
        }
        double* bn = p.B + static_cast<int64_t>(j + 1) * p.ldb;
        double bnew[R];
#pragma unroll
        for (int r = 0; r < R; ++r) bnew[r] = w[r];
        if constexpr (KW > 0) {
#pragma unroll
            for (int a = 0; a < KW; ++a) {
                if (a < kw) {
                    const double h = c2[1 + a];
#pragma unroll
                    for (int r = 0; r < R; ++r) bnew[r] -= h * win[a][r];
                }
            }
        } else {
            for (int a = 0; a < kw; ++a) {
                const double h = c2[1 + a];
#pragma unroll
                for (int r = 0; r < R; ++r) bnew[r] -= h * Wg(j, a, r);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t row = base + static_cast<int64_t>(r) * BLOCK;
            bnew[r] = bnew[r] / nu;
            if (row < n) bn[row] = bnew[r];
        }
        if constexpr (KW > 0) {
#pragma unroll
            for (int a = KW - 1; a > 0; --a)
#pragma unroll
                for (int r = 0; r < R; ++r) win[a][r] = win[a - 1][r];
#pragma unroll
            for (int r = 0; r < R; ++r) win[0][r] = bnew[r];
        }
        bar.sync();
    }
    if (blk == 0 && tid == 0) {
        p.status[0] = dc;
        p.status[1] |= flags;
    }
}

using KernelFn = void (*)(ArnoldiParams);

template <int BLOCK>
KernelFn pick(int R, int KW) {
#define SG_CASE(RR, KK) \
    if (R == RR && KW == KK) return arnoldi_kernel<RR, KK, BLOCK>;
#define SG_ROW(RR) SG_CASE(RR, 0) SG_CASE(RR, 2) SG_CASE(RR, 4) SG_CASE(RR, 8)
    SG_ROW(1) SG_ROW(2) SG_ROW(4) SG_ROW(8)
#undef SG_ROW
#undef SG_CASE
    return nullptr;
}

KernelFn pick_kernel(int block, int R, int KW) {
    switch (block) {
        case 256: return pick<256>(R, KW);
        case 512: return pick<512>(R, KW);
        case 1024: return pick<1024>(R, KW);
        default: return nullptr;
    }
}

}  // namespace

size_t arnoldi_lds_bytes(int block, int R, int s, int k, int zeta) {
    const int nw = block / kWave;
    return sizeof(double) * static_cast<size_t>(2 * s + nw * kRedSlots + kRedSlots + 2 * k + 2) +
           sizeof(uint16_t) * static_cast<size_t>(zeta) * R * block;
}

hipError_t arnoldi_configure(const ArnoldiShape& shape, ArnoldiLaunch* out) {
    const int kw_need = shape.d > 1 ? (shape.k < shape.d - 1 ? shape.k : shape.d - 1) : 1;
    int device = 0;
    hipError_t err = hipGetDevice(&device);
    if (err != hipSuccess) return err;
    int cus = 0;
    err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (err != hipSuccess) return err;
    int lds_max = 0;
    err = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (err != hipSuccess) return err;

    const int blocks_try[3] = {shape.block ? shape.block : 512, 1024, 256};
    const int rows_try[4] = {1, 2, 4, 8};
    for (int bi = 0; bi < 3; ++bi) {
        const int block = blocks_try[bi];
        if (shape.block && block != shape.block) continue;
        for (int ri = 0; ri < 4; ++ri) {
            const int R = rows_try[ri];
            if (shape.rows_per_thread && R != shape.rows_per_thread) continue;
            int KW = 0;
            if (kw_need <= 2) KW = 2;
            else if (kw_need <= 4) KW = 4;
            else if (kw_need <= 8) KW = 8;
            if (KW * R > 32) KW = 0;  // keep the register window within 64 VGPRs
            if (shape.force_global_window) KW = 0;
            const size_t lds = arnoldi_lds_bytes(block, R, shape.s, shape.k, shape.zeta);
            if (lds > static_cast<size_t>(lds_max)) continue;
            KernelFn fn = pick_kernel(block, R, KW);
            if (!fn) continue;
            if (lds > 65536) {
                err = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          static_cast<int>(lds));
                if (err != hipSuccess) continue;
            }
            int per_cu = 0;
            err = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void*>(fn), block, lds);
            if (err != hipSuccess || per_cu < 1) continue;
            const int64_t need = (shape.n + static_cast<int64_t>(R) * block - 1) /
                                 (static_cast<int64_t>(R) * block);
            const int64_t gmax = static_cast<int64_t>(per_cu) * cus;
            if (need > gmax) continue;
            out->fn = reinterpret_cast<const void*>(fn);
            out->block = block;
            out->R = R;
            out->KW = KW;
            out->grid = static_cast<int>(need);
            out->lds = lds;
            return hipSuccess;
        }
    }
    return hipErrorInvalidValue;
}

hipError_t arnoldi_launch(const ArnoldiLaunch& L, ArnoldiParams params, hipStream_t stream) {
    void* args[] = {&params};
    return hipLaunchCooperativeKernel(L.fn, dim3(L.grid), dim3(L.block), args,
                                      static_cast<unsigned>(L.lds), stream);
}

}  // namespace sg
