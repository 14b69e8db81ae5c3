// Batched sGMRES: many independent systems per launch (arXiv:2111.00113,
// Algorithm 1 with restarting, Section 3.5, applied to each system).
//
// One workgroup owns one system for a whole cycle, so every reduction of the
// method is a workgroup reduction and no grid-wide synchronisation exists.
// Persistent workgroups take systems from a queue (largest first).  A system's
// rows are processed in chunks of CH = R * BLOCK (thread t owns rows
// r * BLOCK + t of each chunk).  Per cycle and system:
//   x += B y (previous cycle's least squares; FP64)
//   r = b - A x (FP64), |r|; stop if |r|/|b| <= tol
//   per chunk: sparse sign pattern of its rows, sorted by sketch row into
//     lists (stored for the cycle), and the chunk's share of g = S r
//   b_1 = r/|r|
//   per step j (three passes over the chunks, k-truncated Arnoldi with two
//   classical Gram-Schmidt passes, nu^2 = |w|^2 - |h2|^2):
//     m = A b_j, <m,m>, W^T m, chunk shares of S m           -> h
//     w = m - W h, <w,w>, W^T w                              -> h2, nu
//     b_{j+1} = (w - W h2) / nu
// S m_j is accumulated in LDS chunk by chunk in a fixed order (deterministic).
// The least squares runs afterwards as one workgroup per system (lsq.hip).
#include "common.hpp"
#include "internal.hpp"

namespace sg {

namespace {

constexpr int kBRed = kBatchMaxK + 1;  // window dots + one norm per reduction

__host__ __device__ constexpr int batch_vals_doubles(int CH, int zeta) {
    return (CH > (zeta * CH + 3) / 4) ? CH : (zeta * CH + 3) / 4;
}

template <int R, int BLOCK, typename TC, typename TS>
__global__ __launch_bounds__(BLOCK) void batched_cycle_kernel(BatchParams p) {
    constexpr int NW = BLOCK / kWave;
    constexpr int CH = R * BLOCK;
    extern __shared__ double smem[];
    const int s = p.s, zeta = p.zeta, d = p.d, k = p.k;
    // LDS: vals (one staged chunk vector, or the raw pattern) | reduction
    //      scratch | sketch accumulator (s) | piece sums | y (d) | list starts
    //      (s+1) | counters (s) | lists (zeta CH)
    double* vals = smem;
    double* red_tmp = vals + batch_vals_doubles(CH, zeta);
    double* red_out = red_tmp + NW * kBRed;
    double* acc = red_out + kBRed;
    double* sk_tmp = acc + s;
    double* ylds = sk_tmp + s * kSketchParts;
    int* lstart = reinterpret_cast<int*>(ylds + d);
    int* lcount = lstart + (s + 1);
    uint16_t* lists = reinterpret_cast<uint16_t*>(lcount + s);
    __shared__ int sys_sh;

    const int tid = threadIdx.x;
    const double scale = 1.0 / sqrt(static_cast<double>(zeta));
    const int cycle = *p.cycle;
    const bool combine = cycle > 0;
    const bool build = cycle <= p.restarts;
    constexpr double uround = BasisPrec<TC>::unit_roundoff;
    const int lstride = zeta * CH;  // list entries reserved per chunk

    for (;;) {
        if (tid == 0) {
            const int q = atomicAdd(p.queue, 1);
            sys_sh = q < p.nsys ? p.order[q] : -1;
        }
        __syncthreads();
        const int sid = sys_sh;
        __syncthreads();
        if (sid < 0) break;
        BatchState* st = p.st + sid;
        if (st->status != 0) continue;
        const BatchSys S = p.sys[sid];
        const int64_t n = S.n;
        const int nch = static_cast<int>((n + CH - 1) / CH);
        TS* Bs = static_cast<TS*>(S.B);
        const TC* Av = static_cast<const TC*>(S.valc);
        TC* Ms = static_cast<TC*>(S.m);
        TC* Ws = static_cast<TC*>(S.w);

        // ---- x += B y from the previous cycle --------------------------------
        if (combine) {
            const int de = min(st->d_eff, d);
            for (int c = tid; c < de; c += BLOCK) ylds[c] = S.y[c];
            __syncthreads();
            for (int ch = 0; ch < nch; ++ch) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t row = static_cast<int64_t>(ch) * CH + r * BLOCK + tid;
                    if (row < n) {
                        double a = 0.0;
                        for (int c = 0; c < de; ++c) a += from_basis<double>(Bs[c * n + row]) * ylds[c];
                        S.x[row] += a;
                    }
                }
            }
            __syncthreads();  // x complete before the residual gathers it
        }

        // ---- |b| on the first cycle ---------------------------------------
        double nf;
        if (cycle == 0) {
            double t = 0.0;
            for (int64_t row = tid; row < n; row += BLOCK) t += S.b[row] * S.b[row];
            const double v1[1] = {t};
            block_sum<1>(v1, 1, red_tmp, red_out);
            nf = sqrt(red_out[0]);
            if (tid == 0) st->nf = nf;
            if (!(nf < INFINITY)) {
                if (tid == 0) st->status = 3;
                continue;
            }
            if (nf == 0.0) {
                for (int64_t row = tid; row < n; row += BLOCK) S.x[row] = 0.0;
                if (tid == 0) {
                    st->rho = 0.0;
                    st->status = 1;
                }
                continue;
            }
        } else {
            nf = st->nf;
        }

        // ---- residual, sketch lists, g = S r -------------------------------
        for (int e = tid; e < s; e += BLOCK) acc[e] = 0.0;
        double rr = 0.0;
        for (int ch = 0; ch < nch; ++ch) {
            const int64_t base = static_cast<int64_t>(ch) * CH + tid;
            double rv[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t row = base + r * BLOCK;
                rv[r] = 0.0;
                if (row < n) {
                    double ax = 0.0;
                    const int q1 = S.rp[row + 1];
                    for (int q = S.rp[row]; q < q1; ++q) ax += S.val[q] * S.x[S.ci[q]];
                    rv[r] = S.b[row] - ax;
                    S.r[row] = rv[r];
                    rr += rv[r] * rv[r];
                }
            }
            if (build) {
                __syncthreads();  // the previous chunk's lists and vals are consumed
                sketch_lists_build<R, BLOCK>(p.seed, static_cast<uint32_t>(cycle), base, n, s, zeta,
                                             reinterpret_cast<uint16_t*>(vals), lstart, lcount, lists);
                const int cnt = lstart[s];
                for (int e = tid; e <= s; e += BLOCK) S.lstart[static_cast<int64_t>(ch) * (s + 1) + e] = lstart[e];
                for (int q = tid; q < cnt; q += BLOCK) S.lists[static_cast<int64_t>(ch) * lstride + q] = lists[q];
#pragma unroll
                for (int r = 0; r < R; ++r) vals[r * BLOCK + tid] = rv[r];
                __syncthreads();
                sketch_lists_reduce<BLOCK>(0, 1, 0, s, vals, CH, lstart, lists, sk_tmp,
                                           [&](int, int row, double a) { acc[row] += a; });
            }
        }
        {
            const double v1[1] = {rr};
            block_sum<1>(v1, 1, red_tmp, red_out);
        }
        const double beta = sqrt(red_out[0]);
        const double rho = beta / nf;
        if (tid == 0) {
            st->beta = beta;
            st->rho = rho;
        }
        if (!(rho < INFINITY)) {
            if (tid == 0) st->status = 3;
            continue;
        }
        if (rho <= p.tol) {
            if (tid == 0) st->status = 1;
            continue;
        }
        if (!build) {
            if (tid == 0) st->status = 2;
            continue;
        }
        if (tid == 0) atomicAdd(p.active, 1);
        for (int e = tid; e < s; e += BLOCK) S.g[e] = acc[e] * scale;

        // ---- b_1 = r / |r| ------------------------------------------------
        for (int64_t row = tid; row < n; row += BLOCK)
            Bs[row] = to_basis<TS>(static_cast<TC>(S.r[row] / beta));
        __syncthreads();

        // ---- basis steps ---------------------------------------------------
        int dc = d;
        int flags = 0;
        for (int j = 0; j < d; ++j) {
            const TS* bj = Bs + static_cast<int64_t>(j) * n;
            const int kw = min(j + 1, k);
            auto Wv = [&](int a, int64_t row) -> TC { return from_basis<TC>(Bs[static_cast<int64_t>(j - a) * n + row]); };

            // pass 1: m = A b_j, <m,m>, W^T m, S m
            for (int e = tid; e < s; e += BLOCK) acc[e] = 0.0;
            double dm[kBRed];
#pragma unroll
            for (int q = 0; q < kBRed; ++q) dm[q] = 0.0;
            for (int ch = 0; ch < nch; ++ch) {
                const int64_t base = static_cast<int64_t>(ch) * CH + tid;
                TC mv[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t row = base + r * BLOCK;
                    TC am = TC(0);
                    if (row < n) {
                        const int q1 = S.rp[row + 1];
                        for (int q = S.rp[row]; q < q1; ++q) am += Av[q] * from_basis<TC>(bj[S.ci[q]]);
                        Ms[row] = am;
                        dm[0] += static_cast<double>(am * am);
#pragma unroll
                        for (int a = 0; a < kBatchMaxK; ++a)
                            if (a < kw) dm[1 + a] += static_cast<double>(Wv(a, row) * am);
                    }
                    mv[r] = am;
                }
                __syncthreads();  // the previous chunk's lists and vals are consumed
                const int64_t lo = static_cast<int64_t>(ch) * (s + 1);
                for (int e = tid; e <= s; e += BLOCK) lstart[e] = S.lstart[lo + e];
                const int cnt = S.lstart[lo + s];
                for (int q = tid; q < cnt; q += BLOCK) lists[q] = S.lists[static_cast<int64_t>(ch) * lstride + q];
#pragma unroll
                for (int r = 0; r < R; ++r) vals[r * BLOCK + tid] = static_cast<double>(mv[r]);
                __syncthreads();
                sketch_lists_reduce<BLOCK>(0, 1, 0, s, vals, CH, lstart, lists, sk_tmp,
                                           [&](int, int row, double a) { acc[row] += a; });
            }
            block_sum<kBRed>(dm, kw + 1, red_tmp, red_out);
            const double mm = red_out[0];
            double h[kBatchMaxK];
#pragma unroll
            for (int a = 0; a < kBatchMaxK; ++a) h[a] = (a < kw) ? red_out[1 + a] : 0.0;
            for (int e = tid; e < s; e += BLOCK) S.SAB[static_cast<int64_t>(j) * s + e] = acc[e] * scale;
            if (j == d - 1) break;

            // pass 2: w = m - W h, <w,w>, W^T w
            double dw[kBRed];
#pragma unroll
            for (int q = 0; q < kBRed; ++q) dw[q] = 0.0;
            for (int64_t row = tid; row < n; row += BLOCK) {
                TC wv = Ms[row];
#pragma unroll
                for (int a = 0; a < kBatchMaxK; ++a)
                    if (a < kw) wv -= static_cast<TC>(h[a]) * Wv(a, row);
                Ws[row] = wv;
                dw[0] += static_cast<double>(wv * wv);
#pragma unroll
                for (int a = 0; a < kBatchMaxK; ++a)
                    if (a < kw) dw[1 + a] += static_cast<double>(Wv(a, row) * wv);
            }
            block_sum<kBRed>(dw, kw + 1, red_tmp, red_out);
            double h2[kBatchMaxK];
            double h2sq = 0.0;
#pragma unroll
            for (int a = 0; a < kBatchMaxK; ++a) {
                h2[a] = (a < kw) ? red_out[1 + a] : 0.0;
                h2sq += h2[a] * h2[a];
            }
            const double nu2 = red_out[0] - h2sq;
            if (!(nu2 > 16.0 * uround * uround * mm)) {  // invariant subspace: stop at this column
                dc = j + 1;
                flags |= SGMRES_FLAG_BREAKDOWN;
                break;
            }
            const TC nu = static_cast<TC>(sqrt(nu2));

            // pass 3: b_{j+1} = (w - W h2) / nu
            TS* bn = Bs + static_cast<int64_t>(j + 1) * n;
            for (int64_t row = tid; row < n; row += BLOCK) {
                TC bv = Ws[row];
#pragma unroll
                for (int a = 0; a < kBatchMaxK; ++a)
                    if (a < kw) bv -= static_cast<TC>(h2[a]) * Wv(a, row);
                bn[row] = to_basis<TS>(bv / nu);
            }
            __syncthreads();  // b_{j+1} complete before the next step gathers it
        }
        if (tid == 0) {
            st->dc = dc;
            st->flags |= flags;
            st->cycles += 1;
            st->steps += dc;
        }
        __syncthreads();
    }
}

// ctr: [0] cycle, [1] queue position, [2] systems active this cycle, [3] the
// count of the cycle that just ended (what the host reads)
__global__ void batch_advance_kernel(int* ctr) {
    if (threadIdx.x == 0) {
        ctr[3] = ctr[2];
        ctr[2] = 0;
        ctr[1] = 0;
        ctr[0] += 1;
    }
}

__global__ void batch_reset_kernel(BatchState* st, int nsys, int* ctr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nsys) st[i] = BatchState{};
    if (i < 4) ctr[i] = 0;
}

using KernelFn = void (*)(BatchParams);

template <typename TC, typename TS>
KernelFn pick_typed(int block, int R) {
#define SG_CASE(BB, RR) \
    if (block == BB && R == RR) return batched_cycle_kernel<RR, BB, TC, TS>;
    SG_CASE(256, 4) SG_CASE(512, 2) SG_CASE(512, 4) SG_CASE(1024, 1) SG_CASE(1024, 2) SG_CASE(1024, 4)
#undef SG_CASE
    return nullptr;
}

KernelFn pick_kernel(int block, int R, int precision) {
    switch (precision) {
        case SGMRES_PREC_FP64: return pick_typed<double, double>(block, R);
        case SGMRES_PREC_FP32: return pick_typed<float, float>(block, R);
        case SGMRES_PREC_BF16_BASIS: return pick_typed<float, bf16_t>(block, R);
        default: return nullptr;
    }
}

}  // namespace

hipError_t batch_configure(int block, int R, int d, int s, int zeta, int precision, BatchLaunch* out) {
    KernelFn fn = pick_kernel(block, R, precision);
    if (!fn) return hipErrorInvalidValue;
    const int CH = block * R;
    const size_t lds = sizeof(double) * static_cast<size_t>(batch_vals_doubles(CH, zeta) + (block / kWave) * kBRed +
                                                            kBRed + s + s * kSketchParts + d) +
                       sizeof(int) * static_cast<size_t>(2 * s + 1) + sizeof(uint16_t) * static_cast<size_t>(zeta) * CH;
    int device = 0;
    hipError_t err = hipGetDevice(&device);
    if (err != hipSuccess) return err;
    int cus = 0, lds_max = 0;
    err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (err != hipSuccess) return err;
    err = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (err != hipSuccess) return err;
    if (lds > static_cast<size_t>(lds_max)) return hipErrorInvalidValue;
    err = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(lds));
    if (err != hipSuccess) return err;
    int per_cu = 0;
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn), block, lds);
    if (err != hipSuccess) return err;
    if (per_cu < 1) return hipErrorInvalidValue;
    out->fn = reinterpret_cast<const void*>(fn);
    out->block = block;
    out->R = R;
    out->grid = per_cu * cus;
    out->lds = lds;
    return hipSuccess;
}

hipError_t batch_launch(const BatchLaunch& L, const BatchParams& p, hipStream_t stream) {
    BatchParams q = p;
    void* args[] = {&q};
    return hipLaunchKernel(L.fn, dim3(L.grid), dim3(L.block), args, L.lds, stream);
}

hipError_t launch_batch_advance(int* ctr, hipStream_t stream) {
    batch_advance_kernel<<<1, 64, 0, stream>>>(ctr);
    return hipGetLastError();
}

hipError_t launch_batch_reset(BatchState* st, int nsys, int* ctr, hipStream_t stream) {
    const int n = nsys > 4 ? nsys : 4;
    batch_reset_kernel<<<(n + 255) / 256, 256, 0, stream>>>(st, nsys, ctr);
    return hipGetLastError();
}

}  // namespace sg
