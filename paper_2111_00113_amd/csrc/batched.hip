// Batched sGMRES: many independent systems per launch (arXiv:2111.00113,
// Algorithm 1 with restarting, Section 3.5, applied to each system).
//
// Work unit: a part of a system, i.e. a range of whole chunks of CH = R * BLOCK
// rows (thread t owns rows r * BLOCK + t of each chunk).  Small systems are one
// part; large ones are split so that no workgroup carries much more than a
// fixed number of rows.  Persistent workgroups take parts from a queue in which
// the parts of a system are consecutive (largest systems first); the parts of a
// system synchronise through a per-system counter (bounded waits), and a system
// never has more parts than the grid has workgroups, so every part that waits
// can count on the others being taken by free workgroups.
//
// Per cycle and system (each part on its rows; sums over the parts in fixed
// part order, so every part sees the same bits and takes the same decisions):
//   x += B y (previous cycle's least squares; FP64)
//   r = b - A x (FP64), |r|; stop if |r|/|b| <= tol
//   per chunk: sparse sign pattern of its rows, sorted by sketch row into
//     lists (stored for the cycle), and the chunk's share of g = S r
//   b_1 = r/|r|
//   per step j (k-truncated Arnoldi, two classical Gram-Schmidt passes,
//   nu^2 = |w|^2 - |h2|^2; three group barriers):
//     m = A b_j, <m,m>, W^T m, S m                      -> h, column j of S A B
//     w = m - W h, <w,w>, W^T w                         -> h2, nu
//     b_{j+1} = (w - W h2) / nu                         -> visible to all parts
// The least squares runs afterwards as one workgroup per system (lsq.hip).
#include "common.hpp"
#include "internal.hpp"

namespace sg {

namespace {

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
    double* red_out = red_tmp + NW * kBatchRed;
    double* acc = red_out + kBatchRed;
    double* sk_tmp = acc + s;
    double* ylds = sk_tmp + s * kSketchParts;
    int* lstart = reinterpret_cast<int*>(ylds + d);
    int* lcount = lstart + (s + 1);
    uint16_t* lists = reinterpret_cast<uint16_t*>(lcount + s);
    __shared__ int task_sh;
    __shared__ int fail_sh;

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
            task_sh = q < p.ntask ? q : -1;
        }
        __syncthreads();
        const int ti = task_sh;
        __syncthreads();
        if (ti < 0) break;
        const BatchTask T = p.task[ti];
        const int sid = T.sys, part = T.part, P = T.nparts;
        BatchState* st = p.st + sid;
        if (st->status != 0) continue;  // decided in an earlier cycle: the same for every part
        const BatchSys S = p.sys[sid];
        const int64_t n = S.n;
        const int64_t r0 = T.r0, r1 = T.r1;
        const int ch0 = static_cast<int>(r0 / CH);
        const int nch = static_cast<int>((r1 - r0 + CH - 1) / CH);
        TS* Bs = static_cast<TS*>(S.B);
        const TC* Av = static_cast<const TC*>(S.valc);
        TC* Ms = static_cast<TC*>(S.m);
        TC* Ws = static_cast<TC*>(S.w);
        double* red_slot = p.slots + p.slot_off[sid];    // [2][kBatchRed][P]
        double* sk_slot = red_slot + 2 * P * kBatchRed;  // [s][P]
        unsigned* cnt = p.gcnt + sid;
        unsigned epoch = 0;
        int nred = 0;
        bool failed = false;
        const bool lead = part == 0;

        // barrier among the parts of this system (a workgroup barrier when P = 1)
        auto gsync = [&]() {
            if (P == 1) {
                __syncthreads();
                return;
            }
            ++epoch;
            __syncthreads();
            if (tid == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned target = epoch * static_cast<unsigned>(P);
                const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
                int f = 0;
                while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                    if (__hip_atomic_load(p.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                        f = 1;
                        break;
                    }
                    if (__builtin_amdgcn_s_memrealtime() - t0 > p.spin_limit) {
                        __hip_atomic_store(p.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        f = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                fail_sh = f;
            }
            __syncthreads();
            failed = failed || (fail_sh != 0);
        };
        // Sums over the P parts of src[e * P + q], q = 0 .. P-1, for e in
        // [e0, e1): a group of L lanes (L = P rounded up to a power of two, at
        // most 64) per entry, up to four loads per lane issued together, then a
        // fixed xor butterfly over the group.  Deterministic for a given P.
        static_assert(kBatchMaxParts <= 4 * kWave, "group sums load at most four values per lane");
        auto parts_sum = [&](const double* src, int e0, int e1, auto&& out) {
            const int lane = tid & (kWave - 1);
            int L = 1;
            while (L < P && L < kWave) L <<= 1;
            const int per_wave = kWave / L, ql = lane & (L - 1);
            for (int eb = e0 + (tid / kWave) * per_wave; eb < e1; eb += NW * per_wave) {
                const int e = eb + lane / L;
                double t[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int q = ql + u * L;
                    t[u] = (e < e1 && q < P) ? src[static_cast<int64_t>(e) * P + q] : 0.0;
                }
                double a = 0.0;
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (ql + u * L < P) a += t[u];
                for (int o = L >> 1; o >= 1; o >>= 1) a += __shfl_xor(a, o, kWave);
                if (ql == 0 && e < e1) out(e, a);
            }
        };
        // red_out[0..nv) (this part's workgroup sums) -> sums over all parts.
        // With dst != null also the parts' sketch accumulators are exchanged
        // (one barrier for both); part q sums the sketch rows of its share of
        // [0, s) and writes dst = scale * sum for them.
        auto group_sum = [&](int nv, double* dst) {
            if (P == 1) {
                if (dst)
                    for (int e = tid; e < s; e += BLOCK) dst[e] = acc[e] * scale;
                return;
            }
            double* sl = red_slot + (nred & 1) * P * kBatchRed;
            ++nred;
            if (tid < nv) sl[tid * P + part] = red_out[tid];
            if (dst)
                for (int e = tid; e < s; e += BLOCK) sk_slot[static_cast<int64_t>(e) * P + part] = acc[e];
            gsync();
            parts_sum(sl, 0, nv, [&](int e, double a) { red_out[e] = a; });
            if (dst)
                parts_sum(sk_slot, static_cast<int>(static_cast<int64_t>(part) * s / P),
                          static_cast<int>(static_cast<int64_t>(part + 1) * s / P),
                          [&](int e, double a) { dst[e] = a * scale; });
            __syncthreads();
        };
        auto decide = [&](int code) {
            if (lead && tid == 0) st->next = code;
        };

        // ---- x += B y from the previous cycle --------------------------------
        if (combine) {
            const int de = min(st->d_eff, d);
            for (int c = tid; c < de; c += BLOCK) ylds[c] = S.y[c];
            __syncthreads();
            for (int64_t row = r0 + tid; row < r1; row += BLOCK) {
                double a = 0.0;
                for (int c = 0; c < de; ++c) a = madd(from_basis<double>(Bs[c * n + row]), ylds[c], a);
                S.x[row] += a;
            }
            gsync();  // x complete before the residual gathers it
            if (failed) {
                decide(4);
                continue;
            }
        }

        // ---- |b| on the first cycle ---------------------------------------
        double nf;
        if (cycle == 0) {
            double t = 0.0;
            for (int64_t row = r0 + tid; row < r1; row += BLOCK) t = madd(S.b[row], S.b[row], t);
            const double v1[1] = {t};
            block_sum<1>(v1, 1, red_tmp, red_out);
            group_sum(1, nullptr);
            if (failed) {
                decide(4);
                continue;
            }
            nf = sqrt(red_out[0]);
            if (lead && tid == 0) st->nf = nf;
            if (!(nf < INFINITY)) {
                decide(3);
                continue;
            }
            if (nf == 0.0) {
                for (int64_t row = r0 + tid; row < r1; row += BLOCK) S.x[row] = 0.0;
                if (lead && tid == 0) st->rho = 0.0;
                decide(1);
                continue;
            }
        } else {
            nf = st->nf;
        }

        // ---- residual, sketch lists, g = S r -------------------------------
        for (int e = tid; e < s; e += BLOCK) acc[e] = 0.0;
        double rr = 0.0;
        for (int c = 0; c < nch; ++c) {
            const int ch = ch0 + c;
            const int64_t base = static_cast<int64_t>(ch) * CH + tid;
            // A x with nonzero slot outermost over the R rows (independent
            // loads in flight; each row summed in CSR order)
            int rb[R], rl[R];
            int kmax = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t row = base + r * BLOCK;
                rb[r] = row < r1 ? S.rp[row] : 0;
                rl[r] = row < r1 ? S.rp[row + 1] - rb[r] : 0;
                kmax = max(kmax, rl[r]);
            }
            double ax[R];
#pragma unroll
            for (int r = 0; r < R; ++r) ax[r] = 0.0;
            for (int q = 0; q < kmax; ++q) {
                int c[R];
                double v[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    c[r] = 0;
                    v[r] = 0.0;
                    if (q < rl[r]) {
                        c[r] = S.ci[rb[r] + q];
                        v[r] = S.val[rb[r] + q];
                    }
                }
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (q < rl[r]) ax[r] = madd(v[r], S.x[c[r]], ax[r]);
            }
            double rv[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t row = base + r * BLOCK;
                rv[r] = 0.0;
                if (row < r1) {
                    rv[r] = S.b[row] - ax[r];
                    S.r[row] = rv[r];
                    rr = madd(rv[r], rv[r], rr);
                }
            }
            if (build) {
                __syncthreads();  // the previous chunk's lists and vals are consumed
                sketch_lists_build<R, BLOCK>(p.seed, static_cast<uint32_t>(cycle), base, r1, s, zeta,
                                             reinterpret_cast<uint16_t*>(vals), lstart, lcount, lists);
                const int cntl = lstart[s];
                for (int e = tid; e <= s; e += BLOCK) S.lstart[static_cast<int64_t>(ch) * (s + 1) + e] = lstart[e];
                for (int q = tid; q < cntl; q += BLOCK) S.lists[static_cast<int64_t>(ch) * lstride + q] = lists[q];
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
        group_sum(1, build ? S.g : nullptr);
        if (failed) {
            decide(4);
            continue;
        }
        const double beta = sqrt(red_out[0]);
        const double rho = beta / nf;
        if (lead && tid == 0) {
            st->beta = beta;
            st->rho = rho;
        }
        if (!(rho < INFINITY)) {
            decide(3);
            continue;
        }
        if (rho <= p.tol) {
            decide(1);
            continue;
        }
        if (!build) {
            decide(2);
            continue;
        }
        if (lead && tid == 0) atomicAdd(p.active, 1);

        // ---- b_1 = r / |r| ------------------------------------------------
        for (int64_t row = r0 + tid; row < r1; row += BLOCK)
            Bs[row] = to_basis<TS>(static_cast<TC>(S.r[row] / beta));
        gsync();
        if (failed) {
            decide(4);
            continue;
        }

        // ---- basis steps ---------------------------------------------------
        int dc = d;
        int flags = 0;
        for (int j = 0; j < d; ++j) {
            const TS* bj = Bs + static_cast<int64_t>(j) * n;
            const int kw = min(j + 1, k);
            auto Wv = [&](int a, int64_t row) -> TC { return from_basis<TC>(Bs[static_cast<int64_t>(j - a) * n + row]); };

            // pass 1: m = A b_j, <m,m>, W^T m, S m
            for (int e = tid; e < s; e += BLOCK) acc[e] = 0.0;
            double dm[kBatchRed];
#pragma unroll
            for (int q = 0; q < kBatchRed; ++q) dm[q] = 0.0;
            for (int c = 0; c < nch; ++c) {
                const int ch = ch0 + c;
                const int64_t base = static_cast<int64_t>(ch) * CH + tid;
                // m = A b_j, nonzero slot outermost over the R rows
                int rb[R], rl[R];
                int kmax = 0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t row = base + r * BLOCK;
                    rb[r] = row < r1 ? S.rp[row] : 0;
                    rl[r] = row < r1 ? S.rp[row + 1] - rb[r] : 0;
                    kmax = max(kmax, rl[r]);
                }
                TC mv[R];
#pragma unroll
                for (int r = 0; r < R; ++r) mv[r] = TC(0);
                for (int q = 0; q < kmax; ++q) {
                    int c[R];
                    TC v[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        c[r] = 0;
                        v[r] = TC(0);
                        if (q < rl[r]) {
                            c[r] = S.ci[rb[r] + q];
                            v[r] = Av[rb[r] + q];
                        }
                    }
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (q < rl[r]) mv[r] = madd(v[r], from_basis<TC>(bj[c[r]]), mv[r]);
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t row = base + r * BLOCK;
                    if (row < r1) {
                        const TC am = mv[r];
                        Ms[row] = am;
                        dm[0] = dot_acc(dm[0], am, am);
#pragma unroll
                        for (int a = 0; a < kBatchMaxK; ++a)
                            if (a < kw) dm[1 + a] = dot_acc(dm[1 + a], Wv(a, row), am);
                    }
                }
                __syncthreads();  // the previous chunk's lists and vals are consumed
                const int64_t lo = static_cast<int64_t>(ch) * (s + 1);
                for (int e = tid; e <= s; e += BLOCK) lstart[e] = S.lstart[lo + e];
                const int cntl = S.lstart[lo + s];
                for (int q = tid; q < cntl; q += BLOCK) lists[q] = S.lists[static_cast<int64_t>(ch) * lstride + q];
#pragma unroll
                for (int r = 0; r < R; ++r) vals[r * BLOCK + tid] = static_cast<double>(mv[r]);
                __syncthreads();
                sketch_lists_reduce<BLOCK>(0, 1, 0, s, vals, CH, lstart, lists, sk_tmp,
                                           [&](int, int row, double a) { acc[row] += a; });
            }
            block_sum<kBatchRed>(dm, kw + 1, red_tmp, red_out);
            group_sum(kw + 1, S.SAB + static_cast<int64_t>(j) * s);
            if (failed) break;
            const double mm = red_out[0];
            double h[kBatchMaxK];
#pragma unroll
            for (int a = 0; a < kBatchMaxK; ++a) h[a] = (a < kw) ? red_out[1 + a] : 0.0;
            if (j == d - 1) break;

            // pass 2: w = m - W h, <w,w>, W^T w
            double dw[kBatchRed];
#pragma unroll
            for (int q = 0; q < kBatchRed; ++q) dw[q] = 0.0;
            for (int64_t row = r0 + tid; row < r1; row += BLOCK) {
                TC wv = Ms[row];
#pragma unroll
                for (int a = 0; a < kBatchMaxK; ++a)
                    if (a < kw) wv = madd(-static_cast<TC>(h[a]), Wv(a, row), wv);
                Ws[row] = wv;
                dw[0] = dot_acc(dw[0], wv, wv);
#pragma unroll
                for (int a = 0; a < kBatchMaxK; ++a)
                    if (a < kw) dw[1 + a] = dot_acc(dw[1 + a], Wv(a, row), wv);
            }
            block_sum<kBatchRed>(dw, kw + 1, red_tmp, red_out);
            group_sum(kw + 1, nullptr);
            if (failed) break;
            double h2[kBatchMaxK];
            double h2sq = 0.0;
#pragma unroll
            for (int a = 0; a < kBatchMaxK; ++a) {
                h2[a] = (a < kw) ? red_out[1 + a] : 0.0;
                h2sq = madd(h2[a], h2[a], h2sq);
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
            for (int64_t row = r0 + tid; row < r1; row += BLOCK) {
                TC bv = Ws[row];
#pragma unroll
                for (int a = 0; a < kBatchMaxK; ++a)
                    if (a < kw) bv = madd(-static_cast<TC>(h2[a]), Wv(a, row), bv);
                bn[row] = to_basis<TS>(bv / nu);
            }
            gsync();  // b_{j+1} complete before the next step gathers it
            if (failed) break;
        }
        if (failed) {
            decide(4);
            continue;
        }
        if (lead && tid == 0) {
            st->dc = dc;
            st->flags |= flags;
            st->cycles += 1;
            st->steps += dc;
        }
        __syncthreads();
    }
}

// ctr: [0] cycle, [1] queue position, [2] systems active this cycle, [3] the
// count of the cycle that just ended (what the host reads).  Each system's
// status takes the value decided during the cycle; group counters restart.
__global__ void batch_advance_kernel(int* ctr, BatchState* st, unsigned* gcnt, int nsys) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nsys) {
        if (st[i].status == 0) st[i].status = st[i].next;
        gcnt[i] = 0u;
    }
    if (i == 0) {
        ctr[3] = ctr[2];
        ctr[2] = 0;
        ctr[1] = 0;
        ctr[0] += 1;
    }
}

__global__ void batch_reset_kernel(BatchState* st, unsigned* gcnt, int nsys, int* ctr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nsys) {
        st[i] = BatchState{};
        gcnt[i] = 0u;
    }
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
    const size_t lds = sizeof(double) * static_cast<size_t>(batch_vals_doubles(CH, zeta) + (block / kWave) * kBatchRed +
                                                            kBatchRed + s + s * kSketchParts + d) +
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

// A cooperative launch: the runtime starts the grid only when every workgroup
// can be resident at once (grid <= occupancy x CUs), which the parts of a
// system waiting for each other rely on (a launch that cannot be placed
// fails instead of leaving a part to wait for a partner that never starts).
// The attribute form is also what a stream capture records as a cooperative
// kernel node.
hipError_t batch_launch(const BatchLaunch& L, const BatchParams& p, hipStream_t stream) {
    BatchParams q = p;
    void* args[] = {&q};
    hipLaunchAttribute attr{};
    attr.id = hipLaunchAttributeCooperative;
    attr.val.cooperative = 1;
    hipLaunchConfig_t cfg{};
    cfg.gridDim = dim3(L.grid);
    cfg.blockDim = dim3(L.block);
    cfg.dynamicSmemBytes = L.lds;
    cfg.stream = stream;
    cfg.attrs = &attr;
    cfg.numAttrs = 1;
    return hipLaunchKernelExC(&cfg, L.fn, args);
}

hipError_t launch_batch_advance(int* ctr, BatchState* st, unsigned* gcnt, int nsys, hipStream_t stream) {
    const int n = nsys > 1 ? nsys : 1;
    batch_advance_kernel<<<(n + 255) / 256, 256, 0, stream>>>(ctr, st, gcnt, nsys);
    return hipGetLastError();
}

hipError_t launch_batch_reset(BatchState* st, unsigned* gcnt, int nsys, int* ctr, hipStream_t stream) {
    const int n = nsys > 4 ? nsys : 4;
    batch_reset_kernel<<<(n + 255) / 256, 256, 0, stream>>>(st, gcnt, nsys, ctr);
    return hipGetLastError();
}

}  // namespace sg
