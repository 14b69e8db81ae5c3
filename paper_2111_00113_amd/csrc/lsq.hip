// sketched_lsq: the small sketched least-squares problem of sGMRES
// (arXiv:2111.00113, Algorithm 1 solve step; Section 3.3):
//   unpivoted Householder QR  S A B = Q T  (reflectors applied to g = S r too),
//   condition guard on the diagonal of T (Sections 3.4 and 5.3),
//   back substitution T y = Q^T g on the kept prefix,
//   residual estimate |(Q^T g)[d_eff:]|.
// Two versions: a column-owner pipeline over many workgroups (s <= 512, the
// default) and one workgroup of 1024 threads for larger s, where the s x dc
// matrix stays in global memory (L2-resident) and each reflector is staged in
// LDS.
#include "common.hpp"
#include "internal.hpp"

namespace sg {

namespace {

constexpr int kLsqBlock = 1024;
constexpr int kLsqWaves = kLsqBlock / kWave;
constexpr int kZSlots = kLsqMaxCols / kWave;

// The whole solve on one workgroup of kLsqBlock threads; v: s doubles of LDS.
__device__ void lsq_body(int s, int dc, double* __restrict__ C, double* __restrict__ g, double kappa_max,
                         double* __restrict__ y, double* __restrict__ dout, int* __restrict__ iout, double* v) {
    __shared__ double tmp[kLsqWaves];
    __shared__ double red[1];
    __shared__ double bc[3];
    __shared__ int ibc[1];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;

    for (int p = 0; p < dc; ++p) {
        double* cp = C + static_cast<int64_t>(p) * s;
        double t = 0.0;
        for (int i = p + 1 + tid; i < s; i += kLsqBlock) t += cp[i] * cp[i];
        const double vals[1] = {t};
        block_sum<1>(vals, 1, tmp, red);
        if (tid == 0) {
            const double alpha = cp[p];
            const double xn2 = red[0];
            double beta, tau, sc;
            if (xn2 == 0.0) {  // identity reflector
                beta = alpha;
                tau = 0.0;
                sc = 1.0;
            } else {
                const double nrm = sqrt(alpha * alpha + xn2);
                beta = (alpha >= 0.0) ? -nrm : nrm;
                tau = (beta - alpha) / beta;
                sc = 1.0 / (alpha - beta);
            }
            bc[0] = beta;
            bc[1] = tau;
            bc[2] = sc;
        }
        __syncthreads();
        const double tau = bc[1];
        const double sc = bc[2];
        if (tau != 0.0) {
            for (int i = p + 1 + tid; i < s; i += kLsqBlock) {
                const double c = cp[i] * sc;
                cp[i] = c;
                v[i] = c;
            }
        }
        if (tid == 0) cp[p] = bc[0];
        __syncthreads();
        if (tau != 0.0) {
            // columns p+1 .. dc-1 of C, and g as column dc: one wavefront each
            for (int c = p + 1 + wid; c <= dc; c += kLsqWaves) {
                double* col = (c < dc) ? C + static_cast<int64_t>(c) * s : g;
                double sd = 0.0;
                for (int i = p + 1 + lane; i < s; i += kWave) sd += v[i] * col[i];
                sd = wave_sum(sd);
                const double head = col[p];
                sd = (head + sd) * tau;
                for (int i = p + 1 + lane; i < s; i += kWave) col[i] -= sd * v[i];
                if (lane == 0) col[p] = head - sd;
            }
        }
        __syncthreads();
    }

    // longest prefix whose diagonal ratio stays within kappa_max
    if (tid == 0) {
        int d_eff = 0;
        double tmax = 0.0, tmin = INFINITY, kap = 0.0;
        for (int j = 0; j < dc; ++j) {
            const double a = fabs(C[static_cast<int64_t>(j) * s + j]);
            const double nmax = a > tmax ? a : tmax;
            const double nmin = a < tmin ? a : tmin;
            if (!(nmin > 0.0) || nmax / nmin > kappa_max) break;
            tmax = nmax;
            tmin = nmin;
            kap = tmax / tmin;
            d_eff = j + 1;
        }
        ibc[0] = d_eff;
        dout[1] = kap;
        iout[0] = d_eff;
        if (d_eff < dc) iout[1] |= SGMRES_FLAG_KAPPA_TRUNC;
    }
    __syncthreads();
    const int d_eff = ibc[0];

    // back substitution on one wavefront, Q^T g held in registers
    if (wid == 0) {
        double z[kZSlots];
#pragma unroll
        for (int c = 0; c < kZSlots; ++c) {
            const int q = lane + c * kWave;
            z[c] = (q < d_eff) ? g[q] : 0.0;
        }
        for (int i = d_eff - 1; i >= 0; --i) {
            const int slot = i / kWave;
            double mine = 0.0;
#pragma unroll
            for (int c = 0; c < kZSlots; ++c)
                if (c == slot) mine = z[c];
            const double zi = readlane_d(mine, i & (kWave - 1));
            const double* tcol = C + static_cast<int64_t>(i) * s;
            const double yi = zi / tcol[i];
            if (lane == 0) y[i] = yi;
#pragma unroll
            for (int c = 0; c < kZSlots; ++c) {
                const int q = lane + c * kWave;
                if (q < i) z[c] -= tcol[q] * yi;
            }
        }
    }

    double t = 0.0;
    for (int i = d_eff + tid; i < s; i += kLsqBlock) t += g[i] * g[i];
    const double vals[1] = {t};
    block_sum<1>(vals, 1, tmp, red);
    if (tid == 0) dout[0] = sqrt(red[0]);
}

__global__ __launch_bounds__(kLsqBlock) void lsq_kernel(int s, const int* __restrict__ dc_dev, int dc_host,
                                                        double* __restrict__ C, double* __restrict__ g,
                                                        double kappa_max, double* __restrict__ y,
                                                        double* __restrict__ dout, int* __restrict__ iout) {
    extern __shared__ double v[];  // s doubles: tail of the current reflector
    lsq_body(s, dc_dev ? *dc_dev : dc_host, C, g, kappa_max, y, dout, iout, v);
}

// One workgroup per system of a batch; systems no longer active are skipped.
__global__ __launch_bounds__(kLsqBlock) void lsq_batched_kernel(int s, const BatchSys* __restrict__ sys,
                                                                BatchState* __restrict__ st, double kappa_max) {
    extern __shared__ double v[];
    BatchState* t = st + blockIdx.x;
    if (t->status != 0 || t->next != 0) return;  // only systems that built a basis this cycle
    const BatchSys& S = sys[blockIdx.x];
    lsq_body(s, t->dc, S.SAB, S.g, kappa_max, S.y, &t->rest, &t->d_eff, v);
}

// ---------------------------------------------------------------------------
// Blocked column-owner pipeline (s <= 64*S): wavefront w keeps columns
// [w*CB, w*CB + CB) of C -- column dc stands for g -- in registers for the
// whole factorisation.  It applies the reflectors of earlier wavefronts in
// order as they are published, factors its own columns locally (each new
// reflector applied at once to its later columns), writes them back (T entries
// above the diagonal, beta on it, the reflector tail below) and publishes them
// by raising a counter.  Every column therefore sees the reflectors in the
// same order as in the one-workgroup kernel above.  The wavefront holding g
// finishes with the kappa guard, the back substitution and the residual
// estimate.  Launched cooperatively (all wavefronts resident); every wait is
// bounded by a real-time limit.
// ---------------------------------------------------------------------------
constexpr int kPipeWaves = 4;
constexpr int kPipeBlock = kPipeWaves * kWave;
constexpr int kPipeCols = 8;  // columns per wavefront

struct LsqSync {
    unsigned npub;  // reflectors published (monotone, in order)
    unsigned pad[63];
};

// row p of a register-resident column (row p lives in lane p % 64, slot p / 64)
template <int S>
__device__ __forceinline__ double row_of(const double (&col)[S], int p) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < S; ++q)
        if (q == (p >> 6)) v = col[q];
    return readlane_d(v, p & (kWave - 1));
}

// Reflector p as a register column: zero above row p, 1 on it, the stored tail
// (rows p+1 .. s-1 of vp) below.  live = false gives the zero vector.
template <int S>
__device__ __forceinline__ void load_reflector(double (&v)[S], const double* vp, int p, int s, int lane, bool live) {
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const int r = lane + q * kWave;
        const double x = vp[min(r, s - 1)];  // unconditional load (no branch around it), row clamped into the column
        v[q] = !live ? 0.0 : (r > p && r < s) ? x : (r == p ? 1.0 : 0.0);
    }
}

// col[i] <- (I - tau v v^T) col[i] for the register-resident columns i >= I0.
// v carries its unit entry, so neither the dot product nor the update needs a
// special row; the reductions of the columns are interleaved so that their
// latencies overlap.
template <int I0, int S, int CB>
__device__ __forceinline__ void apply_reflector_cols(double (&col)[CB][S], const double (&v)[S], double tau) {
    double sd[CB];
#pragma unroll
    for (int i = I0; i < CB; ++i) {
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < S; ++q) a += v[q] * col[i][q];
        sd[i] = a;
    }
    // interleaved wave sums (the step order of wave_sum)
#pragma unroll
    for (int i = I0; i < CB; ++i) sd[i] = dpp_add<0xb1, 0xf>(sd[i]);
#pragma unroll
    for (int i = I0; i < CB; ++i) sd[i] = dpp_add<0x4e, 0xf>(sd[i]);
#pragma unroll
    for (int i = I0; i < CB; ++i) sd[i] = dpp_add<0x141, 0xf>(sd[i]);
#pragma unroll
    for (int i = I0; i < CB; ++i) sd[i] = dpp_add<0x140, 0xf>(sd[i]);
#pragma unroll
    for (int i = I0; i < CB; ++i) sd[i] = dpp_add<0x142, 0xa>(sd[i]);
#pragma unroll
    for (int i = I0; i < CB; ++i) sd[i] = dpp_add<0x143, 0xc>(sd[i]);
#pragma unroll
    for (int i = I0; i < CB; ++i) {
        const double t = readlane_d(sd[i], kWave - 1) * tau;
#pragma unroll
        for (int q = 0; q < S; ++q) col[i][q] -= t * v[q];
    }
}

// Factor the held column I (global column c0 + I, if below dc): its reflector
// is written to C and tau, and applied at once to the held columns after it;
// then the next held column.  Unrolled at compile time over I.
template <int I, int S, int CB>
__device__ __forceinline__ void factor_held(double (&col)[CB][S], int c0, int dc, int s, int lane,
                                            double* __restrict__ C, double* __restrict__ tau) {
    if constexpr (I < CB) {
        const int c = c0 + I;
        if (c < dc) {
            double xl = 0.0;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const int r = lane + q * kWave;
                if (r > c) xl += col[I][q] * col[I][q];
            }
            const double xn2 = wave_sum(xl);
            const double alpha = row_of<S>(col[I], c);
            double beta, tc, sc;
            if (xn2 == 0.0) {  // identity reflector
                beta = alpha;
                tc = 0.0;
                sc = 1.0;
            } else {
                const double nrm = sqrt(alpha * alpha + xn2);
                beta = (alpha >= 0.0) ? -nrm : nrm;
                tc = (beta - alpha) / beta;
                sc = 1.0 / (alpha - beta);
            }
            double v[S];
            double* dst = C + static_cast<int64_t>(c) * s;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const int r = lane + q * kWave;
                const double tail = col[I][q] * sc;
                if (r < s) dst[r] = (r < c) ? col[I][q] : (r == c ? beta : tail);
                v[q] = (r > c) ? tail : (r == c ? 1.0 : 0.0);
            }
            if (lane == 0) tau[c] = tc;
            if (tc != 0.0) apply_reflector_cols<I + 1, S, CB>(col, v, tc);
        }
        factor_held<I + 1, S, CB>(col, c0, dc, s, lane, C, tau);
    }
}

template <int S>
__global__ __launch_bounds__(kPipeBlock) void lsq_pipeline_kernel(int s, const int* __restrict__ dc_dev, int dc_host,
                                                                  double* __restrict__ C, double* __restrict__ g,
                                                                  double* __restrict__ tau, double kappa_max,
                                                                  double* __restrict__ y, double* __restrict__ dout,
                                                                  int* __restrict__ iout, LsqSync* sync, int* abort,
                                                                  uint64_t limit) {
    constexpr int CB = kPipeCols;
    const int dc = dc_dev ? *dc_dev : dc_host;
    const int lane = threadIdx.x & (kWave - 1);
    const int c0 = (blockIdx.x * kPipeWaves + threadIdx.x / kWave) * CB;
    if (c0 > dc) return;
    const int ncol = min(CB, dc + 1 - c0);  // columns held (column dc is g); the rest stay zero
    double col[CB][S];
#pragma unroll
    for (int i = 0; i < CB; ++i) {
        const int c = min(c0 + i, dc);  // columns past dc read g and are then zeroed
        const double* src = (c < dc) ? C + static_cast<int64_t>(c) * s : g;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int r = lane + q * kWave;
            const double x = src[min(r, s - 1)];
            col[i][q] = (i < ncol && r < s) ? x : 0.0;
        }
    }

    // reflectors of earlier wavefronts, applied in order as they are published;
    // kBatch of them are loaded together so their loads overlap
    constexpr int kBatch = 4;
    const int pmax = min(c0, dc);
    unsigned avail = 0;
    for (int p0 = 0; p0 < pmax; p0 += kBatch) {
        const int pend = min(p0 + kBatch, pmax);
        if (static_cast<unsigned>(pend) > avail) {
            const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
            while ((avail = __hip_atomic_load(&sync->npub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) <
                   static_cast<unsigned>(pend)) {
                if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
                if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
                    __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    return;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        double v[kBatch][S];
        double tb[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int p = p0 + b;
            tb[b] = (p < pend) ? tau[p] : 0.0;
            // past the batch: a zero reflector (the address stays inside column pend - 1)
            load_reflector<S>(v[b], C + static_cast<int64_t>(min(p, pend - 1)) * s, p, s, lane, p < pend);
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
            if (tb[b] != 0.0) apply_reflector_cols<0, S, CB>(col, v[b], tb[b]);
    }

    // local factorisation of the held columns below dc
    factor_held<0, S, CB>(col, c0, dc, s, lane, C, tau);
    if (c0 < dc && lane == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&sync->npub, static_cast<unsigned>(min(c0 + CB, dc)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (dc >= c0 + CB) return;

    // ---- holder of g: Q^T g out, kappa guard, back substitution, r_est --------
    double z[S];
#pragma unroll
    for (int i = 0; i < CB; ++i)
        if (c0 + i == dc)
#pragma unroll
            for (int q = 0; q < S; ++q) z[q] = col[i][q];
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const int r = lane + q * kWave;
        if (r < s) g[r] = z[q];
    }
    // diagonal of T, one entry per lane-slot (all loads in flight together)
    double dg[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const int j = lane + q * kWave;
        dg[q] = (j < dc) ? fabs(C[static_cast<int64_t>(j) * s + j]) : 0.0;
    }
    int d_eff = 0;
    double tmax = 0.0, tmin = INFINITY, kap = 0.0;
    for (int j = 0; j < dc; ++j) {
        const double a = row_of<S>(dg, j);
        const double nmax = a > tmax ? a : tmax;
        const double nmin = a < tmin ? a : tmin;
        if (!(nmin > 0.0) || nmax / nmin > kappa_max) break;
        tmax = nmax;
        tmin = nmin;
        kap = tmax / tmin;
        d_eff = j + 1;
    }
    double rl = 0.0;
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const int r = lane + q * kWave;
        if (r >= d_eff && r < s) rl += z[q] * z[q];
    }
    const double rest = sqrt(wave_sum(rl));
    // back substitution, column-oriented; the next columns of T are fetched
    // kPrefetch steps ahead so the loads overlap the updates
    constexpr int kPrefetch = 4;
    double tc[kPrefetch][S];
    double td[kPrefetch];
#pragma unroll
    for (int f = 0; f < kPrefetch; ++f) {
        const int i = d_eff - 1 - f;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int r = lane + q * kWave;
            tc[f][q] = (i >= 0 && r < i) ? C[static_cast<int64_t>(i) * s + r] : 0.0;
        }
        td[f] = (i >= 0) ? C[static_cast<int64_t>(i) * s + i] : 1.0;
    }
    for (int i0 = d_eff - 1; i0 >= 0; i0 -= kPrefetch) {
#pragma unroll
        for (int f = 0; f < kPrefetch; ++f) {
            const int i = i0 - f;
            if (i >= 0) {
                const double zi = row_of<S>(z, i);
                const double yi = zi / td[f];
                if (lane == 0) y[i] = yi;
#pragma unroll
                for (int q = 0; q < S; ++q)
                    if (lane + q * kWave < i) z[q] -= tc[f][q] * yi;
            }
            // refill slot f with column i - kPrefetch
            const int inext = i - kPrefetch;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const int r = lane + q * kWave;
                tc[f][q] = (inext >= 0 && r < inext) ? C[static_cast<int64_t>(inext) * s + r] : 0.0;
            }
            td[f] = (inext >= 0) ? C[static_cast<int64_t>(inext) * s + inext] : 1.0;
        }
    }
    if (lane == 0) {
        dout[0] = rest;
        dout[1] = kap;
        iout[0] = d_eff;
        if (d_eff < dc) iout[1] |= SGMRES_FLAG_KAPPA_TRUNC;
    }
}

}  // namespace

hipError_t launch_lsq(int s, const int* dc_dev, int dc_host, double* C, double* g, double kappa_max,
                      double* y, double* dout, int* iout, hipStream_t stream) {
    lsq_kernel<<<1, kLsqBlock, sizeof(double) * s, stream>>>(s, dc_dev, dc_host, C, g, kappa_max, y, dout, iout);
    return hipGetLastError();
}

hipError_t launch_lsq_batched(int nsys, int s, const BatchSys* sys, BatchState* st, double kappa_max,
                              hipStream_t stream) {
    if (nsys <= 0) return hipSuccess;
    lsq_batched_kernel<<<nsys, kLsqBlock, sizeof(double) * s, stream>>>(s, sys, st, kappa_max);
    return hipGetLastError();
}

size_t lsq_sync_bytes() { return sizeof(LsqSync); }

hipError_t launch_lsq_pipeline(int s, int d_max, const int* dc_dev, int dc_host, double* C, double* g, double* tau,
                               double kappa_max, double* y, double* dout, int* iout, void* sync, int* abort,
                               uint64_t limit, hipStream_t stream) {
    const int slots = (s + kWave - 1) / kWave;
    const void* fn = nullptr;
    if (slots <= 1) fn = reinterpret_cast<const void*>(lsq_pipeline_kernel<1>);
    else if (slots <= 2) fn = reinterpret_cast<const void*>(lsq_pipeline_kernel<2>);
    else if (slots <= 4) fn = reinterpret_cast<const void*>(lsq_pipeline_kernel<4>);
    else if (slots <= 8) fn = reinterpret_cast<const void*>(lsq_pipeline_kernel<8>);
    else return hipErrorInvalidValue;
    hipError_t err = hipMemsetAsync(sync, 0, sizeof(LsqSync), stream);
    if (err != hipSuccess) return err;
    const int waves = (d_max + 1 + kPipeCols - 1) / kPipeCols;
    const int blocks = (waves + kPipeWaves - 1) / kPipeWaves;
    LsqSync* sp = static_cast<LsqSync*>(sync);
    void* args[] = {&s, &dc_dev, &dc_host, &C, &g, &tau, &kappa_max, &y, &dout, &iout, &sp, &abort, &limit};
    return hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(kPipeBlock), args, 0, stream);
}

}  // namespace sg
