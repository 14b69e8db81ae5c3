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
        for (int i = p + 1 + tid; i < s; i += kLsqBlock) t = madd(cp[i], cp[i], t);
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
                const double nrm = sqrt(madd(alpha, alpha, xn2));
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
                for (int i = p + 1 + lane; i < s; i += kWave) sd = madd(v[i], col[i], sd);
                sd = wave_sum(sd);
                const double head = col[p];
                sd = (head + sd) * tau;
                for (int i = p + 1 + lane; i < s; i += kWave) col[i] = madd(-sd, v[i], col[i]);
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
                if (q < i) z[c] = madd(-tcol[q], yi, z[c]);
            }
        }
    }

    double t = 0.0;
    for (int i = d_eff + tid; i < s; i += kLsqBlock) t = madd(g[i], g[i], t);
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

// One workgroup per system of a batch (system idx[b] for workgroup b when idx
// is given); systems no longer active are skipped.
__global__ __launch_bounds__(kLsqBlock) void lsq_batched_kernel(int s, const BatchSys* __restrict__ sys,
                                                                BatchState* __restrict__ st, double kappa_max,
                                                                const int* __restrict__ idx) {
    extern __shared__ double v[];
    const int i = idx ? idx[blockIdx.x] : static_cast<int>(blockIdx.x);
    BatchState* t = st + i;
    if (t->status != 0 || t->next != 0) return;  // only systems that built a basis this cycle
    const BatchSys& S = sys[i];
    lsq_body(s, t->dc, S.SAB, S.g, kappa_max, S.y, &t->rest, &t->d_eff, v);
}

// ---------------------------------------------------------------------------
// Column-owner pipeline (s <= 64 S).  Wavefront w keeps columns
// [CB w, CB w + CB) of C -- column dc stands for g -- in registers for the
// whole factorisation; a workgroup holds kPipeWaves consecutive wavefronts, so
// BC = kPipeWaves CB consecutive columns.  A wavefront applies, in order, the
// reflectors of the earlier workgroups (announced by a device-wide counter and
// loaded from C) and then those of the earlier wavefronts of its own workgroup
// (announced one by one by a counter in LDS and read from an LDS copy), and
// factors its own columns: each new reflector is copied to LDS and announced at
// once, written to C, and applied to the wavefront's later columns.  Every
// column thus sees the reflectors in the order of the one-workgroup kernel
// above, and a hand-over between wavefronts of one workgroup costs an LDS
// round trip instead of a device-wide release and acquire.  When its columns
// are done a wavefront publishes them device-wide, in wavefront order (it
// first waits for its predecessor's publication, so its release covers every
// earlier reflector).  The wavefront holding g finishes with the kappa guard,
// the back substitution and the residual estimate.  Launched cooperatively
// (all wavefronts resident); every wait is bounded by a real-time limit.
// ---------------------------------------------------------------------------
constexpr int kPipeWaves = 8;
constexpr int kPipeBlock = kPipeWaves * kWave;
constexpr int kPipeCols = 4;                     // columns per wavefront
constexpr int kPipeBC = kPipeWaves * kPipeCols;  // columns per workgroup

struct LsqSync {
    unsigned npub;  // reflectors published device-wide (monotone, in order)
    unsigned pad[63];
};

// Bounded waits for *p >= target; false (abort raised or seen) on time-out.
__device__ __forceinline__ bool lsq_spin_global(unsigned* p, unsigned target, int* abort, uint64_t limit) {
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
__device__ __forceinline__ unsigned lsq_spin_lds(unsigned* p, unsigned target, int* abort, uint64_t limit) {
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    unsigned v;
    unsigned it = 0;
    while ((v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) < target) {
        if ((++it & 255u) == 0 && __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return 0;
        if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
            __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return 0;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    return v;
}

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
        // the load is used unconditionally (a 0/1 factor rather than a select),
        // so the compiler cannot sink it into a branch with its own wait; the
        // row is clamped into the column
        const double x = vp[min(r, s - 1)];
        v[q] = x * ((live && r > p && r < s) ? 1.0 : 0.0) + ((live && r == p) ? 1.0 : 0.0);
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
        for (int q = 0; q < S; ++q) a = madd(v[q], col[i][q], a);
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
        for (int q = 0; q < S; ++q) col[i][q] = madd(-t, v[q], col[i][q]);
    }
}

// LDS of the pipeline workgroup: the reflectors of its BC columns in register
// layout (slot q of lane l at (p * S + q) * 64 + l), their tau, and the count
// of reflectors announced.
template <int S>
struct PipeLds {
    double* refl;
    double* tau;
    unsigned* pub;
    int bstart;  // first column of the workgroup
};

// Factor the held column I (global column c0 + I, if below dc): the new
// reflector goes to LDS and is announced, then to C and tau, and is applied at
// once to the held columns after it; then the next held column.  Unrolled at
// compile time over I.
template <int I, int S, int CB>
__device__ __forceinline__ void factor_held(double (&col)[CB][S], int c0, int dc, int s, int lane,
                                            double* __restrict__ C, double* __restrict__ tau, const PipeLds<S>& L) {
    if constexpr (I < CB) {
        const int c = c0 + I;
        if (c < dc) {
            double xl = 0.0;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const int r = lane + q * kWave;
                if (r > c) xl = madd(col[I][q], col[I][q], xl);
            }
            const double xn2 = wave_sum(xl);
            const double alpha = row_of<S>(col[I], c);
            double beta, tc, sc;
            if (xn2 == 0.0) {  // identity reflector
                beta = alpha;
                tc = 0.0;
                sc = 1.0;
            } else {
                const double nrm = sqrt(madd(alpha, alpha, xn2));
                beta = (alpha >= 0.0) ? -nrm : nrm;
                tc = (beta - alpha) / beta;
                sc = 1.0 / (alpha - beta);
            }
            double v[S];
            double* lv = L.refl + static_cast<int64_t>(c - L.bstart) * S * kWave;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const int r = lane + q * kWave;
                v[q] = (r > c) ? col[I][q] * sc : (r == c ? 1.0 : 0.0);
                lv[q * kWave + lane] = v[q];
            }
            if (lane == 0) L.tau[c - L.bstart] = tc;
            // announce to the later wavefronts of this workgroup (LDS order only;
            // the global stores below need not have landed)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
            if (lane == 0) __hip_atomic_store(L.pub, static_cast<unsigned>(c + 1), __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP);
            double* dst = C + static_cast<int64_t>(c) * s;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const int r = lane + q * kWave;
                if (r < s) dst[r] = (r < c) ? col[I][q] : (r == c ? beta : v[q]);
            }
            if (lane == 0) tau[c] = tc;
            if (tc != 0.0) apply_reflector_cols<I + 1, S, CB>(col, v, tc);
        }
        factor_held<I + 1, S, CB>(col, c0, dc, s, lane, C, tau, L);
    }
}

// One system's factorisation; blk: this workgroup's index among the system's.
template <int S>
__device__ __forceinline__ void lsq_pipeline_body(int blk, int s, const int* __restrict__ dc_dev, int dc_host,
                                                  double* __restrict__ C, double* __restrict__ g,
                                                  double* __restrict__ tau, double kappa_max,
                                                  double* __restrict__ y, double* __restrict__ dout,
                                                  int* __restrict__ iout, LsqSync* sync, int* abort,
                                                  uint64_t limit) {
    constexpr int CB = kPipeCols;
    extern __shared__ double lds[];
    __shared__ unsigned lpub;
    const int dc = dc_dev ? *dc_dev : dc_host;
    const int lane = threadIdx.x & (kWave - 1);
    const int bstart = blk * kPipeBC;
    const int c0 = bstart + (threadIdx.x / kWave) * CB;
    if (threadIdx.x == 0) lpub = static_cast<unsigned>(bstart);
    __syncthreads();
    if (c0 > dc) return;
    const PipeLds<S> L{lds, lds + kPipeBC * S * kWave, &lpub, bstart};
    const int ncol = min(CB, dc + 1 - c0);  // columns held (column dc is g); the rest stay zero
    double col[CB][S];
    // all loads issued together: addresses clamped into valid columns and the
    // values kept by a 0/1 factor, so no load sits behind a branch
#pragma unroll
    for (int i = 0; i < CB; ++i) {
        const int c = min(c0 + i, dc);  // columns past dc read g and are then zeroed
        const double* src = (c < dc) ? C + static_cast<int64_t>(c) * s : g;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int r = lane + q * kWave;
            col[i][q] = src[min(r, s - 1)] * ((i < ncol && r < s) ? 1.0 : 0.0);
        }
    }

    // reflectors of earlier workgroups, applied in order as they are published
    // device-wide; kBatch of them are loaded together so their loads overlap
    constexpr int kBatch = 4;
    const int pext = min(bstart, dc);
    unsigned avail = 0;
    for (int p0 = 0; p0 < pext; p0 += kBatch) {
        const int pend = min(p0 + kBatch, pext);
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
            tb[b] = (p < pend) ? tau[min(p, pend - 1)] : 0.0;
            // past the batch: a zero reflector (the address stays inside column pend - 1)
            load_reflector<S>(v[b], C + static_cast<int64_t>(min(p, pend - 1)) * s, p, s, lane, p < pend);
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
            if (tb[b] != 0.0) apply_reflector_cols<0, S, CB>(col, v[b], tb[b]);
    }

    // reflectors of the earlier wavefronts of this workgroup, from LDS as they
    // are announced
    const int pown = min(c0, dc);
    unsigned seen = static_cast<unsigned>(bstart);
    for (int p = bstart; p < pown; ++p) {
        if (seen <= static_cast<unsigned>(p)) {
            seen = lsq_spin_lds(&lpub, static_cast<unsigned>(p + 1), abort, limit);
            if (seen == 0) return;
        }
        const double* lv = L.refl + static_cast<int64_t>(p - bstart) * S * kWave;
        double v[S];
#pragma unroll
        for (int q = 0; q < S; ++q) v[q] = lv[q * kWave + lane];
        const double tp = L.tau[p - bstart];
        if (tp != 0.0) apply_reflector_cols<0, S, CB>(col, v, tp);
    }

    // local factorisation of the held columns below dc
    factor_held<0, S, CB>(col, c0, dc, s, lane, C, tau, L);
    // device-wide publication in wavefront order: after the predecessor's, one
    // release covers this wavefront's stores and (already written back) all
    // earlier ones
    if (c0 < dc && lane == 0) {
        if (!lsq_spin_global(&sync->npub, static_cast<unsigned>(c0), abort, limit)) return;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&sync->npub, static_cast<unsigned>(min(c0 + CB, dc)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (dc >= c0 + CB) return;

    // ---- holder of g: Q^T g out, kappa guard, back substitution, r_est --------
    // every earlier reflector published device-wide, then visible here
    {
        const bool ok = lsq_spin_global(&sync->npub, static_cast<unsigned>(c0), abort, limit);
        if (!ok) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
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
    // diagonal of T, one entry per lane-slot (all loads in flight together;
    // entries past dc repeat T_{dc-1,dc-1} and are never consulted)
    double dg[S], rinv[S];
    const int jlast = max(dc - 1, 0);
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const int jj = min(lane + q * kWave, jlast);
        const double t = C[static_cast<int64_t>(jj) * s + jj];
        dg[q] = fabs(t);
        rinv[q] = 1.0 / t;  // for the back substitution (inf where T_jj = 0: past d_eff)
    }
    // kappa guard: d_eff is the first j whose prefix 0..j has a zero diagonal
    // entry or max/min > kappa_max (dc if none).  Prefix max and min by a wave
    // scan per slot, carried across slots; the first violation by ballot.
    int d_eff = dc;
    double kap = 0.0;
    {
        double cmax = 0.0, cmin = INFINITY;
        double pmx[S], pmn[S];
#pragma unroll
        for (int q = 0; q < S; ++q) {
            double mx = dg[q], mn = dg[q];
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const double omx = __shfl_up(mx, off, kWave);
                const double omn = __shfl_up(mn, off, kWave);
                if (lane >= off) {
                    mx = omx > mx ? omx : mx;
                    mn = omn < mn ? omn : mn;
                }
            }
            mx = cmax > mx ? cmax : mx;
            mn = cmin < mn ? cmin : mn;
            pmx[q] = mx;
            pmn[q] = mn;
            cmax = readlane_d(mx, kWave - 1);
            cmin = readlane_d(mn, kWave - 1);
        }
        bool found = false;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int j = lane + q * kWave;
            const bool bad = j < dc && (!(pmn[q] > 0.0) || pmx[q] / pmn[q] > kappa_max);
            const unsigned long long m = __ballot(bad);
            if (!found && m != 0ull) {
                found = true;
                d_eff = q * kWave + __ffsll(static_cast<long long>(m)) - 1;
            }
        }
        if (d_eff > 0) {
            const int jk = d_eff - 1;
            double a = pmx[0], b = pmn[0];
#pragma unroll
            for (int q = 1; q < S; ++q)
                if ((jk >> 6) == q) {
                    a = pmx[q];
                    b = pmn[q];
                }
            kap = readlane_d(a, jk & (kWave - 1)) / readlane_d(b, jk & (kWave - 1));
        }
    }
    double rl = 0.0;
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const int r = lane + q * kWave;
        if (r >= d_eff && r < s) rl = madd(z[q], z[q], rl);
    }
    const double rest = sqrt(wave_sum(rl));
    // back substitution T y = z, column-oriented: y_i = z_i (1 / T_ii), the
    // reciprocals formed in parallel beforehand so no division sits on the
    // serial chain; then z -= T[:, i] y_i over the slots holding rows below
    // row i's slot (rows i and below are no longer read, so whole slots are
    // updated without row masks).  The loops run over slots at compile time,
    // so z_i is read straight from its register.  Columns of T sit in a ring of
    // 8 (column i in entry i mod 8), each refilled with column i - 8 right after
    // use; loads are unconditional (clamped to column 0 past the end).
    constexpr int kRing = 8;
    double tc[kRing][S];
    auto load_tcol = [&](int i, double (&dst)[S]) {
        const double* cp = C + static_cast<int64_t>(max(i, 0)) * s;
#pragma unroll
        for (int q = 0; q < S; ++q) dst[q] = cp[min(lane + q * kWave, s - 1)];
    };
#pragma unroll
    for (int u = 0; u < kRing; ++u) load_tcol(((d_eff - 1 - u) >> 3) * kRing + u, tc[u]);
#pragma unroll
    for (int q = S - 1; q >= 0; --q) {
        for (int gq = min((d_eff - 1) >> 3, 8 * q + 7); gq >= 8 * q; --gq) {
#pragma unroll
            for (int u = kRing - 1; u >= 0; --u) {
                const int i = kRing * gq + u;
                if (i < d_eff) {
                    const double yi = readlane_d(z[q], i & (kWave - 1)) * readlane_d(rinv[q], i & (kWave - 1));
                    if (lane == 0) y[i] = yi;
#pragma unroll
                    for (int qq = 0; qq <= q; ++qq) z[qq] = madd(-tc[u][qq], yi, z[qq]);
                }
                load_tcol(i - kRing, tc[u]);
            }
        }
    }
    if (lane == 0) {
        dout[0] = rest;
        dout[1] = kap;
        iout[0] = d_eff;
        if (d_eff < dc) iout[1] |= SGMRES_FLAG_KAPPA_TRUNC;
    }
}

template <int S>
__global__ __launch_bounds__(kPipeBlock) void lsq_pipeline_kernel(int s, const int* __restrict__ dc_dev, int dc_host,
                                                                  double* __restrict__ C, double* __restrict__ g,
                                                                  double* __restrict__ tau, double kappa_max,
                                                                  double* __restrict__ y, double* __restrict__ dout,
                                                                  int* __restrict__ iout, LsqSync* sync, int* abort,
                                                                  uint64_t limit) {
    lsq_pipeline_body<S>(blockIdx.x, s, dc_dev, dc_host, C, g, tau, kappa_max, y, dout, iout, sync, abort, limit);
}

// Several systems' factorisations in one launch: workgroups [j nblk, (j+1)
// nblk) factor system jobs[j]; each system has its own publication counter.
template <int S>
__global__ __launch_bounds__(kPipeBlock) void lsq_pipeline_batched_kernel(int s, int nblk,
                                                                          const LsqJob* __restrict__ jobs,
                                                                          double kappa_max, int* abort,
                                                                          uint64_t limit) {
    const int j = blockIdx.x / nblk;
    const LsqJob& J = jobs[j];
    lsq_pipeline_body<S>(blockIdx.x - j * nblk, s, J.dc, 0, J.C, J.g, J.tau, kappa_max, J.y, J.dout, J.iout,
                         static_cast<LsqSync*>(J.sync), abort, limit);
}

}  // namespace

hipError_t launch_lsq(int s, const int* dc_dev, int dc_host, double* C, double* g, double kappa_max,
                      double* y, double* dout, int* iout, hipStream_t stream) {
    lsq_kernel<<<1, kLsqBlock, sizeof(double) * s, stream>>>(s, dc_dev, dc_host, C, g, kappa_max, y, dout, iout);
    return hipGetLastError();
}

hipError_t launch_lsq_batched(int nsys, int s, const BatchSys* sys, BatchState* st, double kappa_max,
                              hipStream_t stream, const int* idx) {
    if (nsys <= 0) return hipSuccess;
    lsq_batched_kernel<<<nsys, kLsqBlock, sizeof(double) * s, stream>>>(s, sys, st, kappa_max, idx);
    return hipGetLastError();
}

size_t lsq_sync_bytes() { return sizeof(LsqSync); }

hipError_t launch_lsq_pipeline(int s, int d_max, const int* dc_dev, int dc_host, double* C, double* g, double* tau,
                               double kappa_max, double* y, double* dout, int* iout, void* sync, int* abort,
                               uint64_t limit, hipStream_t stream) {
    const int slots = (s + kWave - 1) / kWave;
    const void* fn = nullptr;
    int S = 0;
    if (slots <= 1) fn = reinterpret_cast<const void*>(lsq_pipeline_kernel<1>), S = 1;
    else if (slots <= 2) fn = reinterpret_cast<const void*>(lsq_pipeline_kernel<2>), S = 2;
    else if (slots <= 4) fn = reinterpret_cast<const void*>(lsq_pipeline_kernel<4>), S = 4;
    else if (slots <= 8) fn = reinterpret_cast<const void*>(lsq_pipeline_kernel<8>), S = 8;
    else return hipErrorInvalidValue;
    const size_t lds = sizeof(double) * static_cast<size_t>(kPipeBC) * (S * kWave + 1);
    hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (err != hipSuccess) return err;
    err = hipMemsetAsync(sync, 0, sizeof(LsqSync), stream);
    if (err != hipSuccess) return err;
    const int blocks = (d_max + 1 + kPipeBC - 1) / kPipeBC;
    LsqSync* sp = static_cast<LsqSync*>(sync);
    void* args[] = {&s, &dc_dev, &dc_host, &C, &g, &tau, &kappa_max, &y, &dout, &iout, &sp, &abort, &limit};
    return hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(kPipeBlock), args, static_cast<unsigned>(lds), stream);
}

hipError_t launch_lsq_pipeline_batched(int njobs, int s, int d_max, const LsqJob* jobs, void* syncs, double kappa_max,
                                       int* abort, uint64_t limit, hipStream_t stream) {
    if (njobs <= 0) return hipSuccess;
    const int slots = (s + kWave - 1) / kWave;
    const void* fn = nullptr;
    int S = 0;
    if (slots <= 1) fn = reinterpret_cast<const void*>(lsq_pipeline_batched_kernel<1>), S = 1;
    else if (slots <= 2) fn = reinterpret_cast<const void*>(lsq_pipeline_batched_kernel<2>), S = 2;
    else if (slots <= 4) fn = reinterpret_cast<const void*>(lsq_pipeline_batched_kernel<4>), S = 4;
    else if (slots <= 8) fn = reinterpret_cast<const void*>(lsq_pipeline_batched_kernel<8>), S = 8;
    else return hipErrorInvalidValue;
    const size_t lds = sizeof(double) * static_cast<size_t>(kPipeBC) * (S * kWave + 1);
    hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (err != hipSuccess) return err;
    // the publication counters start at zero (a fill kernel: capture-safe)
    err = launch_fill_u32(static_cast<unsigned*>(syncs),
                          static_cast<int64_t>(njobs) * static_cast<int64_t>(sizeof(LsqSync) / sizeof(unsigned)), 0u,
                          stream);
    if (err != hipSuccess) return err;
    int nblk = (d_max + 1 + kPipeBC - 1) / kPipeBC;
    void* args[] = {&s, &nblk, &jobs, &kappa_max, &abort, &limit};
    return hipLaunchCooperativeKernel(fn, dim3(njobs * nblk), dim3(kPipeBlock), args, static_cast<unsigned>(lds),
                                      stream);
}

}  // namespace sg
