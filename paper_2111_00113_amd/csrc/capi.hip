// Host driver and C ABI of the sGMRES library (see include/sgmres.h).
//
// One solve = repeated cycles of (arXiv:2111.00113 Algorithm 1; Section 3.5):
//   residual r = b - A x and |r|     -> one 64-byte device->host read per cycle
//   persistent basis + sketch kernel (b_1 .. b_d, S B, S A B, g = S r)
//   sketched least squares (Householder QR, kappa guard, back substitution)
//   x <- x + B y
// All coefficients stay on the device; the host reads the residual norm (stop
// test) and the previous cycle's counters once per cycle.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/sgmres.h"
#include "internal.hpp"

namespace sg {
namespace {

constexpr uint64_t kSpinLimitTicks = 200000000ull;  // 2 s of the 100 MHz real-time counter
constexpr int kMaxD = kLsqMaxCols;
constexpr int kMaxS = 4096;

// Scalars the kernels leave on the device; read back in one copy per cycle.
struct DevScalars {
    double beta;   // |r| of the current residual
    double rho;    // |r| / |b|
    double nf;     // |b|
    double rest;   // last sketched residual estimate
    double kappa;  // last diagonal ratio of T
    double pad0[3];
    int dc;         // columns built by the last basis cycle
    int flags;      // OR of breakdown flags
    int d_eff;      // columns used by the last least-squares solve
    int lsq_flags;  // OR of kappa-truncation flags
    int abort;      // grid-barrier wait limit hit
    int csr_bad;    // CSR validation failed
    int pad1[2];
    unsigned long long phase_ticks[8];  // basis-kernel phase timers (profile)
    int batch_ctr[4];                   // batched solve: cycle, queue, active, active last cycle
    unsigned long long offblock;        // nonzeros reaching outside their row's block
};

struct Workspace {
    double* r = nullptr;
    size_t r_cap = 0;
    double* B = nullptr;
    size_t B_cap = 0;
    double* SB = nullptr;
    size_t SB_cap = 0;
    double* SAB = nullptr;
    size_t SAB_cap = 0;
    double* H = nullptr;
    size_t H_cap = 0;
    double* g = nullptr;
    size_t g_cap = 0;
    double* y = nullptr;
    size_t y_cap = 0;
    double* tau = nullptr;
    size_t tau_cap = 0;
    unsigned* lsq_sync = nullptr;
    // tagged partials of the Arnoldi steps' two reductions, two words each:
    // part_a then part_b, (k+1) x G each, cleared together before a launch
    unsigned long long* part_ab = nullptr;
    size_t part_ab_cap = 0;
    double* part_sk = nullptr;
    size_t part_sk_cap = 0;
    double* part_vec = nullptr;
    size_t part_vec_cap = 0;
    double* part_nrm = nullptr;  // Chebyshev column-norm partials, d x G
    size_t part_nrm_cap = 0;
    double* colnorm = nullptr;  // Chebyshev column norms, d
    size_t colnorm_cap = 0;
    float* valf = nullptr;  // FP32 copy of A's values (mixed-precision cycles)
    size_t valf_cap = 0;
    // two-barrier Arnoldi: halo buffer (n 64-bit words: tagged entries of the
    // rows other blocks gather, or w), and the bitmap of those rows
    unsigned long long* hbuf = nullptr;
    size_t hbuf_cap = 0;
    unsigned* xbits = nullptr;
    size_t xbits_cap = 0;
    // sliced ELL copy of A for the resident basis kernels
    int* sell_K = nullptr;
    size_t sell_K_cap = 0;
    int64_t* sell_sp = nullptr;
    size_t sell_sp_cap = 0;
    int32_t* sell_col = nullptr;
    size_t sell_col_cap = 0;
    double* sell_val = nullptr;  // doubles or floats
    size_t sell_val_cap = 0;
    // batched solve: descriptors, states, order, and one arena for every
    // system's basis, scratch vectors, sketch lists and small matrices
    BatchSys* bt_sys = nullptr;
    size_t bt_sys_cap = 0;
    BatchState* bt_st = nullptr;
    size_t bt_st_cap = 0;
    BatchTask* bt_task = nullptr;
    size_t bt_task_cap = 0;
    double* bt_slots = nullptr;
    size_t bt_slots_cap = 0;
    int64_t* bt_slot_off = nullptr;
    size_t bt_slot_off_cap = 0;
    unsigned* bt_gcnt = nullptr;
    size_t bt_gcnt_cap = 0;
    unsigned char* bt_arena = nullptr;
    size_t bt_arena_cap = 0;
    hipStream_t capture_stream = nullptr;
    // batched solve, several systems per resident basis launch: persistent
    // per-system arena (sliced ELL copies, residuals, small matrices), the
    // per-wave basis / partial-sum / barrier arena, descriptors
    unsigned char* wv_sys_arena = nullptr;
    size_t wv_sys_arena_cap = 0;
    unsigned char* wv_wave_arena = nullptr;
    size_t wv_wave_arena_cap = 0;
    int* wv_K = nullptr;
    size_t wv_K_cap = 0;
    ArnoldiParams* wv_ps = nullptr;
    size_t wv_ps_cap = 0;
    int* wv_idx = nullptr;  // per wave: group of each logical block, then the system of each group
    size_t wv_idx_cap = 0;
    BatchSys* wv_sys = nullptr;
    size_t wv_sys_cap = 0;
    BatchState* wv_st = nullptr;
    size_t wv_st_cap = 0;
    LsqJob* wv_jobs = nullptr;
    size_t wv_jobs_cap = 0;
    TailJob* wv_tail = nullptr;  // per wave: the systems' combine, residual and norm
    size_t wv_tail_cap = 0;
    TailJob* wv_tail0 = nullptr;  // the systems' |b| and first residual
    size_t wv_tail0_cap = 0;
    SellJob* wv_sell = nullptr;  // the systems' sliced ELL builds
    size_t wv_sell_cap = 0;
    int64_t* wv_sp = nullptr;  // the systems' sliced ELL slice starts, one after another
    size_t wv_sp_cap = 0;
    double* wv_tpart = nullptr;  // their residual block partials (one wave at a time)
    size_t wv_tpart_cap = 0;
    unsigned* sync = nullptr;  // grid-barrier words of the basis kernel
    DevScalars* sc = nullptr;
    DevScalars* host_sc = nullptr;  // pinned
    int32_t* t_rp = nullptr;
    size_t t_rp_cap = 0;
    int32_t* t_ci = nullptr;
    size_t t_ci_cap = 0;
    double* t_val = nullptr;
    size_t t_val_cap = 0;
    int32_t* t_scratch = nullptr;
    size_t t_scratch_cap = 0;
    // streaming path: per-chunk sketch lists, block partials of S B, the m / w
    // state buffer (HBM-state instances)
    uint32_t* st_lists = nullptr;
    size_t st_lists_cap = 0;
    double* st_part = nullptr;
    size_t st_part_cap = 0;
    double* st_state = nullptr;
    size_t st_state_cap = 0;
    // block of right-hand sides: interleaved F, X, R; per right-hand side
    // scalars and counters; pointer tables for pack / unpack
    double* mr_F = nullptr;
    size_t mr_F_cap = 0;
    double* mr_X = nullptr;
    size_t mr_X_cap = 0;
    double* mr_R = nullptr;
    size_t mr_R_cap = 0;
    double* mr_part = nullptr;
    size_t mr_part_cap = 0;
    double* mr_scal = nullptr;  // nf, beta, rho, beta for the kernel (32 each), rest / kappa pairs (64)
    size_t mr_scal_cap = 0;
    int* mr_int = nullptr;  // dc (32), flags (32), d_eff / lsq flags pairs (64)
    size_t mr_int_cap = 0;
    void** mr_ptr = nullptr;  // 32 sources, 32 destinations
    size_t mr_ptr_cap = 0;
    // the sliced ELL copy the basis kernels read this call: the workspace's own
    // (build_sell) or a plan's
    const int64_t* cur_sp = nullptr;
    const int32_t* cur_col = nullptr;
    const void* cur_val = nullptr;
};

// Sliced ELL copy of one matrix with values in one arithmetic type (plan-owned).
struct SellCopy {
    int64_t* sp = nullptr;
    int32_t* col = nullptr;
    void* val = nullptr;
};

// A matrix's cached set-up (sgmres_plan_create): validated once, its sliced ELL
// copies and optionally CSR(A^T) with its copies.
struct Plan {
    int device = 0;
    int flags = 0;
    sgmres_csr_t A{};
    sgmres_csr_t At{};
    int32_t* t_rp = nullptr;
    int32_t* t_ci = nullptr;
    double* t_val = nullptr;
    SellCopy sell[2][2];  // [A, A^T][FP64 values, FP32 values]
};

std::mutex g_mutex;
std::unordered_map<int, Workspace> g_ws;

template <typename T>
hipError_t ensure(T*& p, size_t& cap, size_t need) {
    if (need == 0) need = 1;
    if (p && cap >= need) return hipSuccess;
    if (p) {
        hipError_t e = hipFree(p);
        if (e != hipSuccess) return e;
        p = nullptr;
        cap = 0;
    }
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), sizeof(T) * need);
    if (e != hipSuccess) {
        p = nullptr;
        return e;
    }
    cap = need;
    return hipSuccess;
}

int to_code(hipError_t e) {
    if (e == hipSuccess) return SGMRES_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SGMRES_ENOMEM;
    return SGMRES_EHIP;
}

#define SG_TRY(expr)                                  \
    do {                                              \
        hipError_t sg_e_ = (expr);                    \
        if (sg_e_ != hipSuccess) return to_code(sg_e_); \
    } while (0)

int workspace(Workspace** out) {
    int dev = 0;
    SG_TRY(hipGetDevice(&dev));
    Workspace& ws = g_ws[dev];
    if (!ws.sc) {
        SG_TRY(hipMalloc(reinterpret_cast<void**>(&ws.sc), sizeof(DevScalars)));
        SG_TRY(hipMemset(ws.sc, 0, sizeof(DevScalars)));
        SG_TRY(hipMalloc(reinterpret_cast<void**>(&ws.sync), sync_words_bytes()));
        SG_TRY(hipMalloc(reinterpret_cast<void**>(&ws.lsq_sync), lsq_sync_bytes()));
        hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&ws.host_sc), sizeof(DevScalars),
                                     hipHostMallocDefault);
        if (e != hipSuccess) return SGMRES_ENOMEM;
        std::memset(ws.host_sc, 0, sizeof(DevScalars));
    }
    *out = &ws;
    return SGMRES_OK;
}

bool csr_ok(const sgmres_csr_t* A) {
    return A && A->n >= 1 && A->n < (int64_t(1) << 31) - 1 && A->nnz >= 0 && A->nnz < (int64_t(1) << 31) &&
           A->row_ptr && (A->nnz == 0 || (A->col_idx && A->val));
}

bool bad_sizes(int64_t n, int d, int k, int s, int zeta) {
    return d < 1 || d > n || d > kMaxD || k < 1 || s < d + 1 || s > kMaxS || zeta < 1 || zeta > s ||
           zeta > kMaxZeta;
}

struct SolveArgs {
    sgmres_csr_t A;
    const double* b;
    double* x;
    int d, k, s, zeta;
    uint64_t seed;
    double tol;
    int restarts;
    double kappa_max;
    int block, rows_per_thread;
    int profile;
    int per_block_release;
    int spmv_mode;
    int basis;  // SGMRES_BASIS_*
    double cheb_c, cheb_dx, cheb_dy;
    int precision;  // SGMRES_PREC_*
    int halo_off;   // nonzero: three grid barriers per Arnoldi step always
    int path;       // 0 auto, SGMRES_PATH_STREAM / SGMRES_PATH_PART_SPLIT forced
    int stream_state;  // 0 auto, 1 registers, 2 HBM buffer
    const Plan* plan;  // null, or the plan whose copies of A (or A^T) the solve reads
    int plan_t;        // with a plan: 1 for A^T
    hipStream_t stream;
};

// A was validated and its sliced ELL copy built by a plan: point the workspace
// at the copy for this precision (SGMRES_EINVAL when the plan lacks it).
int use_plan_sell(Workspace& ws, const SolveArgs& a) {
    const SellCopy& c = a.plan->sell[a.plan_t][a.precision == SGMRES_PREC_FP64 ? 0 : 1];
    if (!c.sp) return SGMRES_EINVAL;
    ws.cur_sp = c.sp;
    ws.cur_col = c.col;
    ws.cur_val = c.val;
    return SGMRES_OK;
}

// Coefficients of the rescaled Chebyshev recurrence for the box [c +- dx, +-dy]
// (Section 4.4): with rho = max(dx, dy), gamma = (dx^2 - dy^2) / (4 rho^2) and
// the per-step rescale kappa = 2 rho / (dx + dy),
//   bt_2 = (kappa / (2 rho)) (A - c) bt_1,
//   bt_{j+1} = (kappa / rho) (A - c) bt_j - kappa^2 gamma bt_{j-1}.
struct ChebCoef {
    double c, a1, a, q;
};

bool cheb_coefficients(double c, double dx, double dy, ChebCoef* out) {
    if (!std::isfinite(c) || !std::isfinite(dx) || !std::isfinite(dy) || dx < 0.0 || dy < 0.0) return false;
    const double rho = dx > dy ? dx : dy;
    if (!(rho > 0.0)) return false;
    const double kap = 2.0 * rho / (dx + dy);
    const double gam = (dx * dx - dy * dy) / (4.0 * rho * rho);
    out->c = c;
    out->a1 = kap / (2.0 * rho);
    out->a = kap / rho;
    out->q = kap * kap * gam;
    return true;
}

// HIP events bracketing the kernels of one cycle (profiling only).
struct CycleEvents {
    hipEvent_t r0 = nullptr, r1 = nullptr, b0 = nullptr, b1 = nullptr, l1 = nullptr, c1 = nullptr, k1 = nullptr;
    bool on = false;
    hipError_t create() {
        hipEvent_t* all[] = {&r0, &r1, &b0, &b1, &l1, &c1, &k1};
        for (hipEvent_t* e : all) {
            hipError_t err = hipEventCreate(e);
            if (err != hipSuccess) return err;
        }
        on = true;
        return hipSuccess;
    }
    ~CycleEvents() {
        hipEvent_t all[] = {r0, r1, b0, b1, l1, c1, k1};
        for (hipEvent_t e : all)
            if (e) (void)hipEventDestroy(e);
    }
    static double ms(hipEvent_t a, hipEvent_t b) {
        float t = 0.0f;
        return hipEventElapsedTime(&t, a, b) == hipSuccess ? static_cast<double>(t) : 0.0;
    }
};

int copy_scalars(Workspace& ws, hipStream_t stream) {
    SG_TRY(hipMemcpyAsync(ws.host_sc, ws.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, stream));
    SG_TRY(hipStreamSynchronize(stream));
    return SGMRES_OK;
}

// Sliced ELL copy of A (sell.hip) with values in the basis arithmetic type.
int build_sell(Workspace& ws, const sgmres_csr_t& A, int precision, hipStream_t st) {
    const int64_t n = A.n;
    const int64_t nsl = (n + 63) / 64;
    SG_TRY(ensure(ws.sell_K, ws.sell_K_cap, static_cast<size_t>(nsl)));
    SG_TRY(ensure(ws.sell_sp, ws.sell_sp_cap, static_cast<size_t>(nsl + 1)));
    SG_TRY(launch_sell_width(n, A.row_ptr, ws.sell_K, st));
    std::vector<int> K(static_cast<size_t>(nsl));
    SG_TRY(hipMemcpyAsync(K.data(), ws.sell_K, sizeof(int) * nsl, hipMemcpyDeviceToHost, st));
    SG_TRY(hipStreamSynchronize(st));
    std::vector<int64_t> sp(static_cast<size_t>(nsl + 1), 0);
    for (int64_t i = 0; i < nsl; ++i) sp[i + 1] = sp[i] + 64 * static_cast<int64_t>(K[i]);
    const int64_t total = sp[nsl] > 0 ? sp[nsl] : 1;
    SG_TRY(ensure(ws.sell_col, ws.sell_col_cap, static_cast<size_t>(total)));
    const size_t es = precision == SGMRES_PREC_FP64 ? 8 : 4;
    SG_TRY(ensure(ws.sell_val, ws.sell_val_cap, (static_cast<size_t>(total) * es + 7) / 8));
    SG_TRY(hipMemcpyAsync(ws.sell_sp, sp.data(), sizeof(int64_t) * (nsl + 1), hipMemcpyHostToDevice, st));
    SG_TRY(launch_sell_fill(n, A.row_ptr, A.col_idx, A.val, ws.sell_sp, ws.sell_col, ws.sell_val, precision, st));
    SG_TRY(hipStreamSynchronize(st));  // sp (host vector) is read by the copy above
    ws.cur_sp = ws.sell_sp;
    ws.cur_col = ws.sell_col;
    ws.cur_val = ws.sell_val;
    return SGMRES_OK;
}

// The same copy into plan-owned arrays (K: nsl ints of scratch).
int build_sell_copy(SellCopy& c, int* K_dev, const sgmres_csr_t& A, int precision, hipStream_t st) {
    const int64_t n = A.n;
    const int64_t nsl = (n + 63) / 64;
    SG_TRY(launch_sell_width(n, A.row_ptr, K_dev, st));
    std::vector<int> K(static_cast<size_t>(nsl));
    SG_TRY(hipMemcpyAsync(K.data(), K_dev, sizeof(int) * nsl, hipMemcpyDeviceToHost, st));
    SG_TRY(hipStreamSynchronize(st));
    std::vector<int64_t> sp(static_cast<size_t>(nsl + 1), 0);
    for (int64_t i = 0; i < nsl; ++i) sp[i + 1] = sp[i] + 64 * static_cast<int64_t>(K[i]);
    const int64_t total = sp[nsl] > 0 ? sp[nsl] : 1;
    const size_t es = precision == SGMRES_PREC_FP64 ? 8 : 4;
    SG_TRY(hipMalloc(reinterpret_cast<void**>(&c.sp), sizeof(int64_t) * (nsl + 1)));
    SG_TRY(hipMalloc(reinterpret_cast<void**>(&c.col), sizeof(int32_t) * total));
    SG_TRY(hipMalloc(&c.val, es * total));
    SG_TRY(hipMemcpyAsync(c.sp, sp.data(), sizeof(int64_t) * (nsl + 1), hipMemcpyHostToDevice, st));
    SG_TRY(launch_sell_fill(n, A.row_ptr, A.col_idx, A.val, c.sp, c.col, c.val, precision, st));
    SG_TRY(hipStreamSynchronize(st));
    return SGMRES_OK;
}


// One basis cycle on the residual in ws.r (norm already in ws.sc->beta).
// B is stored in the launch's basis type; A is read through the sliced ELL
// copy in ws (build_sell, same arithmetic type).
int run_cycle(Workspace& ws, const sgmres_csr_t& A, int d, int k, int s, int zeta, uint64_t seed,
              uint32_t cycle, const ArnoldiLaunch& L, void* B, int64_t ldb, double* SB, double* SAB,
              double* H, double* g, hipStream_t stream, hipEvent_t ev_start = nullptr,
              int per_block_release = 0, bool phase_timing = false, int spmv_mode = 0, int halo = 0) {
    SG_TRY(launch_fill_u32(ws.sync, static_cast<int64_t>(sync_words_bytes() / sizeof(unsigned)), 0u, stream));
    // halo mode (1: recomputed entries, 2: published entries, FP32
    // arithmetic, whose tags start at 1)
    if (halo == 2)
        SG_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(ws.hbuf), 2 * A.n, 0u, stream));
    // tags of the step partials start at 1: clear the slots of earlier launches
    SG_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(ws.part_ab), static_cast<int64_t>(8 * (k + 1)) * L.grid, 0u,
                           stream));
    if (ev_start) SG_TRY(hipEventRecord(ev_start, stream));
    ArnoldiParams p{};
    p.n = A.n;
    p.rp = A.row_ptr;
    p.sp = ws.cur_sp;
    p.ci = ws.cur_col;
    p.val = ws.cur_val;
    p.r = ws.r;
    p.beta = &ws.sc->beta;
    p.B = B;
    p.ldb = ldb;
    p.SB = SB;
    p.SAB = SAB;
    p.H = H;
    p.g = g;
    p.d = d;
    p.k = k;
    p.s = s;
    p.zeta = zeta;
    p.seed = seed;
    p.cycle = cycle;
    p.part_a = ws.part_ab;
    p.part_b = ws.part_ab + static_cast<int64_t>(2 * (k + 1)) * L.grid;
    p.part_sk = ws.part_sk;
    p.sync = ws.sync;
    p.per_block_release = per_block_release;
    p.abort = &ws.sc->abort;
    p.status = &ws.sc->dc;
    p.spin_limit = kSpinLimitTicks;
    p.phase_ticks = phase_timing ? ws.sc->phase_ticks : nullptr;
    p.spmv_mode = spmv_mode;
    p.hbuf = halo ? ws.hbuf : nullptr;
    p.xbits = halo ? ws.xbits : nullptr;
    SG_TRY(arnoldi_launch(L, p, stream));
    return SGMRES_OK;
}

// One Chebyshev basis cycle on the residual in ws.r (norm in ws.sc->beta).
int run_cheb_cycle(Workspace& ws, const sgmres_csr_t& A, int d, int s, int zeta, uint64_t seed, uint32_t cycle,
                   const ArnoldiLaunch& L, const ChebCoef& cf, void* B, int64_t ldb, double* SB, double* SAB,
                   double* colnorm, double* g, hipStream_t stream, hipEvent_t ev_start = nullptr,
                   int per_block_release = 0, bool phase_timing = false, int sketch_basis = 1) {
    SG_TRY(launch_fill_u32(ws.sync, static_cast<int64_t>(sync_words_bytes() / sizeof(unsigned)), 0u, stream));
    if (ev_start) SG_TRY(hipEventRecord(ev_start, stream));
    ChebParams p{};
    p.n = A.n;
    p.rp = A.row_ptr;
    p.sp = ws.cur_sp;
    p.ci = ws.cur_col;
    p.val = ws.cur_val;
    p.r = ws.r;
    p.beta = &ws.sc->beta;
    p.B = B;
    p.ldb = ldb;
    p.SB = SB;
    p.SAB = SAB;
    p.colnorm = colnorm;
    p.g = g;
    p.d = d;
    p.s = s;
    p.zeta = zeta;
    p.seed = seed;
    p.cycle = cycle;
    p.c = cf.c;
    p.a1 = cf.a1;
    p.a = cf.a;
    p.q = cf.q;
    p.part_sk = ws.part_sk;
    p.part_nrm = ws.part_nrm;
    p.sync = ws.sync;
    p.per_block_release = per_block_release;
    p.abort = &ws.sc->abort;
    p.status = &ws.sc->dc;
    p.spin_limit = kSpinLimitTicks;
    p.phase_ticks = phase_timing ? ws.sc->phase_ticks : nullptr;
    p.sketch_basis = sketch_basis;
    SG_TRY(chebyshev_launch(L, p, stream));
    return SGMRES_OK;
}

// Sketched least squares on C (s x dc): the column-owner pipeline when s fits
// its register layout, else the one-workgroup kernel.
int run_lsq(Workspace& ws, int s, int d_max, const int* dc_dev, int dc_host, double* C, double* g, double kappa_max,
            double* y, hipStream_t st) {
    if (s <= kLsqPipeMaxS) {
        SG_TRY(ensure(ws.tau, ws.tau_cap, static_cast<size_t>(d_max > 0 ? d_max : 1)));
        SG_TRY(launch_lsq_pipeline(s, d_max, dc_dev, dc_host, C, g, ws.tau, kappa_max, y, &ws.sc->rest,
                                   &ws.sc->d_eff, ws.lsq_sync, &ws.sc->abort, kSpinLimitTicks, st));
    } else {
        SG_TRY(launch_lsq(s, dc_dev, dc_host, C, g, kappa_max, y, &ws.sc->rest, &ws.sc->d_eff, st));
    }
    return SGMRES_OK;
}

// Validates the CSR arrays on the device (one pass over row_ptr and col_idx).
int check_csr(Workspace& ws, const sgmres_csr_t& A, hipStream_t st) {
    SG_TRY(hipMemsetAsync(&ws.sc->csr_bad, 0, sizeof(int), st));
    SG_TRY(launch_csr_check(A.n, A.nnz, A.row_ptr, A.col_idx, &ws.sc->csr_bad, st));
    int rc = copy_scalars(ws, st);
    if (rc) return rc;
    return ws.host_sc->csr_bad ? SGMRES_ECSR : SGMRES_OK;
}

// sketch_basis selects the kernel instance that also forms S B (the cycle
// entry point); the solve uses S A B and g only.
int prepare_arnoldi(Workspace& ws, int64_t n, int d, int k, int s, int zeta, int block, int rpt,
                    ArnoldiLaunch* L, int sketch_basis, int precision = SGMRES_PREC_FP64) {
    ArnoldiShape shape{n, d, k, s, zeta, block, rpt, 0, 0, sketch_basis, precision, 0};
    if (arnoldi_configure(shape, L) != hipSuccess) return SGMRES_EINVAL;
    SG_TRY(ensure(ws.part_ab, ws.part_ab_cap, static_cast<size_t>(4 * (k + 1)) * L->grid));
    SG_TRY(ensure(ws.part_sk, ws.part_sk_cap, static_cast<size_t>(2 * s * d + s) * L->grid));
    return SGMRES_OK;
}

int prepare_cheb(Workspace& ws, int64_t n, int d, int s, int zeta, int block, int rpt, ArnoldiLaunch* L,
                 int precision = SGMRES_PREC_FP64) {
    ArnoldiShape shape{n, d, 1, s, zeta, block, rpt, 0, 0, 0, precision, 0};
    if (chebyshev_configure(shape, L) != hipSuccess) return SGMRES_EINVAL;
    SG_TRY(ensure(ws.part_sk, ws.part_sk_cap, static_cast<size_t>(2 * s * d + s) * L->grid));
    SG_TRY(ensure(ws.part_nrm, ws.part_nrm_cap, static_cast<size_t>(d) * L->grid));
    return SGMRES_OK;
}

int batch_solve_locked(int nsys, const sgmres_system_t* systems, int d, int k, int s, uint64_t seed, double tol,
                       int restarts, const sgmres_options_t* opts, sgmres_batch_result_t* results, hipStream_t st,
                       BatchState* st_out);

// A system too large for the resident basis kernel (truncated Arnoldi, k <= 4):
// the part-split kernel of the batched solve, as a batch of one.
int solve_large(const SolveArgs& a, sgmres_info_t* info) {
    sgmres_system_t sys{a.A, a.b, a.x};
    sgmres_options_t o{};
    o.zeta = a.zeta;
    o.kappa_max = a.kappa_max;
    o.precision = a.precision;
    sgmres_batch_result_t r{};
    BatchState t{};
    const int rc = batch_solve_locked(1, &sys, a.d, a.k, a.s, a.seed, a.tol, a.restarts, &o, &r, a.stream, &t);
    if (rc < 0) return rc;
    if (info) {
        sgmres_info_t rep{};
        rep.cycles = r.cycles;
        rep.steps = r.steps;
        rep.d_eff_last = t.d_eff;
        rep.flags = r.flags;
        rep.relres = r.relres;
        rep.rest_est = t.nf > 0 ? t.rest / t.nf : 0.0;
        rep.kappa_est = t.kappa;
        if (r.cycles > 0) rep.path = SGMRES_PATH_PART_SPLIT;
        *info = rep;
    }
    return r.status;
}

// Truncated Arnoldi on the streaming basis kernel (systems beyond the resident
// kernels' capacity, or forced).  Per cycle: residual -> basis kernel (window
// read back from B, b_1 .. b_{d+1} and H) -> the cycle's sketch lists -> g = S r,
// S B of the d + 1 columns, S A B = (S B) H -> sketched least squares ->
// x += B y.  Caller holds g_mutex.
int solve_stream(const SolveArgs& a, Workspace& ws, sgmres_info_t* info) {
    const int64_t n = a.A.n;
    const int kk = (a.k > a.d - 1) ? (a.d > 1 ? a.d - 1 : 1) : a.k;
    hipStream_t st = a.stream;
    if (kk > kStreamMaxK || !basis_sketch_fits(n, a.s, a.zeta)) return SGMRES_EINVAL;
    StreamLaunch L{};
    if (stream_configure(n, 1, kk, a.precision, &L) != hipSuccess) return SGMRES_EINVAL;
    if (a.stream_state == 2 && !L.hst) {
        // HBM state requested: same tile size, one tile per workgroup up to the chip
        StreamLaunch H{};
        if (stream_configure(int64_t(1) << 40, 1, kk, a.precision, &H) != hipSuccess) return SGMRES_EINVAL;
        const int64_t tiles = (n + int64_t(H.P) * kStreamBlock - 1) / (int64_t(H.P) * kStreamBlock);
        H.grid = static_cast<int>(tiles < H.grid ? tiles : H.grid);
        L = H;
    } else if (a.stream_state == 1 && L.hst) {
        return SGMRES_EINVAL;
    }
    int rc = a.plan ? SGMRES_OK : check_csr(ws, a.A, st);
    if (rc) return rc;
    const size_t eb = basis_elem_bytes(a.precision);
    // columns padded to 128 entries (256-byte aligned), d + 1 of them
    const int64_t ldb = (n + 127) / 128 * 128;
    SG_TRY(ensure(ws.r, ws.r_cap, static_cast<size_t>(n)));
    SG_TRY(ensure(ws.B, ws.B_cap, (static_cast<size_t>(ldb) * (a.d + 1) * eb + 7) / 8));
    SG_TRY(ensure(ws.SB, ws.SB_cap, static_cast<size_t>(a.s) * (a.d + 1)));
    SG_TRY(ensure(ws.SAB, ws.SAB_cap, static_cast<size_t>(a.s) * a.d));
    SG_TRY(ensure(ws.H, ws.H_cap, static_cast<size_t>(kk + 1) * a.d));
    SG_TRY(ensure(ws.g, ws.g_cap, static_cast<size_t>(a.s)));
    SG_TRY(ensure(ws.y, ws.y_cap, static_cast<size_t>(a.d)));
    SG_TRY(ensure(ws.part_vec, ws.part_vec_cap, static_cast<size_t>(kMaxVecGrid)));
    SG_TRY(ensure(ws.part_ab, ws.part_ab_cap, static_cast<size_t>(4 * (kStreamMaxK + 1)) * L.grid));
    SG_TRY(ensure(ws.part_sk, ws.part_sk_cap, static_cast<size_t>(a.s) * sketch_grid(n)));
    SG_TRY(ensure(ws.st_lists, ws.st_lists_cap, static_cast<size_t>(basis_lists_words(n, a.s, a.zeta))));
    SG_TRY(ensure(ws.st_part, ws.st_part_cap,
                  static_cast<size_t>(basis_sketch_grid(n)) * (a.d + 1) * static_cast<size_t>(a.s)));
    if (L.hst) SG_TRY(ensure(ws.st_state, ws.st_state_cap, static_cast<size_t>(n)));
    rc = a.plan ? use_plan_sell(ws, a) : build_sell(ws, a.A, a.precision, st);
    if (rc) return rc;

    SG_TRY(hipMemsetAsync(&ws.sc->dc, 0, 5 * sizeof(int), st));
    SG_TRY(hipMemsetAsync(ws.sc->phase_ticks, 0, sizeof(ws.sc->phase_ticks), st));
    SG_TRY(launch_residual(n, nullptr, nullptr, nullptr, a.b, nullptr, ws.r, ws.part_vec, st));
    SG_TRY(launch_norm_finish(ws.part_vec, vec_grid(n), &ws.sc->nf, nullptr, st));
    rc = copy_scalars(ws, st);
    if (rc) return rc;
    const double nf = ws.host_sc->nf;
    sgmres_info_t rep{};
    if (!std::isfinite(nf)) return SGMRES_ENONFINITE;
    if (nf == 0.0) {
        SG_TRY(launch_fill(a.x, n, 0.0, st));
        SG_TRY(hipStreamSynchronize(st));
        if (info) *info = rep;
        return SGMRES_OK;
    }
    int cycles = 0;
    int status = SGMRES_OK;
    CycleEvents ev;
    if (a.profile) SG_TRY(ev.create());
    for (;;) {
        if (ev.on) SG_TRY(hipEventRecord(ev.r0, st));
        SG_TRY(launch_residual(n, a.A.row_ptr, a.A.col_idx, a.A.val, a.b, a.x, ws.r, ws.part_vec, st));
        SG_TRY(launch_norm_finish(ws.part_vec, vec_grid(n), &ws.sc->beta, &ws.sc->nf, st));
        if (ev.on) SG_TRY(hipEventRecord(ev.r1, st));
        rc = copy_scalars(ws, st);
        if (rc) return rc;
        const DevScalars& h = *ws.host_sc;
        if (ev.on) rep.t_residual_ms += CycleEvents::ms(ev.r0, ev.r1);
        if (cycles > 0) {
            rep.steps += h.dc;
            rep.d_eff_last = h.d_eff;
            rep.rest_est = h.rest / nf;
            rep.kappa_est = h.kappa;
            if (ev.on) {
                rep.t_basis_ms += CycleEvents::ms(ev.b0, ev.b1);
                rep.t_sketch_ms += CycleEvents::ms(ev.k1, ev.b1);
                rep.t_lsq_ms += CycleEvents::ms(ev.b1, ev.l1);
                rep.t_combine_ms += CycleEvents::ms(ev.l1, ev.c1);
            }
        }
        rep.flags = h.flags | h.lsq_flags;
        rep.relres = h.rho;
        if (h.abort) {
            status = SGMRES_ETIMEOUT;
            break;
        }
        if (!std::isfinite(h.rho)) {
            status = SGMRES_ENONFINITE;
            break;
        }
        if (h.rho <= a.tol) {
            status = SGMRES_OK;
            break;
        }
        if (cycles > a.restarts) {
            status = SGMRES_NOT_CONVERGED;
            break;
        }
        const uint32_t cyc = static_cast<uint32_t>(cycles);
        SG_TRY(launch_fill_u32(ws.sync, static_cast<int64_t>(sync_words_bytes() / sizeof(unsigned)), 0u, st));
        // tags of the step partials start at 1: clear the slots of earlier launches
        SG_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(ws.part_ab),
                               static_cast<int64_t>(8 * (kStreamMaxK + 1)) * L.grid, 0u, st));
        if (ev.on) SG_TRY(hipEventRecord(ev.b0, st));
        StreamParams p{};
        p.n = n;
        p.sp = ws.cur_sp;
        p.ci = ws.cur_col;
        p.val = ws.cur_val;
        p.r = ws.r;
        p.beta = &ws.sc->beta;
        p.B = ws.B;
        p.ldb = ldb;
        p.H = ws.H;
        p.d = a.d;
        p.k = kk;
        p.part_a = ws.part_ab;
        p.part_b = ws.part_ab + static_cast<int64_t>(2 * (kStreamMaxK + 1)) * L.grid;
        p.state = ws.st_state;
        p.sync = ws.sync;
        p.per_block_release = a.per_block_release;
        p.abort = &ws.sc->abort;
        p.status = &ws.sc->dc;
        p.spin_limit = kSpinLimitTicks;
        p.phase_ticks = ev.on ? ws.sc->phase_ticks : nullptr;
        SG_TRY(stream_launch(L, p, st));
        if (ev.on) SG_TRY(hipEventRecord(ev.k1, st));
        SG_TRY(launch_basis_lists(n, a.seed, cyc, a.s, a.zeta, ws.st_lists, st));
        SG_TRY(launch_residual_sketch(n, ws.r, 1, a.s, a.zeta, ws.st_lists, ws.st_part, ws.g, st));
        SG_TRY(launch_basis_sketch(n, ws.B, ldb, 1, a.precision, a.d + 1, a.s, a.zeta, ws.st_lists, ws.st_part,
                                   ws.SB, st));
        SG_TRY(launch_relation(1, a.d, kk, a.s, ws.H, ws.SB, &ws.sc->dc, ws.SAB, st));
        if (ev.on) SG_TRY(hipEventRecord(ev.b1, st));
        rc = run_lsq(ws, a.s, a.d, &ws.sc->dc, 0, ws.SAB, ws.g, a.kappa_max, ws.y, st);
        if (rc) return rc;
        if (ev.on) SG_TRY(hipEventRecord(ev.l1, st));
        SG_TRY(launch_combine(n, &ws.sc->d_eff, a.d, ws.B, ldb, ws.y, a.x, st, nullptr, a.precision));
        if (ev.on) SG_TRY(hipEventRecord(ev.c1, st));
        ++cycles;
    }
    rep.cycles = cycles;
    if (cycles > 0) {
        rep.path = SGMRES_PATH_STREAM;
        rep.launch_block = kStreamBlock;
        rep.launch_rows = L.hst ? -L.P : L.P;
        rep.launch_grid = L.grid;
    }
    if (ev.on)
        for (int q = 0; q < 8; ++q) rep.phase_us[q] = 1e-2 * static_cast<double>(ws.host_sc->phase_ticks[q]);
    if (info) *info = rep;
    return status;
}

int solve_impl(const SolveArgs& a, sgmres_info_t* info) {
    std::lock_guard<std::mutex> lock(g_mutex);
    Workspace* wsp = nullptr;
    int rc = workspace(&wsp);
    if (rc) return rc;
    Workspace& ws = *wsp;
    const int64_t n = a.A.n;
    const int kk = (a.k > a.d - 1) ? (a.d > 1 ? a.d - 1 : 1) : a.k;
    hipStream_t st = a.stream;

    const bool cheb = a.basis == SGMRES_BASIS_CHEBYSHEV;
    ChebCoef cf{};
    if (cheb && !cheb_coefficients(a.cheb_c, a.cheb_dx, a.cheb_dy, &cf)) return SGMRES_EINVAL;
    if (a.path == SGMRES_PATH_STREAM) return cheb ? SGMRES_EINVAL : solve_stream(a, ws, info);
    if (a.path == SGMRES_PATH_PART_SPLIT) {
        if (cheb || kk > kBatchMaxK) return SGMRES_EINVAL;
        SolveArgs b = a;
        b.k = kk;
        return solve_large(b, info);
    }
    ArnoldiLaunch L{};
    rc = cheb ? prepare_cheb(ws, n, a.d, a.s, a.zeta, a.block, a.rows_per_thread, &L, a.precision)
              : prepare_arnoldi(ws, n, a.d, kk, a.s, a.zeta, a.block, a.rows_per_thread, &L, 0, a.precision);
    if (rc == SGMRES_EINVAL && !cheb && !a.block && !a.rows_per_thread) {
        // beyond the resident capacity: the streaming kernel, else the part-split one
        if (kk <= kStreamMaxK && basis_sketch_fits(n, a.s, a.zeta)) return solve_stream(a, ws, info);
        if (kk <= kBatchMaxK) {
            SolveArgs b = a;
            b.k = kk;
            return solve_large(b, info);
        }
    }
    if (rc) return rc;
    rc = a.plan ? SGMRES_OK : check_csr(ws, a.A, st);
    if (rc) return rc;
    bool halo = false;
    // Two grid barriers per Arnoldi step when at most a quarter of the
    // nonzeros reach outside their row's block (those entries of b_j are then
    // published by their owners as tagged words, rows marked in the bitmap, or
    // recomputed by the block that needs them).
    if (!cheb && !a.halo_off && a.spmv_mode == 0) {
        const size_t xwords = static_cast<size_t>((n + 31) / 32);
        SG_TRY(ensure(ws.xbits, ws.xbits_cap, xwords));
        SG_TRY(launch_fill_u32(ws.xbits, static_cast<int64_t>(xwords), 0u, st));
        SG_TRY(hipMemsetAsync(&ws.sc->offblock, 0, sizeof(unsigned long long), st));
        SG_TRY(launch_offblock_count(n, a.A.row_ptr, a.A.col_idx, static_cast<int64_t>(L.R) * L.block,
                                     &ws.sc->offblock, ws.xbits, st));
        rc = copy_scalars(ws, st);
        if (rc) return rc;
        if (4 * ws.host_sc->offblock <= static_cast<unsigned long long>(a.A.nnz)) {
            ArnoldiShape hs{n, a.d, kk, a.s, a.zeta, L.block, L.R, L.KW == 0, 0, 0, a.precision, 1};
            ArnoldiLaunch H{};
            if (arnoldi_configure(hs, &H) == hipSuccess && H.R == L.R && H.block == L.block && H.KW == L.KW) {
                SG_TRY(ensure(ws.hbuf, ws.hbuf_cap, static_cast<size_t>(n)));
                L = H;
                halo = true;
            }
        }
    }
    SG_TRY(ensure(ws.r, ws.r_cap, static_cast<size_t>(n)));
    // B in the basis storage type (allocated in doubles)
    // columns padded to 128 entries: every column starts on a 256-byte boundary
    // (the basis kernels then read other blocks' rows through L2)
    const int64_t ldb = (n + 127) / 128 * 128;
    SG_TRY(ensure(ws.B, ws.B_cap, (static_cast<size_t>(ldb) * a.d * basis_elem_bytes(a.precision) + 7) / 8));
    SG_TRY(ensure(ws.SB, ws.SB_cap, static_cast<size_t>(a.s) * a.d));
    SG_TRY(ensure(ws.SAB, ws.SAB_cap, static_cast<size_t>(a.s) * a.d));
    SG_TRY(ensure(ws.H, ws.H_cap, static_cast<size_t>(kk + 1) * a.d));
    SG_TRY(ensure(ws.g, ws.g_cap, static_cast<size_t>(a.s)));
    SG_TRY(ensure(ws.y, ws.y_cap, static_cast<size_t>(a.d)));
    SG_TRY(ensure(ws.part_vec, ws.part_vec_cap, static_cast<size_t>(kMaxVecGrid)));
    if (cheb) SG_TRY(ensure(ws.colnorm, ws.colnorm_cap, static_cast<size_t>(a.d)));
    // the basis cycles read A through its sliced ELL copy, values in the
    // cycles' arithmetic type (FP32 in the mixed-precision modes)
    rc = a.plan ? use_plan_sell(ws, a) : build_sell(ws, a.A, a.precision, st);
    if (rc) return rc;

    // |b|, and clear the per-solve counters
    SG_TRY(hipMemsetAsync(&ws.sc->dc, 0, 5 * sizeof(int), st));
    SG_TRY(hipMemsetAsync(ws.sc->phase_ticks, 0, sizeof(ws.sc->phase_ticks), st));
    SG_TRY(launch_residual(n, nullptr, nullptr, nullptr, a.b, nullptr, ws.r, ws.part_vec, st));
    SG_TRY(launch_norm_finish(ws.part_vec, vec_grid(n), &ws.sc->nf, nullptr, st));
    rc = copy_scalars(ws, st);
    if (rc) return rc;
    const double nf = ws.host_sc->nf;
    sgmres_info_t rep{};
    if (cheb) {
        rep.cheb_box[0] = a.cheb_c;
        rep.cheb_box[1] = a.cheb_dx;
        rep.cheb_box[2] = a.cheb_dy;
    }
    if (!std::isfinite(nf)) return SGMRES_ENONFINITE;
    if (nf == 0.0) {
        SG_TRY(launch_fill(a.x, n, 0.0, st));
        SG_TRY(hipStreamSynchronize(st));
        if (info) *info = rep;
        return SGMRES_OK;
    }

    int cycles = 0;
    int status = SGMRES_OK;
    CycleEvents ev;
    if (a.profile) SG_TRY(ev.create());
    for (;;) {
        if (ev.on) SG_TRY(hipEventRecord(ev.r0, st));
        SG_TRY(launch_residual(n, a.A.row_ptr, a.A.col_idx, a.A.val, a.b, a.x, ws.r, ws.part_vec, st));
        SG_TRY(launch_norm_finish(ws.part_vec, vec_grid(n), &ws.sc->beta, &ws.sc->nf, st));
        if (ev.on) SG_TRY(hipEventRecord(ev.r1, st));
        rc = copy_scalars(ws, st);
        if (rc) return rc;
        const DevScalars& h = *ws.host_sc;
        if (ev.on) rep.t_residual_ms += CycleEvents::ms(ev.r0, ev.r1);
        if (cycles > 0) {
            rep.steps += h.dc;
            rep.d_eff_last = h.d_eff;
            rep.rest_est = h.rest / nf;
            rep.kappa_est = h.kappa;
            if (ev.on) {
                rep.t_basis_ms += CycleEvents::ms(ev.b0, ev.b1);
                rep.t_lsq_ms += CycleEvents::ms(ev.b1, ev.l1);
                rep.t_combine_ms += CycleEvents::ms(ev.l1, ev.c1);
            }
        }
        rep.flags = h.flags | h.lsq_flags;
        rep.relres = h.rho;
        if (h.abort) {
            status = SGMRES_ETIMEOUT;
            break;
        }
        if (!std::isfinite(h.rho)) {
            status = SGMRES_ENONFINITE;
            break;
        }
        if (h.rho <= a.tol) {
            status = SGMRES_OK;
            break;
        }
        if (cycles > a.restarts) {
            status = SGMRES_NOT_CONVERGED;
            break;
        }
        // the solve needs S A B and g only; S B is not formed
        if (cheb)
            rc = run_cheb_cycle(ws, a.A, a.d, a.s, a.zeta, a.seed, static_cast<uint32_t>(cycles), L, cf, ws.B, ldb,
                                ws.SB, ws.SAB, ws.colnorm, ws.g, st, ev.on ? ev.b0 : nullptr, a.per_block_release,
                                ev.on, 0);
        else
            rc = run_cycle(ws, a.A, a.d, kk, a.s, a.zeta, a.seed, static_cast<uint32_t>(cycles), L, ws.B, ldb,
                           ws.SB, ws.SAB, ws.H, ws.g, st, ev.on ? ev.b0 : nullptr, a.per_block_release, ev.on,
                           a.spmv_mode, halo ? (a.precision == SGMRES_PREC_FP64 ? 1 : 2) : 0);
        if (rc) return rc;
        if (ev.on) SG_TRY(hipEventRecord(ev.b1, st));
        rc = run_lsq(ws, a.s, a.d, &ws.sc->dc, 0, ws.SAB, ws.g, a.kappa_max, ws.y, st);
        if (rc) return rc;
        if (ev.on) SG_TRY(hipEventRecord(ev.l1, st));
        SG_TRY(launch_combine(n, &ws.sc->d_eff, a.d, ws.B, ldb, ws.y, a.x, st, cheb ? ws.colnorm : nullptr,
                              a.precision));
        if (ev.on) SG_TRY(hipEventRecord(ev.c1, st));
        ++cycles;
    }
    rep.cycles = cycles;
    if (cycles > 0) {
        rep.path = cheb ? SGMRES_PATH_CHEBYSHEV : (halo ? SGMRES_PATH_ARNOLDI_HALO : SGMRES_PATH_ARNOLDI_3BAR);
        rep.launch_block = L.block;
        rep.launch_rows = L.R;
        rep.launch_grid = L.grid;
    }
    if (ev.on)
        for (int q = 0; q < 8; ++q) rep.phase_us[q] = 1e-2 * static_cast<double>(ws.host_sc->phase_ticks[q]);
    if (info) *info = rep;
    return status;
}

constexpr int kBoxSteps = 20;       // Arnoldi steps of the automatic box estimate
constexpr double kBoxMargin = 0.1;  // widening of the Ritz values' half-widths

// Spectral box (c, dx, dy) of A for the Chebyshev basis (Section 4.4: a few
// Arnoldi iterations estimate the spectrum): m + 1 steps of Arnoldi with a
// full window from r (the resident basis kernel, FP64, two Gram-Schmidt
// passes), the Ritz values (eigenvalues of the leading m x m block of the
// Hessenberg matrix; of the leading dc x dc block when the Krylov space is
// invariant after dc columns) and their bounding rectangle, half-widths
// widened by kBoxMargin.  ritz (nullable, 2m): real parts, then imaginary
// parts; *mr: Ritz values found.  Caller holds g_mutex.
int cheb_box_locked(Workspace& ws, const sgmres_csr_t& A, const double* r, int m, double box[3], double* ritz,
                    int* mr, hipStream_t st) {
    const int64_t n = A.n;
    if (m < 1 || m > 64 || m >= n) return SGMRES_EINVAL;
    const int d = m + 1, k = m, zeta = 8;
    const int s = d + 1 > 2 * zeta ? d + 1 : 2 * zeta;
    ArnoldiLaunch L{};
    int rc = prepare_arnoldi(ws, n, d, k, s, zeta, 0, 0, &L, 0);
    if (rc) return rc;
    const int64_t ldb = (n + 127) / 128 * 128;
    SG_TRY(ensure(ws.r, ws.r_cap, static_cast<size_t>(n)));
    SG_TRY(ensure(ws.part_vec, ws.part_vec_cap, static_cast<size_t>(kMaxVecGrid)));
    SG_TRY(ensure(ws.B, ws.B_cap, static_cast<size_t>(ldb) * d));
    SG_TRY(ensure(ws.SB, ws.SB_cap, static_cast<size_t>(s) * d));
    SG_TRY(ensure(ws.SAB, ws.SAB_cap, static_cast<size_t>(s) * d));
    SG_TRY(ensure(ws.H, ws.H_cap, static_cast<size_t>(k + 1) * d));
    SG_TRY(ensure(ws.g, ws.g_cap, static_cast<size_t>(s)));
    rc = check_csr(ws, A, st);
    if (rc) return rc;
    rc = build_sell(ws, A, SGMRES_PREC_FP64, st);
    if (rc) return rc;
    SG_TRY(hipMemsetAsync(&ws.sc->dc, 0, 5 * sizeof(int), st));
    SG_TRY(launch_residual(n, nullptr, nullptr, nullptr, r, nullptr, ws.r, ws.part_vec, st));
    SG_TRY(launch_norm_finish(ws.part_vec, vec_grid(n), &ws.sc->beta, nullptr, st));
    SG_TRY(launch_fill(ws.H, static_cast<int64_t>(k + 1) * d, 0.0, st));
    rc = run_cycle(ws, A, d, k, s, zeta, 0, 0, L, ws.B, ldb, ws.SB, ws.SAB, ws.H, ws.g, st);
    if (rc) return rc;
    std::vector<double> Hh(static_cast<size_t>(k + 1) * d);
    SG_TRY(hipMemcpyAsync(Hh.data(), ws.H, sizeof(double) * Hh.size(), hipMemcpyDeviceToHost, st));
    rc = copy_scalars(ws, st);
    if (rc) return rc;
    if (ws.host_sc->abort) return SGMRES_ETIMEOUT;
    if (!std::isfinite(ws.host_sc->beta)) return SGMRES_ENONFINITE;
    if (ws.host_sc->beta == 0.0) {  // r = 0: no Krylov space; a valid box, no Ritz values
        box[0] = 0.0;
        box[1] = 1.0;
        box[2] = 0.0;
        if (mr) *mr = 0;
        return SGMRES_OK;
    }
    const int me = ws.host_sc->dc < m ? ws.host_sc->dc : m;
    if (me < 1) return SGMRES_EINVAL;
    // leading me x me block, column-major: column j holds h_a = H[j (k+1) + a]
    // in row j - a (window entry a, newest first) and nu_j = H[j (k+1) + k]
    // below the diagonal
    std::vector<double> Hm(static_cast<size_t>(me) * me, 0.0), wr(me), wi(me);
    for (int j = 0; j < me; ++j) {
        for (int a = 0; a <= j; ++a) Hm[(j - a) + static_cast<size_t>(j) * me] = Hh[static_cast<size_t>(j) * (k + 1) + a];
        if (j + 1 < me) Hm[(j + 1) + static_cast<size_t>(j) * me] = Hh[static_cast<size_t>(j) * (k + 1) + k];
    }
    for (double v : Hm)
        if (!std::isfinite(v)) return SGMRES_ENONFINITE;
    if (hessenberg_eigenvalues(me, Hm.data(), me, wr.data(), wi.data()) != 0) return SGMRES_EINVAL;
    box_from_ritz(me, wr.data(), wi.data(), kBoxMargin, box);
    // a single point (A a multiple of I on the Krylov space): keep rho > 0
    if (!(box[1] > 0.0) && !(box[2] > 0.0)) box[1] = std::fabs(box[0]) > 0.0 ? 1e-8 * std::fabs(box[0]) : 1e-8;
    if (ritz)
        for (int i = 0; i < me; ++i) {
            ritz[i] = wr[i];
            ritz[m + i] = wi[i];
        }
    if (mr) *mr = me;
    return SGMRES_OK;
}

int solve_entry(const sgmres_csr_t* A, const double* b, double* x, int d, int k, int s, uint64_t seed,
                double tol, int restarts, const sgmres_options_t* opts, sgmres_info_t* info, void* stream,
                const Plan* plan = nullptr) {
    if (plan) {
        const bool t = opts && opts->transposed;
        if (t && !plan->t_rp) return SGMRES_EINVAL;
        A = t ? &plan->At : &plan->A;
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) return SGMRES_EINVAL;
    }
    if (!csr_ok(A) || !b || !x) return SGMRES_EINVAL;
    const int zeta = (opts && opts->zeta) ? opts->zeta : 8;
    const double kappa_max = (opts && opts->kappa_max > 0) ? opts->kappa_max : 1e14;
    if (bad_sizes(A->n, d, k, s, zeta) || !(tol >= 0.0) || restarts < 0) return SGMRES_EINVAL;
    SolveArgs a{};
    a.A = *A;
    a.b = b;
    a.x = x;
    a.d = d;
    a.k = k;
    a.s = s;
    a.zeta = zeta;
    a.seed = seed;
    a.tol = tol;
    a.restarts = restarts;
    a.kappa_max = kappa_max;
    a.block = opts ? opts->block_size : 0;
    a.rows_per_thread = opts ? opts->rows_per_thread : 0;
    a.profile = opts ? opts->profile : 0;
    a.per_block_release = opts ? opts->barrier_mode : 0;
    a.spmv_mode = opts ? opts->spmv_mode : 0;
    if (a.spmv_mode != 0) return SGMRES_EINVAL;
    a.basis = opts ? opts->basis : SGMRES_BASIS_ARNOLDI;
    a.precision = opts ? opts->precision : SGMRES_PREC_FP64;
    a.halo_off = opts ? opts->halo_off : 0;
    a.path = opts ? opts->path : 0;
    a.stream_state = opts ? opts->stream_state : 0;
    if ((a.path != 0 && a.path != SGMRES_PATH_STREAM && a.path != SGMRES_PATH_PART_SPLIT) || a.stream_state < 0 ||
        a.stream_state > 2)
        return SGMRES_EINVAL;
    if (a.precision != SGMRES_PREC_FP64 && a.precision != SGMRES_PREC_FP32 && a.precision != SGMRES_PREC_BF16_BASIS)
        return SGMRES_EINVAL;
    if (a.basis != SGMRES_BASIS_ARNOLDI && a.basis != SGMRES_BASIS_CHEBYSHEV) return SGMRES_EINVAL;
    a.stream = static_cast<hipStream_t>(stream);
    if (a.basis == SGMRES_BASIS_CHEBYSHEV) {
        a.cheb_c = opts->cheb_c;
        a.cheb_dx = opts->cheb_dx;
        a.cheb_dy = opts->cheb_dy;
        if (a.cheb_dx == 0.0 && a.cheb_dy == 0.0) {
            // no box given: estimate it from b (transposed solves and plans
            // estimate it for the matrix they solve with)
            double box[3];
            const int m = std::min<int64_t>(std::min(kBoxSteps, d), A->n - 1);
            const bool t = opts->transposed != 0;
            const sgmres_csr_t* M = A;
            if (t && plan) M = &plan->At;
            if (t && !plan) return SGMRES_EINVAL;  // the box of A^T: pass it, or use a plan with A^T
            std::lock_guard<std::mutex> lock(g_mutex);
            Workspace* wsp = nullptr;
            int rc = workspace(&wsp);
            if (rc) return rc;
            rc = cheb_box_locked(*wsp, *M, b, m, box, nullptr, nullptr, a.stream);
            if (rc) return rc;
            a.cheb_c = box[0];
            a.cheb_dx = box[1];
            a.cheb_dy = box[2];
        }
        ChebCoef cf{};
        if (!cheb_coefficients(a.cheb_c, a.cheb_dx, a.cheb_dy, &cf)) return SGMRES_EINVAL;
    }
    if (plan) {
        a.plan = plan;
        a.plan_t = (opts && opts->transposed) ? 1 : 0;
        return solve_impl(a, info);
    }
    if (opts && opts->transposed) {
        Workspace* wsp = nullptr;
        {
            std::lock_guard<std::mutex> lock(g_mutex);
            int rc = workspace(&wsp);
            if (rc) return rc;
            const int64_t n = A->n;
            SG_TRY(ensure(wsp->t_rp, wsp->t_rp_cap, static_cast<size_t>(n + 1)));
            SG_TRY(ensure(wsp->t_ci, wsp->t_ci_cap, static_cast<size_t>(A->nnz)));
            SG_TRY(ensure(wsp->t_val, wsp->t_val_cap, static_cast<size_t>(A->nnz)));
            SG_TRY(ensure(wsp->t_scratch, wsp->t_scratch_cap, static_cast<size_t>(transpose_scratch_ints(n))));
            rc = check_csr(*wsp, *A, a.stream);
            if (rc) return rc;
            SG_TRY(launch_csr_transpose(n, A->nnz, A->row_ptr, A->col_idx, A->val, wsp->t_rp, wsp->t_ci,
                                        wsp->t_val, wsp->t_scratch, a.stream));
        }
        a.A.row_ptr = wsp->t_rp;
        a.A.col_idx = wsp->t_ci;
        a.A.val = wsp->t_val;
    }
    return solve_impl(a, info);
}


// ---------------------------------------------------------------------------
// Batched solve: one workgroup per system and cycle (batched.hip), the
// least squares as one workgroup per system, the cycle's kernels replayed from
// a captured hipGraph.  The workgroup shape (rows per chunk) is picked by a
// small autotuner that times the first cycle of each candidate and remembers
// the winner per problem class.
// ---------------------------------------------------------------------------
struct BatchCand {
    int block, R;
};
constexpr BatchCand kBatchCands[] = {{512, 4}, {256, 4}, {512, 2}, {1024, 2}, {1024, 4}, {1024, 1}};
constexpr int kBatchMinChunk = 1024;  // smallest block * R among the candidates
constexpr int kBatchMaxChunk = 4096;  // largest
constexpr size_t kArenaAlign = 256;
constexpr int64_t kBatchTuneRows = int64_t(1) << 20;  // smaller batches use 512 x 4
constexpr int64_t kBatchResidentRows = int64_t(1) << 19;  // such systems go to the resident kernels
constexpr int64_t kBatchPartRows = 16384;              // rows per part of a large system
constexpr int64_t kBlockMinRows = int64_t(1) << 16;  // systems sharing A from this size on: block solve

using BatchKey = std::tuple<int, int, int, int, int, int, int>;
std::map<BatchKey, BatchCand> g_batch_tuned;

size_t align_up(size_t v) { return (v + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

// Caller holds g_mutex.  st_out (nullable, nsys entries) receives the final
// per-system states.
int batch_solve_locked(int nsys, const sgmres_system_t* systems, int d, int k, int s, uint64_t seed, double tol,
                       int restarts, const sgmres_options_t* opts, sgmres_batch_result_t* results, hipStream_t st,
                       BatchState* st_out = nullptr) {
    const int zeta = (opts && opts->zeta) ? opts->zeta : 8;
    const double kappa_max = (opts && opts->kappa_max > 0) ? opts->kappa_max : 1e14;
    const int prec = opts ? opts->precision : SGMRES_PREC_FP64;
    if (prec != SGMRES_PREC_FP64 && prec != SGMRES_PREC_FP32 && prec != SGMRES_PREC_BF16_BASIS) return SGMRES_EINVAL;
    if (nsys < 0 || (nsys > 0 && !systems) || !(tol >= 0.0) || restarts < 0 || k > kBatchMaxK) return SGMRES_EINVAL;
    for (int i = 0; i < nsys; ++i) {
        const sgmres_system_t& y = systems[i];
        if (!csr_ok(&y.A) || !y.b || !y.x || bad_sizes(y.A.n, d, k, s, zeta)) return SGMRES_EINVAL;
    }
    if (nsys == 0) return SGMRES_OK;

    Workspace* wsp = nullptr;
    int rc = workspace(&wsp);
    if (rc) return rc;
    Workspace& ws = *wsp;

    // CSR validation, one flag for the whole batch
    SG_TRY(hipMemsetAsync(&ws.sc->csr_bad, 0, sizeof(int), st));
    for (int i = 0; i < nsys; ++i)
        SG_TRY(launch_csr_check(systems[i].A.n, systems[i].A.nnz, systems[i].A.row_ptr, systems[i].A.col_idx,
                                &ws.sc->csr_bad, st));
    rc = copy_scalars(ws, st);
    if (rc) return rc;
    if (ws.host_sc->csr_bad) return SGMRES_ECSR;

    // arena layout (sized for every candidate chunk length)
    const size_t eb = basis_elem_bytes(prec);
    const size_t ec = (prec == SGMRES_PREC_FP64) ? 8 : 4;
    std::vector<size_t> off(nsys + 1, 0);
    auto sys_bytes = [&](const sgmres_system_t& y) {
        const size_t n = static_cast<size_t>(y.A.n);
        const size_t nch = n / kBatchMinChunk + 1;
        size_t b = 0;
        b += align_up(n * d * eb);                                            // B
        b += 2 * align_up(n * ec);                                            // m, w
        b += align_up(n * 8);                                                 // r
        b += align_up(sizeof(uint16_t) * zeta * (n + kBatchMaxChunk));        // lists
        b += align_up(sizeof(int) * nch * (s + 1));                           // list starts
        b += align_up(8 * static_cast<size_t>(s) * d) + align_up(8 * s) + align_up(8 * d);  // SAB, g, y
        if (prec != SGMRES_PREC_FP64) b += align_up(4 * static_cast<size_t>(y.A.nnz));      // FP32 values
        return b;
    };
    for (int i = 0; i < nsys; ++i) off[i + 1] = off[i] + sys_bytes(systems[i]);
    SG_TRY(ensure(ws.bt_arena, ws.bt_arena_cap, off[nsys]));
    SG_TRY(ensure(ws.bt_sys, ws.bt_sys_cap, static_cast<size_t>(nsys)));
    SG_TRY(ensure(ws.bt_st, ws.bt_st_cap, static_cast<size_t>(nsys)));

    std::vector<BatchSys> desc(nsys);
    int64_t total_rows = 0;
    for (int i = 0; i < nsys; ++i) {
        const sgmres_system_t& y = systems[i];
        const size_t n = static_cast<size_t>(y.A.n);
        const size_t nch = n / kBatchMinChunk + 1;
        unsigned char* p = ws.bt_arena + off[i];
        BatchSys& D = desc[i];
        D.n = y.A.n;
        D.rp = y.A.row_ptr;
        D.ci = y.A.col_idx;
        D.val = y.A.val;
        D.b = y.b;
        D.x = y.x;
        D.B = p;
        p += align_up(n * d * eb);
        D.m = p;
        p += align_up(n * ec);
        D.w = p;
        p += align_up(n * ec);
        D.r = reinterpret_cast<double*>(p);
        p += align_up(n * 8);
        D.lists = reinterpret_cast<uint16_t*>(p);
        p += align_up(sizeof(uint16_t) * zeta * (n + kBatchMaxChunk));
        D.lstart = reinterpret_cast<int*>(p);
        p += align_up(sizeof(int) * nch * (s + 1));
        D.SAB = reinterpret_cast<double*>(p);
        p += align_up(8 * static_cast<size_t>(s) * d);
        D.g = reinterpret_cast<double*>(p);
        p += align_up(8 * s);
        D.y = reinterpret_cast<double*>(p);
        p += align_up(8 * d);
        D.valc = y.A.val;
        if (prec != SGMRES_PREC_FP64) {
            float* vf = reinterpret_cast<float*>(p);
            SG_TRY(launch_to_f32(y.A.nnz, y.A.val, vf, st));
            D.valc = vf;
        }
        total_rows += y.A.n;
    }
    // largest systems first; each system split into parts of whole chunks
    std::vector<int> order(nsys);
    for (int i = 0; i < nsys; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return systems[a].A.n > systems[b].A.n; });
    std::vector<int64_t> slot_off(nsys + 1, 0);
    for (int i = 0; i < nsys; ++i) {
        const int64_t pm = std::min<int64_t>(kBatchMaxParts, (systems[i].A.n + kBatchPartRows - 1) / kBatchPartRows);
        slot_off[i + 1] = slot_off[i] + (2 * kBatchRed + s) * std::max<int64_t>(pm, 1);
    }
    SG_TRY(ensure(ws.bt_slots, ws.bt_slots_cap, static_cast<size_t>(slot_off[nsys])));
    SG_TRY(ensure(ws.bt_slot_off, ws.bt_slot_off_cap, static_cast<size_t>(nsys)));
    SG_TRY(ensure(ws.bt_gcnt, ws.bt_gcnt_cap, static_cast<size_t>(nsys)));
    SG_TRY(ensure(ws.bt_task, ws.bt_task_cap, static_cast<size_t>(nsys) * kBatchMaxParts));
    SG_TRY(hipMemcpyAsync(ws.bt_sys, desc.data(), sizeof(BatchSys) * nsys, hipMemcpyHostToDevice, st));
    SG_TRY(hipMemcpyAsync(ws.bt_slot_off, slot_off.data(), sizeof(int64_t) * nsys, hipMemcpyHostToDevice, st));
    std::vector<BatchTask> tasks;
    // parts for chunks of CH rows on a grid of G workgroups (a system never has
    // more parts than the grid has workgroups)
    auto make_tasks = [&](int CH, int G) {
        tasks.clear();
        for (int i : order) {
            const int64_t n = systems[i].A.n;
            const int64_t nchs = (n + CH - 1) / CH;
            int64_t P = (n + kBatchPartRows - 1) / kBatchPartRows;
            P = std::max<int64_t>(1, std::min<int64_t>({P, nchs, static_cast<int64_t>(kBatchMaxParts),
                                                        static_cast<int64_t>(G)}));
            for (int64_t q = 0; q < P; ++q) {
                BatchTask t{};
                t.sys = i;
                t.part = static_cast<int>(q);
                t.nparts = static_cast<int>(P);
                t.r0 = (q * nchs / P) * CH;
                t.r1 = std::min<int64_t>(n, ((q + 1) * nchs / P) * CH);
                tasks.push_back(t);
            }
        }
        return hipMemcpyAsync(ws.bt_task, tasks.data(), sizeof(BatchTask) * tasks.size(), hipMemcpyHostToDevice, st);
    };

    int* ctr = ws.sc->batch_ctr;
    BatchParams bp{};
    bp.task = ws.bt_task;
    bp.sys = ws.bt_sys;
    bp.st = ws.bt_st;
    bp.slots = ws.bt_slots;
    bp.slot_off = ws.bt_slot_off;
    bp.gcnt = ws.bt_gcnt;
    bp.queue = ctr + 1;
    bp.active = ctr + 2;
    bp.cycle = ctr;
    bp.abort = &ws.sc->abort;
    bp.spin_limit = kSpinLimitTicks;
    bp.d = d;
    bp.k = k;
    bp.s = s;
    bp.zeta = zeta;
    bp.restarts = restarts;
    bp.seed = seed;
    bp.tol = tol;
    SG_TRY(hipMemsetAsync(&ws.sc->abort, 0, sizeof(int), st));

    // workgroup shape: given, the default for small batches, remembered, or
    // timed on the first cycle
    BatchLaunch L{};
    const int want_block = opts ? opts->block_size : 0;
    const int want_R = opts ? opts->rows_per_thread : 0;
    if (want_block || want_R || total_rows < kBatchTuneRows) {
        if (batch_configure(want_block ? want_block : 512, want_R ? want_R : 4, d, s, zeta, prec, &L) != hipSuccess)
            return SGMRES_EINVAL;
    } else {
        const BatchKey key{nsys, static_cast<int>(total_rows >> 16), d, k, s, zeta, prec};
        auto it = g_batch_tuned.find(key);
        if (it != g_batch_tuned.end()) {
            SG_TRY(batch_configure(it->second.block, it->second.R, d, s, zeta, prec, &L));
        } else {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            SG_TRY(hipEventCreate(&e0));
            SG_TRY(hipEventCreate(&e1));
            float best = 0.0f;
            BatchCand win{0, 0};
            for (const BatchCand& c : kBatchCands) {
                BatchLaunch T{};
                if (batch_configure(c.block, c.R, d, s, zeta, prec, &T) != hipSuccess) continue;
                SG_TRY(make_tasks(batch_chunk(T), T.grid));
                bp.ntask = static_cast<int>(tasks.size());
                SG_TRY(launch_batch_reset(ws.bt_st, ws.bt_gcnt, nsys, ctr, st));
                SG_TRY(hipEventRecord(e0, st));
                SG_TRY(batch_launch(T, bp, st));
                SG_TRY(hipEventRecord(e1, st));
                SG_TRY(hipEventSynchronize(e1));
                float ms = 0.0f;
                SG_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (win.block == 0 || ms < best) {
                    best = ms;
                    win = c;
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            if (win.block == 0) return SGMRES_EINVAL;
            g_batch_tuned[key] = win;
            SG_TRY(batch_configure(win.block, win.R, d, s, zeta, prec, &L));
        }
    }
    SG_TRY(make_tasks(batch_chunk(L), L.grid));
    bp.ntask = static_cast<int>(tasks.size());

    SG_TRY(launch_batch_reset(ws.bt_st, ws.bt_gcnt, nsys, ctr, st));
    bool eager = opts && opts->batch_eager;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (!eager) {
        if (!ws.capture_stream) SG_TRY(hipStreamCreateWithFlags(&ws.capture_stream, hipStreamNonBlocking));
        hipStream_t cs = ws.capture_stream;
        SG_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        hipError_t e = batch_launch(L, bp, cs);
        if (e == hipSuccess) e = launch_lsq_batched(nsys, s, ws.bt_sys, ws.bt_st, kappa_max, cs);
        if (e == hipSuccess) e = launch_batch_advance(ctr, ws.bt_st, ws.bt_gcnt, nsys, cs);
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            // a runtime that cannot record the cooperative launch: launch the
            // cycles directly (same kernels, same bits)
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            exec = nullptr;
            graph = nullptr;
            (void)hipGetLastError();
            eager = true;
        }
    }
    int status = SGMRES_OK;
    for (int c = 0; c <= restarts + 2; ++c) {
        hipError_t e;
        if (eager) {
            e = batch_launch(L, bp, st);
            if (e == hipSuccess) e = launch_lsq_batched(nsys, s, ws.bt_sys, ws.bt_st, kappa_max, st);
            if (e == hipSuccess) e = launch_batch_advance(ctr, ws.bt_st, ws.bt_gcnt, nsys, st);
        } else {
            e = hipGraphLaunch(exec, st);
        }
        if (e != hipSuccess) {
            status = to_code(e);
            break;
        }
        rc = copy_scalars(ws, st);
        if (rc) {
            status = rc;
            break;
        }
        if (ws.host_sc->batch_ctr[3] == 0 || ws.host_sc->abort) break;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (status != SGMRES_OK) return status;

    std::vector<BatchState> hs(nsys);
    SG_TRY(hipMemcpyAsync(hs.data(), ws.bt_st, sizeof(BatchState) * nsys, hipMemcpyDeviceToHost, st));
    SG_TRY(hipStreamSynchronize(st));
    if (ws.host_sc->abort) return SGMRES_ETIMEOUT;
    if (st_out) std::copy(hs.begin(), hs.end(), st_out);
    int all = SGMRES_OK;
    for (int i = 0; i < nsys; ++i) {
        const BatchState& t = hs[i];
        const int code = t.status == 1 ? SGMRES_OK : (t.status == 3 ? SGMRES_ENONFINITE : SGMRES_NOT_CONVERGED);
        if (code != SGMRES_OK) all = SGMRES_NOT_CONVERGED;
        if (results) {
            results[i].status = code;
            results[i].cycles = t.cycles;
            results[i].steps = t.steps;
            results[i].flags = t.flags | t.lsq_flags;
            results[i].relres = t.rho;
        }
    }
    return all;
}

// ---------------------------------------------------------------------------
// Batched solve, several systems per resident basis launch.  Each system runs
// the cycles of sgmres_solve (same sketch keys, same stopping rule), its basis
// cycle on its own group of G_i = ceil(n_i / rows) workgroups of the
// multi-system kernel.  Systems are packed, largest first, into waves of at
// most `capacity` workgroups (first fit); a round runs one cycle of every
// active system, wave after wave on the stream:
//   basis launch (all groups of the wave) -> least squares (one workgroup per
//   system) -> per system x += B y, r = b - A x, |r|, |r|/|b|
// and ends with one read of the per-system states, which decides the next
// round.  The basis arena (B, partial sums, barrier words) is sized for one
// wave and reused by the next (stream order).
// Caller holds g_mutex; sizes were validated and the CSR arrays checked.
int wave_solve_locked(int nsys, const sgmres_system_t* systems, int d, int k, int s, uint64_t seed, double tol,
                      int restarts, int zeta, double kappa_max, int prec, int R, sgmres_batch_result_t* results,
                      hipStream_t st) {
    const int kk = (k > d - 1) ? (d > 1 ? d - 1 : 1) : k;
    MultiLaunch L{};
    if (arnoldi_multi_configure(R, kk, s, zeta, prec, &L) != hipSuccess) return SGMRES_EINVAL;
    for (int i = 0; i < nsys; ++i)
        if ((systems[i].A.n + L.rows - 1) / L.rows > L.capacity) return SGMRES_EINVAL;
    Workspace* wsp = nullptr;
    int rc = workspace(&wsp);
    if (rc) return rc;
    Workspace& ws = *wsp;
    const size_t eb = basis_elem_bytes(prec);
    const size_t ev = prec == SGMRES_PREC_FP64 ? 8 : 4;  // sliced ELL value bytes

    // ---- sliced ELL copies: widths of every system, one read, then fills ----
    std::vector<int64_t> koff(nsys + 1, 0);
    for (int i = 0; i < nsys; ++i) koff[i + 1] = koff[i] + (systems[i].A.n + 63) / 64;
    SG_TRY(ensure(ws.wv_K, ws.wv_K_cap, static_cast<size_t>(koff[nsys])));
    // one launch for all systems' widths, one for all fills (below)
    std::vector<SellJob> sj(nsys);  // read by copies: kept to the synchronisations below
    int wblocks = 0;
    for (int i = 0; i < nsys; ++i) {
        SellJob& J = sj[i];
        J = SellJob{};
        J.n = systems[i].A.n;
        J.rp = systems[i].A.row_ptr;
        J.ci = systems[i].A.col_idx;
        J.val = systems[i].A.val;
        J.K = ws.wv_K + koff[i];
        J.wblk0 = wblocks;
        J.wnblk = sell_width_blocks(J.n);
        wblocks += J.wnblk;
    }
    SG_TRY(ensure(ws.wv_sell, ws.wv_sell_cap, static_cast<size_t>(nsys)));
    SG_TRY(hipMemcpyAsync(ws.wv_sell, sj.data(), sizeof(SellJob) * nsys, hipMemcpyHostToDevice, st));
    SG_TRY(launch_sell_jobs(ws.wv_sell, nsys, wblocks, false, prec, st));
    std::vector<int> K(static_cast<size_t>(koff[nsys]));
    SG_TRY(hipMemcpyAsync(K.data(), ws.wv_K, sizeof(int) * K.size(), hipMemcpyDeviceToHost, st));
    SG_TRY(hipStreamSynchronize(st));
    // slice starts of all systems in one array (one copy); per-system arena:
    // col, val, r, SAB, H, g, y
    std::vector<int64_t> sp(static_cast<size_t>(koff[nsys] + nsys), 0);
    std::vector<size_t> off(nsys + 1, 0);
    for (int i = 0; i < nsys; ++i) {
        const int64_t n = systems[i].A.n, nsl = (n + 63) / 64;
        int64_t* spi = sp.data() + koff[i] + i;
        for (int64_t q = 0; q < nsl; ++q) spi[q + 1] = spi[q] + 64 * static_cast<int64_t>(K[koff[i] + q]);
        const size_t tot = static_cast<size_t>(spi[nsl] > 0 ? spi[nsl] : 1);
        size_t b = align_up(4 * tot) + align_up(ev * tot) + align_up(8 * static_cast<size_t>(n));
        b += align_up(8 * static_cast<size_t>(s) * d) + align_up(8 * static_cast<size_t>(kk + 1) * d) +
             align_up(8 * static_cast<size_t>(s)) + 2 * align_up(8 * static_cast<size_t>(d));
        off[i + 1] = off[i] + b;
    }
    SG_TRY(ensure(ws.wv_sys_arena, ws.wv_sys_arena_cap, off[nsys]));
    SG_TRY(ensure(ws.wv_sp, ws.wv_sp_cap, sp.size()));
    SG_TRY(hipMemcpyAsync(ws.wv_sp, sp.data(), sizeof(int64_t) * sp.size(), hipMemcpyHostToDevice, st));
    SG_TRY(ensure(ws.wv_sys, ws.wv_sys_cap, static_cast<size_t>(nsys)));
    SG_TRY(ensure(ws.wv_st, ws.wv_st_cap, static_cast<size_t>(nsys)));
    SG_TRY(ensure(ws.part_vec, ws.part_vec_cap, static_cast<size_t>(kMaxVecGrid)));
    struct SysBufs {
        int64_t* sp;
        int32_t* col;
        void* val;
        double *r, *SAB, *H, *g, *y, *tau;
    };
    std::vector<SysBufs> sb(nsys);
    std::vector<BatchSys> desc(nsys);
    int fblocks = 0;
    for (int i = 0; i < nsys; ++i) {
        const sgmres_csr_t& A = systems[i].A;
        const int64_t n = A.n, nsl = (n + 63) / 64;
        const int64_t* spi = sp.data() + koff[i] + i;
        const size_t tot = static_cast<size_t>(spi[nsl] > 0 ? spi[nsl] : 1);
        unsigned char* q = ws.wv_sys_arena + off[i];
        SysBufs& B = sb[i];
        B.sp = ws.wv_sp + koff[i] + i;
        B.col = reinterpret_cast<int32_t*>(q);
        q += align_up(4 * tot);
        B.val = q;
        q += align_up(ev * tot);
        B.r = reinterpret_cast<double*>(q);
        q += align_up(8 * static_cast<size_t>(n));
        B.SAB = reinterpret_cast<double*>(q);
        q += align_up(8 * static_cast<size_t>(s) * d);
        B.H = reinterpret_cast<double*>(q);
        q += align_up(8 * static_cast<size_t>(kk + 1) * d);
        B.g = reinterpret_cast<double*>(q);
        q += align_up(8 * static_cast<size_t>(s));
        B.y = reinterpret_cast<double*>(q);
        q += align_up(8 * static_cast<size_t>(d));
        B.tau = reinterpret_cast<double*>(q);
        SellJob& J = sj[i];
        J.sp = B.sp;
        J.scol = B.col;
        J.sval = B.val;
        J.fblk0 = fblocks;
        J.fnblk = sell_fill_blocks(n);
        fblocks += J.fnblk;
        BatchSys& D = desc[i];
        D = BatchSys{};
        D.n = n;
        D.rp = A.row_ptr;
        D.ci = A.col_idx;
        D.val = A.val;
        D.b = systems[i].b;
        D.x = systems[i].x;
        D.r = B.r;
        D.SAB = B.SAB;
        D.g = B.g;
        D.y = B.y;
    }
    SG_TRY(hipMemcpyAsync(ws.wv_sell, sj.data(), sizeof(SellJob) * nsys, hipMemcpyHostToDevice, st));
    SG_TRY(launch_sell_jobs(ws.wv_sell, nsys, fblocks, true, prec, st));
    SG_TRY(hipMemcpyAsync(ws.wv_sys, desc.data(), sizeof(BatchSys) * nsys, hipMemcpyHostToDevice, st));
    SG_TRY(hipStreamSynchronize(st));  // the host vectors above are read by the copies
    SG_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(ws.wv_st), static_cast<int64_t>(sizeof(BatchState) / 4) * nsys,
                           0u, st));
    SG_TRY(hipMemsetAsync(&ws.sc->abort, 0, sizeof(int), st));

    // ---- |b| and the first residual of every system: two passes of the
    // tail jobs without a combine (the bits of launch_residual and
    // launch_norm_finish per system) ----------------------------------------
    std::vector<TailJob> t0(2 * static_cast<size_t>(nsys));  // read by a copy: kept to the next synchronisation
    {
        int rb = 0;
        for (int i = 0; i < nsys; ++i) {
            const sgmres_csr_t& A = systems[i].A;
            TailJob& a = t0[i];
            a = TailJob{};
            a.n = A.n;
            a.f = systems[i].b;
            a.r = sb[i].r;
            a.rblk0 = rb;
            a.rnblk = vec_grid(A.n);
            a.part = nullptr;  // set below, once the partial buffer is sized
            a.beta = &ws.wv_st[i].nf;  // pass 1: r = b, out[0] = |b|
            rb += a.rnblk;
            TailJob& c = t0[nsys + i];
            c = a;
            c.rp = A.row_ptr;
            c.ci = A.col_idx;
            c.val = A.val;
            c.x = systems[i].x;
            c.beta = &ws.wv_st[i].beta;  // pass 2: r = b - A x0, beta and rho
            c.nf = &ws.wv_st[i].nf;
        }
        SG_TRY(ensure(ws.wv_tpart, ws.wv_tpart_cap,
                      std::max(static_cast<size_t>(rb), static_cast<size_t>(L.capacity) * kMaxVecGrid)));
        for (auto& j : t0) j.part = ws.wv_tpart + j.rblk0;
        SG_TRY(ensure(ws.wv_tail0, ws.wv_tail0_cap, t0.size()));
        SG_TRY(hipMemcpyAsync(ws.wv_tail0, t0.data(), sizeof(TailJob) * t0.size(), hipMemcpyHostToDevice, st));
        SG_TRY(launch_tail_jobs(ws.wv_tail0, nsys, 0, rb, d, prec, st));
        SG_TRY(launch_tail_jobs(ws.wv_tail0 + nsys, nsys, 0, rb, d, prec, st));
    }
    std::vector<BatchState> hs(nsys);
    auto read_states = [&]() -> int {
        SG_TRY(hipMemcpyAsync(hs.data(), ws.wv_st, sizeof(BatchState) * nsys, hipMemcpyDeviceToHost, st));
        return copy_scalars(ws, st);  // synchronises
    };
    rc = read_states();
    if (rc) return rc;
    // status per system: 0 active, else the final code + 1 (codes are <= 0 or 1)
    std::vector<int> code(nsys, 0), done(nsys, 0), cycles(nsys, 0), steps(nsys, 0);
    for (int i = 0; i < nsys; ++i) {
        if (!std::isfinite(hs[i].nf)) {
            code[i] = SGMRES_ENONFINITE;
            done[i] = 1;
        } else if (hs[i].nf == 0.0) {
            SG_TRY(launch_fill(systems[i].x, systems[i].A.n, 0.0, st));
            hs[i].rho = 0.0;
            code[i] = SGMRES_OK;
            done[i] = 1;
        }
    }

    // ---- rounds -----------------------------------------------------------
    const int cap = L.capacity;
    const size_t sync_u32 = sync_words_bytes() / sizeof(unsigned);
    const size_t pab_u64 = static_cast<size_t>(4 * (kk + 1)) * cap;
    const size_t psk_dbl = static_cast<size_t>(2 * s * d + s) * cap;
    // B of one wave: at most cap groups, each column padded to 128 entries
    const size_t b_bytes = align_up(static_cast<size_t>(cap * L.rows + 128 * static_cast<int64_t>(cap)) * d * eb);
    const size_t lsq_bytes = align_up(lsq_sync_bytes() * cap);
    const size_t wave_bytes =
        align_up(sync_u32 * 4 * cap) + align_up(8 * pab_u64) + align_up(8 * psk_dbl) + b_bytes + lsq_bytes;
    SG_TRY(ensure(ws.wv_wave_arena, ws.wv_wave_arena_cap, wave_bytes));
    unsigned* w_sync = reinterpret_cast<unsigned*>(ws.wv_wave_arena);
    unsigned long long* w_pab = reinterpret_cast<unsigned long long*>(ws.wv_wave_arena + align_up(sync_u32 * 4 * cap));
    double* w_psk = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(w_pab) + align_up(8 * pab_u64));
    unsigned char* w_B = reinterpret_cast<unsigned char*>(w_psk) + align_up(8 * psk_dbl);
    void* w_lsq = w_B + b_bytes;  // publication counters of the pipelined least squares
    const bool pipe = s <= kLsqPipeMaxS;

    std::vector<int> order(nsys);
    for (int i = 0; i < nsys; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return systems[a].A.n > systems[b].A.n; });
    int status_all = SGMRES_OK;
    for (;;) {
        // decide every undecided system from its last residual (as sgmres_solve)
        std::vector<int> active;
        for (int i : order) {
            if (done[i]) continue;
            const double rho = hs[i].rho;
            if (!std::isfinite(rho)) code[i] = SGMRES_ENONFINITE, done[i] = 1;
            else if (rho <= tol) code[i] = SGMRES_OK, done[i] = 1;
            else if (cycles[i] > restarts) code[i] = SGMRES_NOT_CONVERGED, done[i] = 1;
            else active.push_back(i);
        }
        if (active.empty()) break;
        // first-fit waves, largest systems first
        std::vector<std::vector<int>> waves;
        {
            std::vector<int> room;
            for (int i : active) {
                const int G = static_cast<int>((systems[i].A.n + L.rows - 1) / L.rows);
                size_t w = 0;
                while (w < waves.size() && room[w] < G) ++w;
                if (w == waves.size()) {
                    waves.emplace_back();
                    room.push_back(cap);
                }
                waves[w].push_back(i);
                room[w] -= G;
            }
        }
        const size_t nw = waves.size();
        SG_TRY(ensure(ws.wv_ps, ws.wv_ps_cap, nw * cap));
        SG_TRY(ensure(ws.wv_idx, ws.wv_idx_cap, nw * 2 * cap));
        SG_TRY(ensure(ws.wv_jobs, ws.wv_jobs_cap, nw * cap));
        SG_TRY(ensure(ws.wv_tail, ws.wv_tail_cap, nw * cap));
        SG_TRY(ensure(ws.wv_tpart, ws.wv_tpart_cap, static_cast<size_t>(cap) * kMaxVecGrid));
        std::vector<ArnoldiParams> ps(nw * cap);
        std::vector<LsqJob> jobs(nw * cap);
        std::vector<TailJob> tails(nw * cap);
        std::vector<int> cblocks(nw, 0), rblocks(nw, 0);
        std::vector<int> idx(nw * 2 * cap, -1);
        std::vector<int> grids(nw);
        struct Slot {
            int sys;
            int64_t ldb;
            void* B;
        };
        std::vector<std::vector<Slot>> slots(nw);
        for (size_t w = 0; w < nw; ++w) {
            int blk0 = 0;
            size_t boff = 0;
            for (size_t g = 0; g < waves[w].size(); ++g) {
                const int i = waves[w][g];
                const sgmres_csr_t& A = systems[i].A;
                const int G = static_cast<int>((A.n + L.rows - 1) / L.rows);
                const int64_t ldb = (A.n + 127) / 128 * 128;
                void* B = w_B + boff;
                boff += align_up(static_cast<size_t>(ldb) * d * eb);
                ArnoldiParams& p = ps[w * cap + g];
                p = ArnoldiParams{};
                p.n = A.n;
                p.rp = A.row_ptr;
                p.sp = sb[i].sp;
                p.ci = sb[i].col;
                p.val = sb[i].val;
                p.r = sb[i].r;
                p.beta = &ws.wv_st[i].beta;
                p.B = B;
                p.ldb = ldb;
                p.SB = nullptr;
                p.SAB = sb[i].SAB;
                p.H = sb[i].H;
                p.g = sb[i].g;
                p.d = d;
                p.k = kk;
                p.s = s;
                p.zeta = zeta;
                p.seed = seed;
                p.cycle = static_cast<uint32_t>(cycles[i]);
                p.part_a = w_pab + static_cast<size_t>(4 * (kk + 1)) * blk0;
                p.part_b = p.part_a + static_cast<size_t>(2 * (kk + 1)) * G;
                p.part_sk = w_psk + static_cast<size_t>(2 * s * d + s) * blk0;
                p.sync = w_sync + sync_u32 * g;
                p.per_block_release = 0;
                p.abort = &ws.sc->abort;
                p.status = &ws.wv_st[i].dc;
                p.spin_limit = kSpinLimitTicks;
                p.phase_ticks = nullptr;
                p.spmv_mode = 0;
                p.hbuf = nullptr;
                p.xbits = nullptr;
                p.G = G;
                p.blk0 = blk0;
                for (int b = 0; b < G; ++b) idx[w * 2 * cap + blk0 + b] = static_cast<int>(g);
                idx[w * 2 * cap + cap + g] = i;
                LsqJob& J = jobs[w * cap + g];
                J.dc = &ws.wv_st[i].dc;
                J.C = sb[i].SAB;
                J.g = sb[i].g;
                J.tau = sb[i].tau;
                J.y = sb[i].y;
                J.dout = &ws.wv_st[i].rest;
                J.iout = &ws.wv_st[i].d_eff;
                J.sync = static_cast<unsigned char*>(w_lsq) + lsq_sync_bytes() * g;
                TailJob& T = tails[w * cap + g];
                T.n = A.n;
                T.d_eff = &ws.wv_st[i].d_eff;
                T.B = B;
                T.ldb = ldb;
                T.y = sb[i].y;
                T.x = systems[i].x;
                T.rp = A.row_ptr;
                T.ci = A.col_idx;
                T.val = A.val;
                T.f = systems[i].b;
                T.r = sb[i].r;
                T.beta = &ws.wv_st[i].beta;
                T.nf = &ws.wv_st[i].nf;
                T.cblk0 = cblocks[w];
                T.cnblk = A.n >= 4 ? combine4_grid(A.n) : 0;  // fewer rows: combined on its own
                cblocks[w] += T.cnblk;
                T.rblk0 = rblocks[w];
                T.rnblk = vec_grid(A.n);
                T.part = ws.wv_tpart + rblocks[w];
                rblocks[w] += T.rnblk;
                slots[w].push_back(Slot{i, ldb, B});
                blk0 += G;
            }
            grids[w] = (blk0 + 7) / 8 * 8;
        }
        SG_TRY(hipMemcpyAsync(ws.wv_ps, ps.data(), sizeof(ArnoldiParams) * ps.size(), hipMemcpyHostToDevice, st));
        SG_TRY(hipMemcpyAsync(ws.wv_idx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice, st));
        SG_TRY(hipMemcpyAsync(ws.wv_jobs, jobs.data(), sizeof(LsqJob) * jobs.size(), hipMemcpyHostToDevice, st));
        SG_TRY(hipMemcpyAsync(ws.wv_tail, tails.data(), sizeof(TailJob) * tails.size(), hipMemcpyHostToDevice, st));
        for (size_t w = 0; w < nw; ++w) {
            const int ng = static_cast<int>(waves[w].size());
            SG_TRY(launch_fill_u32(w_sync, static_cast<int64_t>(sync_u32) * ng, 0u, st));
            SG_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(w_pab), static_cast<int64_t>(2 * pab_u64), 0u, st));
            SG_TRY(arnoldi_multi_launch(L, grids[w], ws.wv_ps + w * cap, ws.wv_idx + w * 2 * cap, st));
            if (pipe)
                SG_TRY(launch_lsq_pipeline_batched(ng, s, d, ws.wv_jobs + w * cap, w_lsq, kappa_max, &ws.sc->abort,
                                                   kSpinLimitTicks, st));
            else
                SG_TRY(launch_lsq_batched(ng, s, ws.wv_sys, ws.wv_st, kappa_max, st, ws.wv_idx + w * 2 * cap + cap));
            // the wave's systems' combines, residuals and norms: one launch
            // each (a system of fewer than four rows is combined on its own)
            for (const Slot& sl : slots[w]) {
                const int i = sl.sys;
                const sgmres_csr_t& A = systems[i].A;
                if (A.n < 4)
                    SG_TRY(launch_combine(A.n, &ws.wv_st[i].d_eff, d, sl.B, sl.ldb, sb[i].y, systems[i].x, st,
                                          nullptr, prec));
            }
            SG_TRY(launch_tail_jobs(ws.wv_tail + w * cap, static_cast<int>(slots[w].size()), cblocks[w],
                                    rblocks[w], d, prec, st));
        }
        rc = read_states();  // also orders the host vectors' copies above
        if (rc) return rc;
        if (ws.host_sc->abort) return SGMRES_ETIMEOUT;
        for (int i : active) {
            ++cycles[i];
            steps[i] += hs[i].dc;
        }
    }
    for (int i = 0; i < nsys; ++i) {
        if (code[i] != SGMRES_OK) status_all = SGMRES_NOT_CONVERGED;
        if (results) {
            results[i].status = code[i];
            results[i].cycles = cycles[i];
            results[i].steps = steps[i];
            results[i].flags = hs[i].flags | hs[i].lsq_flags;
            results[i].relres = hs[i].rho;
        }
    }
    return status_all;
}


// A block of nb <= 32 right-hand sides sharing A, solved together: one
// streaming basis launch per cycle builds all nb bases, reading each nonzero
// of A once for all of them (pairs (row, right-hand side) interleaved), then
// per right-hand side the sketched least squares and x += B y.  A right-hand
// side that has converged (or run out of restarts) rides along as a zero
// basis.  Caller holds g_mutex and has checked A.
constexpr int kBlockRhs = 32;
int block_solve_locked(const sgmres_csr_t& A, int nb, const sgmres_system_t* sys, int d, int k, int s, uint64_t seed,
                       double tol, int restarts, int zeta, double kappa_max, int prec, sgmres_batch_result_t* res,
                       hipStream_t st) {
    constexpr int NR = kBlockRhs;
    if (nb < 1 || nb > NR) return SGMRES_EINVAL;
    const int64_t n = A.n;
    const int kk = (k > d - 1) ? (d > 1 ? d - 1 : 1) : k;
    if (kk > kStreamMaxK || !basis_sketch_fits(n, s, zeta)) return SGMRES_EINVAL;
    Workspace* wsp = nullptr;
    int rc = workspace(&wsp);
    if (rc) return rc;
    Workspace& ws = *wsp;
    StreamLaunch L{};
    if (stream_configure(n, NR, kk, prec, &L) != hipSuccess) return SGMRES_EINVAL;
    const size_t np = static_cast<size_t>(n) * NR;
    const int64_t ldb = static_cast<int64_t>((np + 127) / 128 * 128);
    const size_t eb = basis_elem_bytes(prec);
    SG_TRY(ensure(ws.mr_F, ws.mr_F_cap, np));
    SG_TRY(ensure(ws.mr_X, ws.mr_X_cap, np));
    SG_TRY(ensure(ws.mr_R, ws.mr_R_cap, np));
    SG_TRY(ensure(ws.mr_part, ws.mr_part_cap, static_cast<size_t>(multi_grid(n, NR)) * NR));
    SG_TRY(ensure(ws.mr_scal, ws.mr_scal_cap, static_cast<size_t>(6 * NR)));
    SG_TRY(ensure(ws.mr_int, ws.mr_int_cap, static_cast<size_t>(4 * NR)));
    SG_TRY(ensure(ws.mr_ptr, ws.mr_ptr_cap, static_cast<size_t>(2 * NR)));
    SG_TRY(ensure(ws.B, ws.B_cap, (static_cast<size_t>(ldb) * (d + 1) * eb + 7) / 8));
    SG_TRY(ensure(ws.H, ws.H_cap, static_cast<size_t>(NR) * (kk + 1) * d));
    SG_TRY(ensure(ws.SB, ws.SB_cap, static_cast<size_t>(NR) * s * (d + 1)));
    SG_TRY(ensure(ws.SAB, ws.SAB_cap, static_cast<size_t>(NR) * s * d));
    SG_TRY(ensure(ws.g, ws.g_cap, static_cast<size_t>(NR) * s));
    SG_TRY(ensure(ws.y, ws.y_cap, static_cast<size_t>(NR) * d));
    SG_TRY(ensure(ws.tau, ws.tau_cap, static_cast<size_t>(d)));
    SG_TRY(ensure(ws.part_ab, ws.part_ab_cap, static_cast<size_t>(4 * (kStreamMaxK + 1) * NR) * L.grid));
    SG_TRY(ensure(ws.st_lists, ws.st_lists_cap, static_cast<size_t>(basis_lists_words(n, s, zeta))));
    SG_TRY(ensure(ws.st_part, ws.st_part_cap,
                  static_cast<size_t>(basis_sketch_grid(n)) * (d + 1) * NR * static_cast<size_t>(s)));
    if (L.hst) SG_TRY(ensure(ws.st_state, ws.st_state_cap, np));
    rc = build_sell(ws, A, prec, st);
    if (rc) return rc;

    double* nf_d = ws.mr_scal;
    double* beta_d = nf_d + NR;
    double* rho_d = beta_d + NR;
    double* betak_d = rho_d + NR;
    double* rk_d = betak_d + NR;  // (rest, kappa) per right-hand side
    int* dc_d = ws.mr_int;
    int* fl_d = dc_d + NR;
    int* de_d = fl_d + NR;  // (d_eff, lsq flags) per right-hand side
    std::vector<void*> ptrs(2 * NR, nullptr);
    for (int r = 0; r < nb; ++r) {
        ptrs[r] = const_cast<double*>(sys[r].b);
        ptrs[NR + r] = sys[r].x;
    }
    SG_TRY(hipMemcpyAsync(ws.mr_ptr, ptrs.data(), sizeof(void*) * 2 * NR, hipMemcpyHostToDevice, st));
    SG_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(ws.mr_int), 4 * NR, 0u, st));
    SG_TRY(launch_pack(n, NR, reinterpret_cast<const double* const*>(ws.mr_ptr), ws.mr_F, st));
    SG_TRY(launch_pack(n, NR, reinterpret_cast<const double* const*>(ws.mr_ptr + NR), ws.mr_X, st));
    SG_TRY(launch_residual_multi(n, NR, A.row_ptr, A.col_idx, A.val, ws.mr_F, nullptr, ws.mr_R, ws.mr_part, nullptr,
                                 nf_d, nullptr, st));
    std::vector<double> hs(6 * NR);
    std::vector<int> hi(4 * NR);
    auto read_back = [&]() -> int {
        SG_TRY(hipMemcpyAsync(hs.data(), ws.mr_scal, sizeof(double) * 6 * NR, hipMemcpyDeviceToHost, st));
        SG_TRY(hipMemcpyAsync(hi.data(), ws.mr_int, sizeof(int) * 4 * NR, hipMemcpyDeviceToHost, st));
        SG_TRY(hipStreamSynchronize(st));
        return SGMRES_OK;
    };
    // b = 0 gives x = 0 (as sgmres_solve): pack those initial guesses as zero
    rc = read_back();
    if (rc) return rc;
    bool zero_b = false;
    for (int r = 0; r < nb; ++r)
        if (hs[r] == 0.0) {
            ptrs[NR + r] = nullptr;
            zero_b = true;
        }
    if (zero_b) {
        SG_TRY(hipMemcpyAsync(ws.mr_ptr + NR, ptrs.data() + NR, sizeof(void*) * NR, hipMemcpyHostToDevice, st));
        SG_TRY(launch_pack(n, NR, reinterpret_cast<const double* const*>(ws.mr_ptr + NR), ws.mr_X, st));
        for (int r = 0; r < nb; ++r) ptrs[NR + r] = sys[r].x;
        SG_TRY(hipMemcpyAsync(ws.mr_ptr + NR, ptrs.data() + NR, sizeof(void*) * NR, hipMemcpyHostToDevice, st));
        SG_TRY(hipStreamSynchronize(st));
    }
    std::vector<int> cycles(NR, 0), steps(NR, 0), flags(NR, 0), code(NR, SGMRES_NOT_CONVERGED);
    std::vector<char> done(NR, 1);
    for (int r = 0; r < nb; ++r) done[r] = 0;
    std::vector<double> relres(NR, 0.0), betak(NR, 0.0);
    SG_TRY(hipMemsetAsync(&ws.sc->abort, 0, sizeof(int), st));
    for (int c = 0;; ++c) {
        SG_TRY(launch_residual_multi(n, NR, A.row_ptr, A.col_idx, A.val, ws.mr_F, ws.mr_X, ws.mr_R, ws.mr_part, nf_d,
                                     beta_d, rho_d, st));
        rc = read_back();
        if (rc) return rc;
        if (c > 0) {
            SG_TRY(hipMemcpyAsync(ws.host_sc, ws.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
            SG_TRY(hipStreamSynchronize(st));
            if (ws.host_sc->abort) return SGMRES_ETIMEOUT;
        }
        int active = 0;
        for (int r = 0; r < nb; ++r) {
            if (done[r]) continue;
            if (c > 0) {
                steps[r] += hi[r];
                flags[r] |= hi[NR + r] | hi[2 * NR + 2 * r + 1];
            }
            const double rho = hs[2 * NR + r];
            relres[r] = rho;
            if (!std::isfinite(rho) || !std::isfinite(hs[r])) {
                code[r] = SGMRES_ENONFINITE;
                done[r] = 1;
            } else if (rho <= tol) {
                code[r] = SGMRES_OK;
                done[r] = 1;
            } else if (cycles[r] > restarts) {
                code[r] = SGMRES_NOT_CONVERGED;
                done[r] = 1;
            } else {
                ++active;
            }
        }
        if (!active) break;
        for (int r = 0; r < NR; ++r) betak[r] = (r < nb && !done[r]) ? hs[NR + r] : 0.0;
        SG_TRY(hipMemcpyAsync(betak_d, betak.data(), sizeof(double) * NR, hipMemcpyHostToDevice, st));
        const uint32_t cyc = static_cast<uint32_t>(c);
        SG_TRY(launch_fill_u32(ws.sync, static_cast<int64_t>(sync_words_bytes() / sizeof(unsigned)), 0u, st));
        SG_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(ws.part_ab),
                               static_cast<int64_t>(8 * (kStreamMaxK + 1) * NR) * L.grid, 0u, st));
        SG_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(dc_d), 2 * NR, 0u, st));
        StreamParams p{};
        p.n = n;
        p.sp = ws.cur_sp;
        p.ci = ws.cur_col;
        p.val = ws.cur_val;
        p.r = ws.mr_R;
        p.beta = betak_d;
        p.B = ws.B;
        p.ldb = ldb;
        p.H = ws.H;
        p.d = d;
        p.k = kk;
        p.part_a = ws.part_ab;
        p.part_b = ws.part_ab + static_cast<int64_t>(2 * (kStreamMaxK + 1) * NR) * L.grid;
        p.state = ws.st_state;
        p.sync = ws.sync;
        p.abort = &ws.sc->abort;
        p.dc_rhs = dc_d;
        p.flags_rhs = fl_d;
        p.spin_limit = kSpinLimitTicks;
        SG_TRY(stream_launch(L, p, st));
        SG_TRY(launch_basis_lists(n, seed, cyc, s, zeta, ws.st_lists, st));
        SG_TRY(launch_residual_sketch(n, ws.mr_R, NR, s, zeta, ws.st_lists, ws.st_part, ws.g, st));
        SG_TRY(launch_basis_sketch(n, ws.B, ldb, NR, prec, (d + 1) * NR, s, zeta, ws.st_lists, ws.st_part, ws.SB, st));
        SG_TRY(launch_relation(NR, d, kk, s, ws.H, ws.SB, dc_d, ws.SAB, st));
        SG_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(de_d), 2 * NR, 0u, st));
        for (int r = 0; r < nb; ++r) {
            if (done[r]) continue;
            double* C = ws.SAB + static_cast<int64_t>(r) * d * s;
            double* gr = ws.g + static_cast<int64_t>(r) * s;
            double* yr = ws.y + static_cast<int64_t>(r) * d;
            if (s <= kLsqPipeMaxS)
                SG_TRY(launch_lsq_pipeline(s, d, dc_d + r, 0, C, gr, ws.tau, kappa_max, yr, rk_d + 2 * r, de_d + 2 * r,
                                           ws.lsq_sync, &ws.sc->abort, kSpinLimitTicks, st));
            else
                SG_TRY(launch_lsq(s, dc_d + r, 0, C, gr, kappa_max, yr, rk_d + 2 * r, de_d + 2 * r, st));
            ++cycles[r];
        }
        SG_TRY(launch_combine_multi(n, NR, d, de_d, 2, ws.B, ldb, ws.y, ws.mr_X, prec, st));
    }
    SG_TRY(launch_unpack(n, NR, ws.mr_X, reinterpret_cast<double* const*>(ws.mr_ptr + NR), st));
    SG_TRY(hipStreamSynchronize(st));
    int all = SGMRES_OK;
    for (int r = 0; r < nb; ++r) {
        if (code[r] != SGMRES_OK) all = SGMRES_NOT_CONVERGED;
        if (res) {
            res[r].status = code[r];
            res[r].cycles = cycles[r];
            res[r].steps = steps[r];
            res[r].flags = flags[r];
            res[r].relres = relres[r];
        }
    }
    return all;
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" {

int sgmres_solve(const sgmres_csr_t* A, const double* b, double* x, int d, int k, int s, uint64_t seed,
                 double tol, int restarts, sgmres_info_t* info, void* stream) {
    return solve_entry(A, b, x, d, k, s, seed, tol, restarts, nullptr, info, stream);
}

int sgmres_solve_transposed(const sgmres_csr_t* A, const double* b, double* x, int d, int k, int s,
                            uint64_t seed, double tol, int restarts, sgmres_info_t* info, void* stream) {
    sgmres_options_t o{};
    o.transposed = 1;
    return solve_entry(A, b, x, d, k, s, seed, tol, restarts, &o, info, stream);
}

int sgmres_solve_ex(const sgmres_csr_t* A, const double* b, double* x, int d, int k, int s, uint64_t seed,
                    double tol, int restarts, const sgmres_options_t* opts, sgmres_info_t* info, void* stream) {
    return solve_entry(A, b, x, d, k, s, seed, tol, restarts, opts, info, stream);
}

struct sgmres_plan {
    sg::Plan p;
};

int sgmres_plan_create(const sgmres_csr_t* A, int flags, sgmres_plan_t** out, void* stream) {
    if (!out) return SGMRES_EINVAL;
    *out = nullptr;
    if (!csr_ok(A) || (flags & ~(SGMRES_PLAN_TRANSPOSE | SGMRES_PLAN_FP32))) return SGMRES_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lock(g_mutex);
    Workspace* ws = nullptr;
    int rc = workspace(&ws);
    if (rc) return rc;
    rc = check_csr(*ws, *A, st);
    if (rc) return rc;
    sgmres_plan* h = new (std::nothrow) sgmres_plan();
    if (!h) return SGMRES_ENOMEM;
    Plan& P = h->p;
    P.flags = flags;
    P.A = *A;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        delete h;
        return SGMRES_EHIP;
    }
    P.device = dev;
    const int64_t n = A->n;
    int* K = nullptr;
    int32_t* tscr = nullptr;
    auto cleanup = [&](int code) -> int {
        if (K) (void)hipFree(K);
        if (tscr) (void)hipFree(tscr);
        if (code != SGMRES_OK) {
            for (auto& row : P.sell)
                for (SellCopy& c : row) {
                    if (c.sp) (void)hipFree(c.sp);
                    if (c.col) (void)hipFree(c.col);
                    if (c.val) (void)hipFree(c.val);
                }
            if (P.t_rp) (void)hipFree(P.t_rp);
            if (P.t_ci) (void)hipFree(P.t_ci);
            if (P.t_val) (void)hipFree(P.t_val);
            delete h;
        }
        return code;
    };
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&K), sizeof(int) * ((n + 63) / 64));
    if (e != hipSuccess) return cleanup(to_code(e));
    rc = build_sell_copy(P.sell[0][0], K, P.A, SGMRES_PREC_FP64, st);
    if (!rc && (flags & SGMRES_PLAN_FP32)) rc = build_sell_copy(P.sell[0][1], K, P.A, SGMRES_PREC_FP32, st);
    if (rc) return cleanup(rc);
    if (flags & SGMRES_PLAN_TRANSPOSE) {
        const size_t nnz = static_cast<size_t>(A->nnz);
        e = hipMalloc(reinterpret_cast<void**>(&P.t_rp), sizeof(int32_t) * (n + 1));
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&P.t_ci), sizeof(int32_t) * (nnz ? nnz : 1));
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&P.t_val), sizeof(double) * (nnz ? nnz : 1));
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&tscr), sizeof(int32_t) * transpose_scratch_ints(n));
        if (e == hipSuccess)
            e = launch_csr_transpose(n, A->nnz, A->row_ptr, A->col_idx, A->val, P.t_rp, P.t_ci, P.t_val, tscr, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return cleanup(to_code(e));
        P.At = sgmres_csr_t{n, A->nnz, P.t_rp, P.t_ci, P.t_val};
        rc = build_sell_copy(P.sell[1][0], K, P.At, SGMRES_PREC_FP64, st);
        if (!rc && (flags & SGMRES_PLAN_FP32)) rc = build_sell_copy(P.sell[1][1], K, P.At, SGMRES_PREC_FP32, st);
        if (rc) return cleanup(rc);
    }
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return cleanup(to_code(e));
    cleanup(SGMRES_OK);
    *out = h;
    return SGMRES_OK;
}

int sgmres_plan_destroy(sgmres_plan_t* plan) {
    if (!plan) return SGMRES_OK;
    std::lock_guard<std::mutex> lock(g_mutex);
    Plan& P = plan->p;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(P.device);
    for (auto& row : P.sell)
        for (SellCopy& c : row) {
            if (c.sp) (void)hipFree(c.sp);
            if (c.col) (void)hipFree(c.col);
            if (c.val) (void)hipFree(c.val);
        }
    if (P.t_rp) (void)hipFree(P.t_rp);
    if (P.t_ci) (void)hipFree(P.t_ci);
    if (P.t_val) (void)hipFree(P.t_val);
    (void)hipSetDevice(cur);
    delete plan;
    return SGMRES_OK;
}

int sgmres_solve_plan(const sgmres_plan_t* plan, const double* b, double* x, int d, int k, int s, uint64_t seed,
                      double tol, int restarts, const sgmres_options_t* opts, sgmres_info_t* info, void* stream) {
    if (!plan) return SGMRES_EINVAL;
    return solve_entry(nullptr, b, x, d, k, s, seed, tol, restarts, opts, info, stream, &plan->p);
}

int sgmres_sketch_pattern(uint64_t seed, uint32_t cycle, int64_t i0, int64_t count, int s, int zeta,
                          int32_t* rows, int8_t* signs, void* stream) {
    if (count < 0 || i0 < 0 || s < 1 || s > 32767 || zeta < 1 || zeta > s || zeta > kMaxZeta ||
        (count > 0 && (!rows || !signs)))
        return SGMRES_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    SG_TRY(launch_sketch_pattern(seed, cycle, i0, count, s, zeta, rows, signs, st));
    SG_TRY(hipStreamSynchronize(st));
    return SGMRES_OK;
}

int sgmres_sketch_apply(int64_t n, const double* v, uint64_t seed, uint32_t cycle, int s, int zeta, double* g,
                        void* stream) {
    if (n < 0 || (n > 0 && !v) || !g || s < 1 || s > kMaxS || zeta < 1 || zeta > s || zeta > kMaxZeta)
        return SGMRES_EINVAL;
    std::lock_guard<std::mutex> lock(g_mutex);
    Workspace* ws = nullptr;
    int rc = workspace(&ws);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    SG_TRY(ensure(ws->part_sk, ws->part_sk_cap, static_cast<size_t>(s) * sketch_grid(n)));
    SG_TRY(launch_sketch_apply(n, v, seed, cycle, s, zeta, ws->part_sk, g, st));
    SG_TRY(hipStreamSynchronize(st));
    return SGMRES_OK;
}

int sgmres_residual(const sgmres_csr_t* A, const double* f, const double* x, double* r, double* norm,
                    void* stream) {
    if (!csr_ok(A) || !f || !x || !r) return SGMRES_EINVAL;
    std::lock_guard<std::mutex> lock(g_mutex);
    Workspace* ws = nullptr;
    int rc = workspace(&ws);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    SG_TRY(ensure(ws->part_vec, ws->part_vec_cap, static_cast<size_t>(kMaxVecGrid)));
    rc = check_csr(*ws, *A, st);
    if (rc) return rc;
    SG_TRY(launch_residual(A->n, A->row_ptr, A->col_idx, A->val, f, x, r, ws->part_vec, st));
    SG_TRY(launch_norm_finish(ws->part_vec, vec_grid(A->n), &ws->sc->beta, nullptr, st));
    rc = copy_scalars(*ws, st);
    if (rc) return rc;
    if (norm) *norm = ws->host_sc->beta;
    return SGMRES_OK;
}

int sgmres_arnoldi_cycle(const sgmres_csr_t* A, const double* r, int d, int k, int s, int zeta, uint64_t seed,
                         uint32_t cycle, double* B, int64_t ldb, double* SB, double* SAB, double* H, double* g,
                         int* dc, int* flags, void* stream) {
    if (!csr_ok(A) || !r || !B || !SB || !SAB || !H || !g || ldb < A->n) return SGMRES_EINVAL;
    if (d < 1 || d > kMaxD || k < 1 || k > 1024 || s < 1 || s > kMaxS || zeta < 1 || zeta > s || zeta > kMaxZeta)
        return SGMRES_EINVAL;
    std::lock_guard<std::mutex> lock(g_mutex);
    Workspace* ws = nullptr;
    int rc = workspace(&ws);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = A->n;
    SG_TRY(ensure(ws->r, ws->r_cap, static_cast<size_t>(n)));
    SG_TRY(ensure(ws->part_vec, ws->part_vec_cap, static_cast<size_t>(kMaxVecGrid)));
    ArnoldiLaunch L{};
    rc = prepare_arnoldi(*ws, n, d, k, s, zeta, 0, 0, &L, 1);
    if (rc) return rc;
    rc = check_csr(*ws, *A, st);
    if (rc) return rc;
    rc = build_sell(*ws, *A, SGMRES_PREC_FP64, st);
    if (rc) return rc;
    // |r| into the scalar block, r copied into the workspace residual
    SG_TRY(hipMemsetAsync(&ws->sc->dc, 0, 5 * sizeof(int), st));
    SG_TRY(launch_residual(n, nullptr, nullptr, nullptr, r, nullptr, ws->r, ws->part_vec, st));
    SG_TRY(launch_norm_finish(ws->part_vec, vec_grid(n), &ws->sc->beta, nullptr, st));
    SG_TRY(launch_fill(H, static_cast<int64_t>(k + 1) * d, 0.0, st));
    rc = run_cycle(*ws, *A, d, k, s, zeta, seed, cycle, L, B, ldb, SB, SAB, H, g, st);
    if (rc) return rc;
    rc = copy_scalars(*ws, st);
    if (rc) return rc;
    if (ws->host_sc->abort) return SGMRES_ETIMEOUT;
    if (dc) *dc = ws->host_sc->dc;
    if (flags) *flags |= ws->host_sc->flags;
    return SGMRES_OK;
}

int sgmres_chebyshev_cycle(const sgmres_csr_t* A, const double* r, int d, int s, int zeta, uint64_t seed,
                           uint32_t cycle, double c, double dx, double dy, double* B, int64_t ldb, double* SB,
                           double* SAB, double* colnorm, double* g, void* stream) {
    if (!csr_ok(A) || !r || !B || !SB || !SAB || !colnorm || !g || ldb < A->n) return SGMRES_EINVAL;
    if (d < 1 || d > kMaxD || s < 1 || s > kMaxS || zeta < 1 || zeta > s || zeta > kMaxZeta) return SGMRES_EINVAL;
    ChebCoef cf{};
    if (!cheb_coefficients(c, dx, dy, &cf)) return SGMRES_EINVAL;
    std::lock_guard<std::mutex> lock(g_mutex);
    Workspace* ws = nullptr;
    int rc = workspace(&ws);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = A->n;
    SG_TRY(ensure(ws->r, ws->r_cap, static_cast<size_t>(n)));
    SG_TRY(ensure(ws->part_vec, ws->part_vec_cap, static_cast<size_t>(kMaxVecGrid)));
    ArnoldiLaunch L{};
    rc = prepare_cheb(*ws, n, d, s, zeta, 0, 0, &L);
    if (rc) return rc;
    rc = check_csr(*ws, *A, st);
    if (rc) return rc;
    rc = build_sell(*ws, *A, SGMRES_PREC_FP64, st);
    if (rc) return rc;
    SG_TRY(hipMemsetAsync(&ws->sc->dc, 0, 5 * sizeof(int), st));
    SG_TRY(launch_residual(n, nullptr, nullptr, nullptr, r, nullptr, ws->r, ws->part_vec, st));
    SG_TRY(launch_norm_finish(ws->part_vec, vec_grid(n), &ws->sc->beta, nullptr, st));
    rc = run_cheb_cycle(*ws, *A, d, s, zeta, seed, cycle, L, cf, B, ldb, SB, SAB, colnorm, g, st);
    if (rc) return rc;
    rc = copy_scalars(*ws, st);
    if (rc) return rc;
    if (ws->host_sc->abort) return SGMRES_ETIMEOUT;
    return SGMRES_OK;
}

int sgmres_sketched_lsq(int s, int dc, double* C, double* g, double kappa_max, double* y, int* d_eff,
                        double* rest, double* kappa, int* flags, void* stream) {
    if (s < 1 || s > 32767 || dc < 0 || dc > s || dc > kLsqMaxCols || !C || !g || (dc > 0 && !y) ||
        !(kappa_max > 0))
        return SGMRES_EINVAL;
    std::lock_guard<std::mutex> lock(g_mutex);
    Workspace* ws = nullptr;
    int rc = workspace(&ws);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    SG_TRY(hipMemsetAsync(&ws->sc->d_eff, 0, 2 * sizeof(int), st));
    SG_TRY(hipMemsetAsync(&ws->sc->abort, 0, sizeof(int), st));
    rc = run_lsq(*ws, s, dc, nullptr, dc, C, g, kappa_max, y, st);
    if (rc) return rc;
    rc = copy_scalars(*ws, st);
    if (rc) return rc;
    if (ws->host_sc->abort) return SGMRES_ETIMEOUT;
    if (d_eff) *d_eff = ws->host_sc->d_eff;
    if (rest) *rest = ws->host_sc->rest;
    if (kappa) *kappa = ws->host_sc->kappa;
    if (flags) *flags |= ws->host_sc->lsq_flags;
    return SGMRES_OK;
}

int sgmres_basis_combine(int64_t n, int d_eff, const double* B, int64_t ldb, const double* y, double* x,
                         void* stream) {
    if (n < 1 || d_eff < 0 || d_eff > kMaxD || ldb < n || !x || (d_eff > 0 && (!B || !y))) return SGMRES_EINVAL;
    if (d_eff == 0) return SGMRES_OK;
    std::lock_guard<std::mutex> lock(g_mutex);
    Workspace* ws = nullptr;
    int rc = workspace(&ws);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    ws->host_sc->d_eff = d_eff;
    SG_TRY(hipMemcpyAsync(&ws->sc->d_eff, &ws->host_sc->d_eff, sizeof(int), hipMemcpyHostToDevice, st));
    SG_TRY(launch_combine(n, &ws->sc->d_eff, d_eff, B, ldb, y, x, st));
    SG_TRY(hipStreamSynchronize(st));
    return SGMRES_OK;
}

int sgmres_csr_transpose(const sgmres_csr_t* A, int32_t* t_row_ptr, int32_t* t_col_idx, double* t_val,
                         void* stream) {
    if (!csr_ok(A) || !t_row_ptr || (A->nnz > 0 && (!t_col_idx || !t_val))) return SGMRES_EINVAL;
    std::lock_guard<std::mutex> lock(g_mutex);
    Workspace* ws = nullptr;
    int rc = workspace(&ws);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    SG_TRY(ensure(ws->t_scratch, ws->t_scratch_cap, static_cast<size_t>(transpose_scratch_ints(A->n))));
    rc = check_csr(*ws, *A, st);
    if (rc) return rc;
    SG_TRY(launch_csr_transpose(A->n, A->nnz, A->row_ptr, A->col_idx, A->val, t_row_ptr, t_col_idx, t_val,
                                ws->t_scratch, st));
    SG_TRY(hipStreamSynchronize(st));
    return SGMRES_OK;
}

int sgmres_csr_outer_grad(const sgmres_csr_t* A, const double* u, const double* v, double alpha, double* dval,
                          void* stream) {
    if (!csr_ok(A) || !u || !v || (A->nnz > 0 && !dval)) return SGMRES_EINVAL;
    std::lock_guard<std::mutex> lock(g_mutex);
    Workspace* ws = nullptr;
    int rc = workspace(&ws);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = check_csr(*ws, *A, st);
    if (rc) return rc;
    SG_TRY(launch_csr_outer(A->n, A->row_ptr, A->col_idx, u, v, alpha, dval, st));
    SG_TRY(hipStreamSynchronize(st));
    return SGMRES_OK;
}

void sgmres_release_workspace(void) {
    std::lock_guard<std::mutex> lock(g_mutex);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_ws) {
        (void)hipSetDevice(kv.first);
        Workspace& w = kv.second;
        if (w.capture_stream) (void)hipStreamDestroy(w.capture_stream);
        void* ptrs[] = {w.bt_sys, w.bt_st, w.bt_task, w.bt_slots, w.bt_slot_off, w.bt_gcnt, w.bt_arena,
                        w.r, w.B, w.SB, w.SAB, w.H, w.g, w.y, w.tau, w.lsq_sync, w.part_ab, w.part_sk,
                        w.part_vec, w.part_nrm, w.colnorm, w.valf, w.hbuf, w.xbits, w.sell_K, w.sell_sp, w.sell_col,
                        w.sell_val, w.sync, w.sc, w.t_rp, w.t_ci, w.t_val,
                        w.t_scratch, w.st_lists, w.st_part, w.st_state, w.mr_F, w.mr_X, w.mr_R,
                        w.mr_part, w.mr_scal, w.mr_int, w.mr_ptr, w.wv_sys_arena, w.wv_wave_arena, w.wv_K,
                        w.wv_ps, w.wv_idx, w.wv_sys, w.wv_st, w.wv_jobs, w.wv_tail, w.wv_tpart, w.wv_tail0,
                        w.wv_sp, w.wv_sell};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
        if (w.host_sc) (void)hipHostFree(w.host_sc);
    }
    g_ws.clear();
    (void)hipSetDevice(cur);
}

int sgmres_solve_batched(int nsys, const sgmres_system_t* systems, int d, int k, int s, uint64_t seed, double tol,
                         int restarts, const sgmres_options_t* opts, sgmres_batch_result_t* results, void* stream) {
    // Systems of at least kBatchResidentRows rows fill the chip on their own:
    // they are solved one after another by the resident basis kernels (as
    // sgmres_solve_ex would), the rest together by the part-split kernel.
    const int zeta = (opts && opts->zeta) ? opts->zeta : 8;
    const int prec = opts ? opts->precision : SGMRES_PREC_FP64;
    if (prec != SGMRES_PREC_FP64 && prec != SGMRES_PREC_FP32 && prec != SGMRES_PREC_BF16_BASIS) return SGMRES_EINVAL;
    if (nsys < 0 || (nsys > 0 && !systems) || !(tol >= 0.0) || restarts < 0 || k < 1 || k > kBatchMaxK)
        return SGMRES_EINVAL;
    std::vector<int> big, small;
    for (int i = 0; i < nsys; ++i) {
        const sgmres_system_t& y = systems[i];
        if (!csr_ok(&y.A) || !y.b || !y.x || bad_sizes(y.A.n, d, k, s, zeta)) return SGMRES_EINVAL;
    }
    // Systems that share one matrix (the same CSR arrays) with at least
    // kBlockMinRows rows go, up to 32 at a time, to the block solve (one
    // streaming basis launch per cycle for all of them, each nonzero of A read
    // once per step for the whole block)
    std::vector<std::vector<int>> blocks;
    {
        std::map<std::tuple<const void*, const void*, const void*, int64_t>, std::vector<int>> by_matrix;
        for (int i = 0; i < nsys; ++i) {
            const sgmres_csr_t& A = systems[i].A;
            by_matrix[std::make_tuple(static_cast<const void*>(A.row_ptr), static_cast<const void*>(A.col_idx),
                                      static_cast<const void*>(A.val), A.n)]
                .push_back(i);
        }
        std::vector<char> in_block(nsys, 0);
        const bool blockable = k <= kStreamMaxK && !(opts && opts->path == SGMRES_PATH_PART_SPLIT);
        for (auto& kv : by_matrix) {
            std::vector<int>& v = kv.second;
            std::sort(v.begin(), v.end());
            const int64_t n = std::get<3>(kv.first);
            if (!blockable || v.size() < 2 || n < kBlockMinRows || !basis_sketch_fits(n, s, zeta)) continue;
            for (size_t q = 0; q < v.size(); q += kBlockRhs) {
                blocks.emplace_back(v.begin() + q, v.begin() + std::min(v.size(), q + kBlockRhs));
                for (size_t u = q; u < std::min(v.size(), q + kBlockRhs); ++u) in_block[v[u]] = 1;
            }
        }
        for (int i = 0; i < nsys; ++i)
            if (!in_block[i]) (systems[i].A.n >= kBatchResidentRows ? big : small).push_back(i);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    int all = SGMRES_OK;
    if (!big.empty() || !blocks.empty()) {
        // every CSR is checked before anything is solved
        std::lock_guard<std::mutex> lock(g_mutex);
        Workspace* wsp = nullptr;
        int rc = workspace(&wsp);
        if (rc) return rc;
        SG_TRY(hipMemsetAsync(&wsp->sc->csr_bad, 0, sizeof(int), st));
        for (int i = 0; i < nsys; ++i)
            SG_TRY(launch_csr_check(systems[i].A.n, systems[i].A.nnz, systems[i].A.row_ptr, systems[i].A.col_idx,
                                    &wsp->sc->csr_bad, st));
        rc = copy_scalars(*wsp, st);
        if (rc) return rc;
        if (wsp->host_sc->csr_bad) return SGMRES_ECSR;
    }
    for (const std::vector<int>& blk : blocks) {
        std::vector<sgmres_system_t> sub(blk.size());
        std::vector<sgmres_batch_result_t> sres(blk.size());
        for (size_t q = 0; q < blk.size(); ++q) sub[q] = systems[blk[q]];
        const double kmax = (opts && opts->kappa_max > 0) ? opts->kappa_max : 1e14;
        int rc;
        {
            std::lock_guard<std::mutex> lock(g_mutex);
            rc = block_solve_locked(sub[0].A, static_cast<int>(sub.size()), sub.data(), d, k, s, seed, tol, restarts,
                                    zeta, kmax, prec, sres.data(), st);
        }
        if (rc < 0) return rc;
        if (rc != SGMRES_OK) all = SGMRES_NOT_CONVERGED;
        if (results)
            for (size_t q = 0; q < blk.size(); ++q) results[blk[q]] = sres[q];
    }
    for (int i : big) {
        sgmres_options_t o{};
        o.zeta = zeta;
        o.kappa_max = opts ? opts->kappa_max : 0.0;
        o.precision = prec;
        sgmres_info_t info{};
        const int rc = solve_entry(&systems[i].A, systems[i].b, systems[i].x, d, k, s, seed, tol, restarts, &o,
                                   &info, stream);
        if (rc < 0 && rc != SGMRES_ENONFINITE) return rc;
        if (rc != SGMRES_OK) all = SGMRES_NOT_CONVERGED;
        if (results) {
            results[i].status = rc;
            results[i].cycles = info.cycles;
            results[i].steps = info.steps;
            results[i].flags = info.flags;
            results[i].relres = info.relres;
        }
    }
    if (small.empty()) return all;
    std::vector<sgmres_system_t> sub(small.size());
    std::vector<sgmres_batch_result_t> sres(small.size());
    for (size_t q = 0; q < small.size(); ++q) sub[q] = systems[small[q]];
    // the rest: several systems per resident basis launch (unless the
    // part-split kernel is asked for, or no instance fits the shape)
    const int path = opts ? opts->path : 0;
    const int kk = (k > d - 1) ? (d > 1 ? d - 1 : 1) : k;
    int rc = SGMRES_EINVAL;
    if (path != SGMRES_PATH_PART_SPLIT && kk <= kMultiMaxK) {
        const int R = (opts && opts->rows_per_thread == 2) ? 2 : 4;
        const double kmax = (opts && opts->kappa_max > 0) ? opts->kappa_max : 1e14;
        {
            // every CSR is checked before anything is solved
            std::lock_guard<std::mutex> lock(g_mutex);
            Workspace* wsp = nullptr;
            rc = workspace(&wsp);
            if (rc) return rc;
            SG_TRY(hipMemsetAsync(&wsp->sc->csr_bad, 0, sizeof(int), st));
            for (const sgmres_system_t& y : sub)
                SG_TRY(launch_csr_check(y.A.n, y.A.nnz, y.A.row_ptr, y.A.col_idx, &wsp->sc->csr_bad, st));
            rc = copy_scalars(*wsp, st);
            if (rc) return rc;
            if (wsp->host_sc->csr_bad) return SGMRES_ECSR;
        }
        {
            std::lock_guard<std::mutex> lock(g_mutex);
            rc = wave_solve_locked(static_cast<int>(sub.size()), sub.data(), d, k, s, seed, tol, restarts, zeta,
                                   kmax, prec, R, sres.data(), st);
        }
        if (rc == SGMRES_EINVAL && path == SGMRES_PATH_MULTI) return rc;
    }
    if (rc == SGMRES_EINVAL) {
        std::lock_guard<std::mutex> lock(g_mutex);
        rc = batch_solve_locked(static_cast<int>(sub.size()), sub.data(), d, k, s, seed, tol, restarts, opts,
                                sres.data(), st);
    }
    if (rc < 0) return rc;
    if (rc != SGMRES_OK) all = SGMRES_NOT_CONVERGED;
    if (results)
        for (size_t q = 0; q < small.size(); ++q) results[small[q]] = sres[q];
    return all;
}

int sgmres_chebyshev_box(const sgmres_csr_t* A, const double* r, int m, double* box, double* ritz, int* nritz,
                         void* stream) {
    if (!csr_ok(A) || !r || !box) return SGMRES_EINVAL;
    std::lock_guard<std::mutex> lock(g_mutex);
    Workspace* wsp = nullptr;
    int rc = workspace(&wsp);
    if (rc) return rc;
    return cheb_box_locked(*wsp, *A, r, m, box, ritz, nritz, static_cast<hipStream_t>(stream));
}

int sgmres_hessenberg_eigenvalues(int m, const double* H, int ldh, double* wr, double* wi) {
    if (m < 1 || ldh < m || !H || !wr || !wi) return SGMRES_EINVAL;
    std::vector<double> work(static_cast<size_t>(m) * m);
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) work[i + static_cast<size_t>(j) * m] = H[i + static_cast<size_t>(j) * ldh];
    return hessenberg_eigenvalues(m, work.data(), m, wr, wi) == 0 ? SGMRES_OK : SGMRES_EINVAL;
}

const char* sgmres_version(void) { return "sgmres-gfx950 0.1.0"; }

}  // extern "C"
