// Internal interfaces between the host driver and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sg {

constexpr int kMaxZeta = 32;  // largest sketch column sparsity supported

// ---- persistent basis kernel (arnoldi.hip) --------------------------------
struct ArnoldiParams {
    int64_t n;
    const int32_t* rp;
    const int64_t* sp;   // sliced ELL copy of A (sell.hip): slice starts,
    const int32_t* ci;   // columns
    const void* val;     // and values in the kernel's arithmetic type
    const double* r;     // cycle residual, n
    const double* beta;  // device scalar |r|
    void* B;             // n x d in the basis storage type, leading dim ldb
    int64_t ldb;
    double* SB;   // s x d
    double* SAB;  // s x d
    double* H;    // (k+1) x d
    double* g;    // s
    int d, k, s, zeta;
    uint64_t seed;
    uint32_t cycle;
    unsigned long long* part_a;  // (k+1) x G tagged partials (two words each), zero at launch
    unsigned long long* part_b;  // (k+1) x G tagged partials, zero at launch
    double* part_sk;  // (2s x G) per step for d steps, then s x G for g
    void* sync;       // SyncWords, zero at launch
    int per_block_release;
    int* abort;
    int* status;  // [0] columns built, [1] flags (OR)
    uint64_t spin_limit;
    unsigned long long* phase_ticks;  // null, or 8 accumulators (block 0's time per phase)
    int spmv_mode;                    // 0 row per thread, 1 CSR-stream through LDS
    // halo mode, n 64-bit words: FP32 arithmetic, the tagged basis entries of
    // the rows other blocks gather (bit i of xbits[i / 32]; zero at launch);
    // FP64, w of the current step
    void* hbuf;
    const unsigned* xbits;
    int G, blk0;  // several systems per launch: the group's blocks and first logical block
};

struct ArnoldiShape {
    int64_t n;
    int d, k, s, zeta;
    int block;            // 0 = auto
    int rows_per_thread;  // 0 = auto
    int force_global_window;
    int per_block_release;
    int sketch_basis;  // nonzero: the instance that also forms S b_j
    int precision;     // SGMRES_PREC_*
    int halo;          // nonzero: the two-barrier (halo) instance
};

struct ArnoldiLaunch {
    const void* fn;
    int block, R, KW, grid;
    size_t lds;
};

// doubles of the LDS value area: two staged vectors (also the SpMV product
// buffer), or the raw sketch pattern at init
__host__ __device__ constexpr int arnoldi_vals_doubles(int RB, int zeta) {
    return (2 * RB > (zeta * RB + 3) / 4) ? 2 * RB : (zeta * RB + 3) / 4;
}

size_t arnoldi_lds_bytes(int block, int R, int s, int k, int zeta);

// ---- Chebyshev box from a short Arnoldi pass (box.hip, host) ---------------
int hessenberg_eigenvalues(int m, double* H, int ldh, double* wr, double* wi);
void box_from_ritz(int m, const double* wr, const double* wi, double margin, double box[3]);
// ---- several systems per basis launch (arnoldi_multi.hip) ------------------
constexpr int kMultiBlock = 1024;  // threads per workgroup
constexpr int kMultiMaxK = 4;      // register window of the instances
struct MultiLaunch {
    const void* fn;
    int R;
    int64_t rows;   // rows per workgroup (R * kMultiBlock)
    int capacity;   // workgroups that can be resident at once
    size_t lds;
};
hipError_t arnoldi_multi_configure(int R, int k, int s, int zeta, int precision, MultiLaunch* out);
// grid: a multiple of 8 (XCD-aware block numbering) up to capacity; ps: one
// ArnoldiParams per group (G, blk0 set); grp: group of each logical block
hipError_t arnoldi_multi_launch(const MultiLaunch& L, int grid, const ArnoldiParams* ps, const int* grp,
                                hipStream_t stream);

hipError_t arnoldi_configure(const ArnoldiShape& shape, ArnoldiLaunch* out);
hipError_t arnoldi_launch(const ArnoldiLaunch& L, ArnoldiParams params, hipStream_t stream);
size_t sync_words_bytes();
// instance of the basis kernel that also forms S b_j (arnoldi_sb.hip)
const void* arnoldi_pick_sb(int block, int R, int KW);
// FP32 arithmetic with an FP32 / bfloat16 basis (arnoldi_f32.hip, arnoldi_bf16.hip)
const void* arnoldi_pick_f32(int block, int R, int KW);
const void* arnoldi_pick_bf16(int block, int R, int KW);
// two-barrier (halo) solve instances (arnoldi_halo_*.hip)
const void* arnoldi_pick_halo_f64(int block, int R, int KW);
const void* arnoldi_pick_halo_f32(int block, int R, int KW);
const void* arnoldi_pick_halo_bf16(int block, int R, int KW);
// bytes of one stored basis entry for SGMRES_PREC_*
inline size_t basis_elem_bytes(int precision) { return precision == 1 ? 4 : (precision == 2 ? 2 : 8); }

// ---- Chebyshev basis kernel (chebyshev.hip) --------------------------------
struct ChebParams {
    int64_t n;
    const int32_t* rp;
    const int64_t* sp;   // sliced ELL copy of A (sell.hip): slice starts,
    const int32_t* ci;   // columns
    const void* val;     // and values in the kernel's arithmetic type
    const double* r;     // cycle residual, n
    const double* beta;  // device scalar |r|
    void* B;             // n x d raw recurrence vectors (storage type), leading dim ldb
    int64_t ldb;
    double* SB;       // s x d, sketches of the normalised columns (when sketch_basis)
    double* SAB;      // s x d, S A of the normalised columns
    double* colnorm;  // d, |B[:, j]|
    double* g;        // s
    int d, s, zeta;
    uint64_t seed;
    uint32_t cycle;
    double c;   // centre of the spectral box
    double a1;  // B[:,1] = a1 (A - c) B[:,0]
    double a;   // B[:,j+1] = a (A - c) B[:,j] - q B[:,j-1]
    double q;
    double* part_sk;   // (2s x G) per step for d steps, then s x G for g
    double* part_nrm;  // d x G
    void* sync;        // SyncWords, zero at launch
    int per_block_release;
    int* abort;
    int* status;  // [0] columns built
    uint64_t spin_limit;
    unsigned long long* phase_ticks;
    int sketch_basis;
};

size_t chebyshev_lds_bytes(int block, int R, int s, int zeta);
hipError_t chebyshev_configure(const ArnoldiShape& shape, ArnoldiLaunch* out);
hipError_t chebyshev_launch(const ArnoldiLaunch& L, ChebParams params, hipStream_t stream);

// ---- streaming basis kernel (stream.hip) ----------------------------------
// k-truncated Arnoldi for systems beyond the resident capacity and for blocks
// of NR right-hand sides sharing A (pairs q = i * NR + rhs; see stream_kernel.hpp).
constexpr int kStreamBlock = 1024;
constexpr int kStreamMaxK = 4;
struct StreamParams {
    int64_t n;
    const int64_t* sp;   // sliced ELL copy of A: slice starts,
    const int32_t* ci;   // columns
    const void* val;     // and values in the arithmetic type
    const double* r;     // residuals, n * NR (pair order)
    const double* beta;  // NR norms of r
    void* B;             // d + 1 columns of n * NR entries (storage type), column stride ldb
    int64_t ldb;
    double* H;           // per right-hand side (k+1) x d, H[(rhs * d + j) * (k+1) + a]
    int d, k;
    unsigned long long* part_a;  // NR (k+1) x G tagged partials (two words each), zero at launch
    unsigned long long* part_b;
    void* state;         // HBM-state instances: n * NR entries (arithmetic type)
    void* sync;          // SyncWords, zero at launch
    int per_block_release;
    int* abort;
    int* status;         // NR = 1: [0] columns built, [1] flags (OR)
    int* dc_rhs;         // NR > 1: columns built per right-hand side
    int* flags_rhs;      // NR > 1: flags per right-hand side (OR)
    uint64_t spin_limit;
    unsigned long long* phase_ticks;
    int nl;              // register state: newest basis columns kept in the LDS ring (0..4)
};
struct StreamLaunch {
    const void* fn;
    int NR, P, hst, grid;
    int nl;              // LDS ring columns (register state)
    size_t lds;          // dynamic LDS bytes
};
// precision SGMRES_PREC_*; nr right-hand sides (1 or a divisor of 64)
hipError_t stream_configure(int64_t n, int nr, int k, int precision, StreamLaunch* out);
hipError_t stream_launch(const StreamLaunch& L, StreamParams params, hipStream_t stream);

// ---- sketch of a finished basis (sketch_basis.hip) --------------------------
// lists: the cycle's sparse sign pattern per 512-row chunk, basis_lists_words
// 32-bit words; part: basis_sketch_grid(n) * nvec * s doubles; SB: nvec * s
// (vector v = column v / nr, right-hand side v % nr; column-major s x nvec).
// Requires basis_sketch_fits(n, s, zeta) (s <= 1024, n < 2^26).
int64_t basis_lists_words(int64_t n, int s, int zeta);
int basis_sketch_grid(int64_t n);
bool basis_sketch_fits(int64_t n, int s, int zeta);
hipError_t launch_basis_lists(int64_t n, uint64_t seed, uint32_t cycle, int s, int zeta, uint32_t* lists,
                              hipStream_t stream);
hipError_t launch_basis_sketch(int64_t n, const void* B, int64_t ldb, int nr, int precision, int nvec, int s,
                               int zeta, const uint32_t* lists, double* part, double* SB, hipStream_t stream);
// g (nr x s, right-hand side-major) = S r for nr interleaved FP64 residuals
// (n * nr entries); part as above with nvec = nr
hipError_t launch_residual_sketch(int64_t n, const double* r, int nr, int s, int zeta, const uint32_t* lists,
                                  double* part, double* g, hipStream_t stream);
// S A B per right-hand side from S B and H (Arnoldi relation); dc_dev: 1 or nr ints
hipError_t launch_relation(int nr, int d, int k, int s, const double* H, const double* SB, const int* dc_dev,
                           double* SAB, hipStream_t stream);

// ---- blocks of right-hand sides, interleaved (multi.hip) -------------------
constexpr int kMultiMaxGrid = 2048;
int multi_grid(int64_t n, int nr);  // workgroups of the residual (slots of part)
// dst[i nr + r] = src[r][i] (src[r] null: 0); dst[r][i] = src[i nr + r] (dst[r] null: skipped)
hipError_t launch_pack(int64_t n, int nr, const double* const* src, double* dst, hipStream_t stream);
hipError_t launch_unpack(int64_t n, int nr, const double* src, double* const* dst, hipStream_t stream);
// R = F - A X (X null: R = F); out[r] = |R_r|, rel[r] = out[r] / nf[r] when nf
// is given; part: multi_grid(n, nr) * nr doubles
hipError_t launch_residual_multi(int64_t n, int nr, const int32_t* rp, const int32_t* ci, const double* val,
                                 const double* F, const double* X, double* R, double* part, const double* nf,
                                 double* out, double* rel, hipStream_t stream);
// X += B[:, :d_eff[r dstride]] y_r per right-hand side (B interleaved, column stride ldb)
hipError_t launch_combine_multi(int64_t n, int nr, int d, const int* d_eff, int dstride, const void* B, int64_t ldb,
                                const double* y, double* X, int precision, hipStream_t stream);

// ---- batched solve (batched.hip) ------------------------------------------
// One descriptor per system (device copy); the basis, scratch vectors and the
// sketch lists of a system live at its own offsets in the batch workspace.
struct BatchSys {
    int64_t n;
    const int32_t* rp;
    const int32_t* ci;
    const double* val;   // FP64 values (residual)
    const void* valc;    // values in the cycle's arithmetic type
    const double* b;
    double* x;
    void* B;             // n x d, storage type, leading dim n
    void* m;             // n, arithmetic type: A b_j of the current step
    void* w;             // n, arithmetic type: first Gram-Schmidt update
    double* r;           // n: residual
    uint16_t* lists;     // per chunk of CH rows: zeta * CH entries (sorted sketch lists)
    int* lstart;         // per chunk: s + 1 list starts
    double* SAB;         // s x d
    double* g;           // s
    double* y;           // d
};

// Per-system state, kept across the cycles of one batched solve.
struct BatchState {
    double nf;      // |b|
    double beta;    // |r| of the last residual
    double rho;     // |r| / |b|
    double rest;    // least-squares residual estimate   (rest, kappa adjacent:
    double kappa;   // diagonal ratio of T                 the LSQ writes both)
    int d_eff;      // columns used by the least squares   (d_eff, lsq_flags
    int lsq_flags;  //                                       adjacent likewise)
    int status;     // as of the start of the cycle: 0 active, 1 converged,
                    // 2 out of restarts, 3 non-finite, 4 wait limit hit
    int next;       // status decided during the cycle (copied at its end)
    int dc;         // columns built in the last cycle
    int flags;      // OR of breakdown flags
    int cycles;     // basis cycles run
    int steps;      // basis columns built, summed
};

// A unit of work: rows [r0, r1) (whole chunks) of one system; the nparts parts
// of a system are consecutive in the task list and synchronise with each
// other through the system's counter.
struct BatchTask {
    int sys;
    int part;
    int nparts;
    int pad;
    int64_t r0, r1;
};

struct BatchParams {
    int ntask;
    const BatchTask* task;
    const BatchSys* sys;
    BatchState* st;
    double* slots;       // per system: 2 x kBatchRed x nparts reduction slots, then s x nparts sketch slots
    const int64_t* slot_off;  // per system: offset of its slots (doubles)
    unsigned* gcnt;      // per system: arrivals at the group barrier this cycle
    int* queue;          // next task (zero at launch)
    int* active;         // systems that built a basis this cycle
    const int* cycle;    // device cycle counter (the counter array of launch_batch_advance)
    int* abort;          // raised when a group wait exceeds its limit
    uint64_t spin_limit;
    int d, k, s, zeta;
    int restarts;
    uint64_t seed;
    double tol;
};

struct BatchLaunch {
    const void* fn;
    int block, R, grid;
    size_t lds;
};
constexpr int kBatchMaxK = 4;
constexpr int kBatchRed = kBatchMaxK + 1;  // values per group reduction (window dots + a norm)
constexpr int kBatchMaxParts = 256;         // parts per system; the group sums load at most 4 per lane
// chunk rows a kernel instance handles at a time
inline int batch_chunk(const BatchLaunch& L) { return L.block * L.R; }
hipError_t batch_configure(int block, int R, int d, int s, int zeta, int precision, BatchLaunch* out);
hipError_t batch_launch(const BatchLaunch& L, const BatchParams& p, hipStream_t stream);
// ctr (4 ints): [0] cycle, [1] queue position, [2] active systems, [3] active
// systems of the cycle that just ended.  advance: end of a cycle (also moves
// each system's decided status into place and clears the group counters);
// reset: start of a solve (clears every BatchState and counter).
hipError_t launch_batch_advance(int* ctr, BatchState* st, unsigned* gcnt, int nsys, hipStream_t stream);
hipError_t launch_batch_reset(BatchState* st, unsigned* gcnt, int nsys, int* ctr, hipStream_t stream);
// One system of a batched pipelined least squares: its dc (device), C = S A B
// (s x d, overwritten), g (s, overwritten), tau (d scratch), y (d out),
// dout (rest, kappa), iout (d_eff, flags |=), sync (lsq_sync_bytes(), per job)
struct LsqJob {
    const int* dc;
    double* C;
    double* g;
    double* tau;
    double* y;
    double* dout;
    int* iout;
    void* sync;
};
// jobs (device array of njobs) run concurrently, each on the workgroups of
// launch_lsq_pipeline; syncs: njobs consecutive sync blocks (cleared here);
// s <= 512
hipError_t launch_lsq_pipeline_batched(int njobs, int s, int d_max, const LsqJob* jobs, void* syncs,
                                       double kappa_max, int* abort, uint64_t limit, hipStream_t stream);
hipError_t launch_lsq_batched(int nsys, int s, const BatchSys* sys, BatchState* st, double kappa_max,
                              hipStream_t stream, const int* idx = nullptr);

// ---- sliced ELL copy of A for the basis kernels (sell.hip) ----------------
// K[i] = longest row of slice i (rows 64 i .. 64 i + 63); sp = exclusive prefix
// of 64 K; scol / sval (sval in the basis arithmetic type: double for
// SGMRES_PREC_FP64, float otherwise) hold sp[nslices] entries.
hipError_t launch_sell_width(int64_t n, const int32_t* rp, int* K, hipStream_t stream);
// Several matrices' width or fill passes in one launch (the batched solve):
// each job's blocks [wblk0, wblk0 + wnblk) / [fblk0, fblk0 + fnblk) do what
// launch_sell_width / launch_sell_fill do for that matrix; jobs in block order.
struct SellJob {
    int64_t n;
    const int32_t* rp;
    const int32_t* ci;
    const double* val;
    int* K;             // width pass output, (n + 63) / 64 entries
    const int64_t* sp;  // fill pass input
    int32_t* scol;
    void* sval;
    int wblk0, wnblk;
    int fblk0, fnblk;
};
int sell_width_blocks(int64_t n);
int sell_fill_blocks(int64_t n);
hipError_t launch_sell_jobs(const SellJob* jobs, int njobs, int blocks, bool fill, int precision,
                            hipStream_t stream);
hipError_t launch_sell_fill(int64_t n, const int32_t* rp, const int32_t* ci, const double* val, const int64_t* sp,
                            int32_t* scol, void* sval, int precision, hipStream_t stream);

// ---- vector kernels (vec.hip) ----------------------------------------------
constexpr int kVecBlock = 256;
int vec_grid(int64_t n);  // blocks used by the partial-sum kernels (<= kMaxVecGrid)
constexpr int kMaxVecGrid = 1024;

// r = f - A x (x may be null: r = f); partial |r|^2 per block into part[G]
hipError_t launch_residual(int64_t n, const int32_t* rp, const int32_t* ci, const double* val,
                           const double* f, const double* x, double* r, double* part,
                           hipStream_t stream);
// out[0] = sqrt(sum part[0..G)); if nf != null also out[1] = out[0] / *nf
hipError_t launch_norm_finish(const double* part, int G, double* out, const double* nf,
                              hipStream_t stream);
// bad[0] |= 1 when the CSR arrays are malformed
hipError_t launch_csr_check(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, int* bad,
                            hipStream_t stream);
// out[0] += nonzeros (i, c) of A with c / RB != i / RB (columns outside the
// row's block of RB rows)
hipError_t launch_offblock_count(int64_t n, const int32_t* rp, const int32_t* ci, int64_t RB,
                                 unsigned long long* out, unsigned* xbits, hipStream_t stream);
// dval[q] = alpha * u[row(q)] * v[col(q)] on the sparsity pattern of A
hipError_t launch_csr_outer(int64_t n, const int32_t* rp, const int32_t* ci, const double* u, const double* v,
                            double alpha, double* dval, hipStream_t stream);
// x[i] = v  for i < n
hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t stream);
hipError_t launch_fill_u32(unsigned* x, int64_t n, unsigned v, hipStream_t stream);
// x += B[:, :*d_eff] y, or x += B[:, :*d_eff] (y ./ colnorm) when colnorm is
// given (columns with colnorm 0 are skipped); B stored per SGMRES_PREC_*
hipError_t launch_combine(int64_t n, const int* d_eff, int d_max, const void* B, int64_t ldb,
                          const double* y, double* x, hipStream_t stream, const double* colnorm = nullptr,
                          int precision = 0);
// The tail of one system's cycle in a multi-system wave: x += B y (blocks
// [cblk0, cblk0 + cnblk) of the combine launch; cnblk = 0: not in it), then
// r = f - A x with block partials of |r|^2 (blocks [rblk0, rblk0 + rnblk),
// rnblk = vec_grid(n)), then beta[0] = |r|, beta[1] = |r| / *nf.  Jobs are in
// block order in both launches.
struct TailJob {
    int64_t n;
    const int* d_eff;
    const void* B;  // aligned to four entries, as is ldb
    int64_t ldb;
    const double* y;
    double* x;
    const int32_t* rp;
    const int32_t* ci;
    const double* val;
    const double* f;
    double* r;
    double* part;  // rnblk partials
    double* beta;
    const double* nf;
    int cblk0, cnblk;
    int rblk0, rnblk;
};
// blocks of the four-rows-per-thread combine for n rows
int combine4_grid(int64_t n);
hipError_t launch_tail_jobs(const TailJob* jobs, int njobs, int cblocks, int rblocks, int d_max, int precision,
                            hipStream_t stream);
// out[i] = (float) in[i]
hipError_t launch_to_f32(int64_t count, const double* in, float* out, hipStream_t stream);

// ---- sketch kernels (sketch.hip) -------------------------------------------
hipError_t launch_sketch_pattern(uint64_t seed, uint32_t cycle, int64_t i0, int64_t count, int s,
                                 int zeta, int32_t* rows, int8_t* signs, hipStream_t stream);
// g = S v using part (s x G workspace, G = sketch_grid(n)); dynamic LDS of
// sketch_apply_lds_bytes(s, zeta) (at most 159,752 bytes for s <= 4096, zeta <= 32)
int sketch_grid(int64_t n);
size_t sketch_apply_lds_bytes(int s, int zeta);
hipError_t launch_sketch_apply(int64_t n, const double* v, uint64_t seed, uint32_t cycle, int s,
                               int zeta, double* part, double* g, hipStream_t stream);

// ---- sketched least squares (lsq.hip) --------------------------------------
// dc read from *dc_dev (device) when dc_dev != null, else dc_host.
// dout: [0] rest, [1] kappa; iout: [0] d_eff, [1] flags (OR)
hipError_t launch_lsq(int s, const int* dc_dev, int dc_host, double* C, double* g,
                      double kappa_max, double* y, double* dout, int* iout, hipStream_t stream);
constexpr int kLsqMaxCols = 1024;
// Column-owner pipeline version for s <= 512: one wavefront per column of C
// (and one for g); tau needs d_max doubles, sync lsq_sync_bytes() (cleared here).
constexpr int kLsqPipeMaxS = 512;
size_t lsq_sync_bytes();
hipError_t launch_lsq_pipeline(int s, int d_max, const int* dc_dev, int dc_host, double* C, double* g, double* tau,
                               double kappa_max, double* y, double* dout, int* iout, void* sync, int* abort,
                               uint64_t limit, hipStream_t stream);

// ---- CSR transpose (transpose.hip) -----------------------------------------
// scratch: transpose_scratch_ints(n) int32 (counts, fill counters, scan tile sums)
int64_t transpose_scratch_ints(int64_t n);
hipError_t launch_csr_transpose(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci,
                                const double* val, int32_t* trp, int32_t* tci, double* tval,
                                int32_t* scratch, hipStream_t stream);

}  // namespace sg
