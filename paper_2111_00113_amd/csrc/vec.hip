// Bandwidth-bound vector kernels of the sGMRES cycle (arXiv:2111.00113):
//   residual r = f - A x with partial |r|^2   (Algorithm 1, residual step)
//   norm finish (fixed-order sum of block partials)
//   basis combine x <- x + B y                (Section 3.3, solution step)
//   fills (graph-capture-safe clears)
#include "common.hpp"
#include "internal.hpp"

namespace sg {

int vec_grid(int64_t n) {
    const int64_t g = (n + kVecBlock - 1) / kVecBlock;
    return static_cast<int>(g < 1 ? 1 : (g > kMaxVecGrid ? kMaxVecGrid : g));
}

namespace {

// Block blk of nblk: rows blk * kVecBlock + t + k * nblk * kVecBlock; its
// partial |r|^2 into part[blk].
__device__ __forceinline__ void residual_body(int blk, int nblk, int64_t n, const int32_t* __restrict__ rp,
                                              const int32_t* __restrict__ ci, const double* __restrict__ val,
                                              const double* __restrict__ f, const double* __restrict__ x,
                                              double* __restrict__ r, double* __restrict__ part) {
    __shared__ double tmp[kVecBlock / kWave];
    __shared__ double out[1];
    double acc = 0.0;
    const int64_t stride = static_cast<int64_t>(nblk) * kVecBlock;
    for (int64_t i = static_cast<int64_t>(blk) * kVecBlock + threadIdx.x; i < n; i += stride) {
        double ax = 0.0;
        if (x) {
            const int q1 = rp[i + 1];
            for (int q = rp[i]; q < q1; ++q) ax = madd(val[q], x[ci[q]], ax);
        }
        const double ri = f[i] - ax;
        r[i] = ri;
        acc = madd(ri, ri, acc);
    }
    const double v[1] = {acc};
    block_sum<1>(v, 1, tmp, out);
    if (threadIdx.x == 0) part[blk] = out[0];
}

__global__ __launch_bounds__(kVecBlock) void residual_kernel(int64_t n, const int32_t* __restrict__ rp,
                                                             const int32_t* __restrict__ ci,
                                                             const double* __restrict__ val,
                                                             const double* __restrict__ f,
                                                             const double* __restrict__ x,
                                                             double* __restrict__ r,
                                                             double* __restrict__ part) {
    residual_body(blockIdx.x, gridDim.x, n, rp, ci, val, f, x, r, part);
}

__device__ __forceinline__ void norm_finish_body(const double* __restrict__ part, int G, double* __restrict__ out,
                                                 const double* __restrict__ nf) {
    __shared__ double res[1];
    grid_sum(part, G, 1, res);
    if (threadIdx.x == 0) {
        const double nrm = sqrt(res[0]);
        out[0] = nrm;
        if (nf) out[1] = nrm / *nf;
    }
}

__global__ __launch_bounds__(kVecBlock) void norm_finish_kernel(const double* __restrict__ part, int G,
                                                                double* __restrict__ out,
                                                                const double* __restrict__ nf) {
    norm_finish_body(part, G, out, nf);
}

__global__ void fill_kernel(double* x, int64_t n, double v) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = v;
}

__global__ void fill_u32_kernel(unsigned* x, int64_t n, unsigned v) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = v;
}

// x[i] += sum_{c < d_eff} B[c*ldb + i] y[c]; y staged in LDS; eight columns in
// flight per thread.
constexpr int kCombineBlock = 256;
template <typename TS>
__global__ __launch_bounds__(kCombineBlock) void combine_kernel(int64_t n, const int* __restrict__ d_eff_p,
                                                                const TS* __restrict__ B, int64_t ldb,
                                                                const double* __restrict__ y,
                                                                double* __restrict__ x,
                                                                const double* __restrict__ cn) {
    extern __shared__ double ys[];
    const int d_eff = *d_eff_p;
    for (int c = threadIdx.x; c < d_eff; c += kCombineBlock)
        ys[c] = cn ? (cn[c] > 0.0 ? y[c] / cn[c] : 0.0) : y[c];
    __syncthreads();
    if (d_eff <= 0) return;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kCombineBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kCombineBlock + threadIdx.x; i < n; i += stride) {
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int c = 0;
        for (; c + 8 <= d_eff; c += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u)
                acc[u] = madd(from_basis<double>(B[static_cast<int64_t>(c + u) * ldb + i]), ys[c + u], acc[u]);
        }
        for (; c < d_eff; ++c) acc[0] = madd(from_basis<double>(B[static_cast<int64_t>(c) * ldb + i]), ys[c], acc[0]);
        const double sum = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        x[i] += sum;
    }
}

// Four consecutive basis entries of one column as doubles, with one 16-byte
// load (FP32), two (FP64) or one 8-byte load (bfloat16); p must be aligned to
// the four entries.
__device__ __forceinline__ void load_quad(const double* p, double (&o)[4]) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    o[0] = a.x;
    o[1] = a.y;
    o[2] = b.x;
    o[3] = b.y;
}
__device__ __forceinline__ void load_quad(const float* p, double (&o)[4]) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    o[0] = a.x;
    o[1] = a.y;
    o[2] = a.z;
    o[3] = a.w;
}
__device__ __forceinline__ void load_quad(const bf16_t* p, double (&o)[4]) {
    const uint2 a = *reinterpret_cast<const uint2*>(p);
    o[0] = from_basis<double>(bf16_t{static_cast<uint16_t>(a.x & 0xffffu)});
    o[1] = from_basis<double>(bf16_t{static_cast<uint16_t>(a.x >> 16)});
    o[2] = from_basis<double>(bf16_t{static_cast<uint16_t>(a.y & 0xffffu)});
    o[3] = from_basis<double>(bf16_t{static_cast<uint16_t>(a.y >> 16)});
}

// combine_kernel with four consecutive rows per thread: each column is read in
// runs of 64 x 4 entries per wavefront, sixteen columns in flight, and every row
// keeps two interleaved sums (even and odd columns).  Needs B and ldb aligned
// to four entries; the n % 4 last rows are done by block 0 one per thread.
constexpr int kCombineCols = 16;
// Block blk of nblk; the n % 4 last rows by block 0.
template <typename TS>
__device__ __forceinline__ void combine4_body(int blk, int nblk, int64_t n, const int* __restrict__ d_eff_p,
                                              const TS* __restrict__ B, int64_t ldb, const double* __restrict__ y,
                                              double* __restrict__ x, const double* __restrict__ cn) {
    extern __shared__ double ys[];
    const int d_eff = *d_eff_p;
    for (int c = threadIdx.x; c < d_eff; c += kCombineBlock)
        ys[c] = cn ? (cn[c] > 0.0 ? y[c] / cn[c] : 0.0) : y[c];
    __syncthreads();
    if (d_eff <= 0) return;
    const int64_t nq = n / 4;
    const int64_t stride = static_cast<int64_t>(nblk) * kCombineBlock;
    for (int64_t t = static_cast<int64_t>(blk) * kCombineBlock + threadIdx.x; t < nq; t += stride) {
        const int64_t i0 = 4 * t;
        double acc[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
        int c = 0;
        for (; c + kCombineCols <= d_eff; c += kCombineCols) {
            double b[kCombineCols][4];
#pragma unroll
            for (int u = 0; u < kCombineCols; ++u) load_quad(B + static_cast<int64_t>(c + u) * ldb + i0, b[u]);
#pragma unroll
            for (int u = 0; u < kCombineCols; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r][u & 1] = __builtin_fma(b[u][r], ys[c + u], acc[r][u & 1]);
        }
        for (; c < d_eff; ++c) {
            double b[4];
            load_quad(B + static_cast<int64_t>(c) * ldb + i0, b);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r][c & 1] = __builtin_fma(b[r], ys[c], acc[r][c & 1]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) x[i0 + r] += acc[r][0] + acc[r][1];
    }
    if (blk == 0 && threadIdx.x < (n & 3)) {
        const int64_t i = 4 * nq + threadIdx.x;
        double a0 = 0.0, a1 = 0.0;
        for (int c = 0; c < d_eff; ++c) {
            const double b = from_basis<double>(B[static_cast<int64_t>(c) * ldb + i]);
            if (c & 1) a1 = madd(b, ys[c], a1);
            else a0 = madd(b, ys[c], a0);
        }
        x[i] += a0 + a1;
    }
}

template <typename TS>
__global__ __launch_bounds__(kCombineBlock) void combine4_kernel(int64_t n, const int* __restrict__ d_eff_p,
                                                                 const TS* __restrict__ B, int64_t ldb,
                                                                 const double* __restrict__ y,
                                                                 double* __restrict__ x,
                                                                 const double* __restrict__ cn) {
    combine4_body<TS>(blockIdx.x, gridDim.x, n, d_eff_p, B, ldb, y, x, cn);
}

// ---- the tails of several systems' cycles, one launch per kernel ----------
// Each job's blocks run as the single-system launch would with its own grid
// (combine4_grid / vec_grid of its n), so every system gets the bits of
// launch_combine, launch_residual and launch_norm_finish.

// the job whose blocks [first, first + count) hold block b (jobs in block order)
__device__ __forceinline__ int tail_job_of(const TailJob* __restrict__ jobs, int njobs, int b, bool combine) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if ((combine ? jobs[mid].cblk0 : jobs[mid].rblk0) <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename TS>
__global__ __launch_bounds__(kCombineBlock) void combine4_jobs_kernel(const TailJob* __restrict__ jobs, int njobs) {
    __shared__ int sj;
    if (threadIdx.x == 0) sj = tail_job_of(jobs, njobs, blockIdx.x, true);
    __syncthreads();
    const TailJob& J = jobs[sj];
    if (J.cnblk == 0) return;  // this system's combine is launched on its own
    combine4_body<TS>(blockIdx.x - J.cblk0, J.cnblk, J.n, J.d_eff, static_cast<const TS*>(J.B), J.ldb, J.y, J.x,
                      nullptr);
}

__global__ __launch_bounds__(kVecBlock) void residual_jobs_kernel(const TailJob* __restrict__ jobs, int njobs) {
    __shared__ int sj;
    if (threadIdx.x == 0) sj = tail_job_of(jobs, njobs, blockIdx.x, false);
    __syncthreads();
    const TailJob& J = jobs[sj];
    residual_body(blockIdx.x - J.rblk0, J.rnblk, J.n, J.rp, J.ci, J.val, J.f, J.x, J.r, J.part);
}

__global__ __launch_bounds__(kVecBlock) void norm_jobs_kernel(const TailJob* __restrict__ jobs) {
    const TailJob& J = jobs[blockIdx.x];
    norm_finish_body(J.part, J.rnblk, J.beta, J.nf);
}

// bad[0] = 1 if row_ptr is not a valid prefix array for nnz entries or a
// column index falls outside [0, n)
__global__ void csr_check_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rp,
                                 const int32_t* __restrict__ ci, int* __restrict__ bad) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    bool err = false;
    for (int64_t i = tid; i < n; i += stride) err |= rp[i] > rp[i + 1];
    if (tid == 0) err |= rp[0] != 0 || static_cast<int64_t>(rp[n]) != nnz;
    for (int64_t q = tid; q < nnz; q += stride) err |= ci[q] < 0 || static_cast<int64_t>(ci[q]) >= n;
    if (err) atomicOr(bad, 1);
}

// dval[q] = alpha * u[i] * v[col[q]] for every nonzero q of row i
__global__ void csr_outer_kernel(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                 const double* __restrict__ u, const double* __restrict__ v, double alpha,
                                 double* __restrict__ dval) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double ai = alpha * u[i];
        const int q1 = rp[i + 1];
        for (int q = rp[i]; q < q1; ++q) dval[q] = ai * v[ci[q]];
    }
}

}  // namespace

hipError_t launch_csr_outer(int64_t n, const int32_t* rp, const int32_t* ci, const double* u, const double* v,
                            double alpha, double* dval, hipStream_t stream) {
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    csr_outer_kernel<<<static_cast<int>(g), 256, 0, stream>>>(n, rp, ci, u, v, alpha, dval);
    return hipGetLastError();
}

hipError_t launch_csr_check(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, int* bad,
                            hipStream_t stream) {
    int64_t g = (n + nnz + 255) / 256;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    csr_check_kernel<<<static_cast<int>(g), 256, 0, stream>>>(n, nnz, rp, ci, bad);
    return hipGetLastError();
}

hipError_t launch_residual(int64_t n, const int32_t* rp, const int32_t* ci, const double* val,
                           const double* f, const double* x, double* r, double* part,
                           hipStream_t stream) {
    const int G = vec_grid(n);
    residual_kernel<<<G, kVecBlock, 0, stream>>>(n, rp, ci, val, f, x, r, part);
    return hipGetLastError();
}

hipError_t launch_norm_finish(const double* part, int G, double* out, const double* nf,
                              hipStream_t stream) {
    norm_finish_kernel<<<1, kVecBlock, 0, stream>>>(part, G, out, nf);
    return hipGetLastError();
}

int combine4_grid(int64_t n) {
    int64_t g4 = (n / 4 + kCombineBlock - 1) / kCombineBlock;
    if (g4 > 2048) g4 = 2048;
    if (g4 < 1) g4 = 1;
    return static_cast<int>(g4);
}

hipError_t launch_tail_jobs(const TailJob* jobs, int njobs, int cblocks, int rblocks, int d_max, int precision,
                            hipStream_t stream) {
    if (njobs <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * (d_max > 0 ? d_max : 1);
    if (cblocks > 0) {
        if (precision == SGMRES_PREC_FP32)
            combine4_jobs_kernel<float><<<cblocks, kCombineBlock, lds, stream>>>(jobs, njobs);
        else if (precision == SGMRES_PREC_BF16_BASIS)
            combine4_jobs_kernel<bf16_t><<<cblocks, kCombineBlock, lds, stream>>>(jobs, njobs);
        else
            combine4_jobs_kernel<double><<<cblocks, kCombineBlock, lds, stream>>>(jobs, njobs);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    residual_jobs_kernel<<<rblocks, kVecBlock, 0, stream>>>(jobs, njobs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    norm_jobs_kernel<<<njobs, kVecBlock, 0, stream>>>(jobs);
    return hipGetLastError();
}

hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    fill_kernel<<<static_cast<int>(g), 256, 0, stream>>>(x, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned* x, int64_t n, unsigned v, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    fill_u32_kernel<<<static_cast<int>(g), 256, 0, stream>>>(x, n, v);
    return hipGetLastError();
}

hipError_t launch_combine(int64_t n, const int* d_eff, int d_max, const void* B, int64_t ldb,
                          const double* y, double* x, hipStream_t stream, const double* colnorm, int precision) {
    int64_t g = (n + kCombineBlock - 1) / kCombineBlock;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    const size_t lds = sizeof(double) * (d_max > 0 ? d_max : 1);
    // four rows per thread where the columns allow aligned quad loads
    const size_t esz = precision == SGMRES_PREC_FP32 ? 4 : precision == SGMRES_PREC_BF16_BASIS ? 2 : 8;
    const size_t qa = esz == 8 ? 16 : 4 * esz;
    if (((reinterpret_cast<uintptr_t>(B) | static_cast<uintptr_t>(ldb) * esz) % qa) == 0 && n >= 4) {
        const int g4 = combine4_grid(n);
        if (precision == SGMRES_PREC_FP32)
            combine4_kernel<float><<<static_cast<int>(g4), kCombineBlock, lds, stream>>>(
                n, d_eff, static_cast<const float*>(B), ldb, y, x, colnorm);
        else if (precision == SGMRES_PREC_BF16_BASIS)
            combine4_kernel<bf16_t><<<static_cast<int>(g4), kCombineBlock, lds, stream>>>(
                n, d_eff, static_cast<const bf16_t*>(B), ldb, y, x, colnorm);
        else
            combine4_kernel<double><<<static_cast<int>(g4), kCombineBlock, lds, stream>>>(
                n, d_eff, static_cast<const double*>(B), ldb, y, x, colnorm);
        return hipGetLastError();
    }
    if (precision == SGMRES_PREC_FP32)
        combine_kernel<float><<<static_cast<int>(g), kCombineBlock, lds, stream>>>(
            n, d_eff, static_cast<const float*>(B), ldb, y, x, colnorm);
    else if (precision == SGMRES_PREC_BF16_BASIS)
        combine_kernel<bf16_t><<<static_cast<int>(g), kCombineBlock, lds, stream>>>(
            n, d_eff, static_cast<const bf16_t*>(B), ldb, y, x, colnorm);
    else
        combine_kernel<double><<<static_cast<int>(g), kCombineBlock, lds, stream>>>(
            n, d_eff, static_cast<const double*>(B), ldb, y, x, colnorm);
    return hipGetLastError();
}

// Nonzeros whose column lies outside their row's block of RB rows (summed
// into *out), and, when xbits is given, bit c of xbits set for every such
// column c (the rows that other blocks gather; OR is order-independent)
__global__ void offblock_kernel(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                int64_t RB, unsigned long long* __restrict__ out, unsigned* __restrict__ xbits) {
    __shared__ double tmp[kVecBlock / kWave];
    __shared__ double sum[1];
    double cnt = 0.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t b = i / RB;
        for (int q = rp[i]; q < rp[i + 1]; ++q) {
            const int c = ci[q];
            if (c / RB != b) {
                cnt += 1.0;
                if (xbits) atomicOr(xbits + (c >> 5), 1u << (c & 31));
            }
        }
    }
    const double v[1] = {cnt};
    block_sum<1>(v, 1, tmp, sum);
    if (threadIdx.x == 0) atomicAdd(out, static_cast<unsigned long long>(sum[0]));
}

hipError_t launch_offblock_count(int64_t n, const int32_t* rp, const int32_t* ci, int64_t RB,
                                 unsigned long long* out, unsigned* xbits, hipStream_t stream) {
    offblock_kernel<<<vec_grid(n), kVecBlock, 0, stream>>>(n, rp, ci, RB, out, xbits);
    return hipGetLastError();
}

__global__ void to_f32_kernel(int64_t count, const double* __restrict__ in, float* __restrict__ out) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride)
        out[i] = static_cast<float>(in[i]);
}

hipError_t launch_to_f32(int64_t count, const double* in, float* out, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    int64_t g = (count + 255) / 256;
    if (g > 4096) g = 4096;
    to_f32_kernel<<<static_cast<int>(g), 256, 0, stream>>>(count, in, out);
    return hipGetLastError();
}

}  // namespace sg
