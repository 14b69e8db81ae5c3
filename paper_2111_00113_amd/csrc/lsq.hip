// sketched_lsq: the small sketched least-squares problem of sGMRES
// (arXiv:2111.00113, Algorithm 1 solve step; Section 3.3):
//   unpivoted Householder QR  S A B = Q T  (reflectors applied to g = S r too),
//   condition guard on the diagonal of T (Sections 3.4 and 5.3),
//   back substitution T y = Q^T g on the kept prefix,
//   residual estimate |(Q^T g)[d_eff:]|.
// One workgroup of 1024 threads; the s x dc matrix stays in global memory
// (L2-resident), the current reflector is staged in LDS.
#include "common.hpp"
#include "internal.hpp"

namespace sg {

namespace {

constexpr int kLsqBlock = 1024;
constexpr int kLsqWaves = kLsqBlock / kWave;
constexpr int kZSlots = kLsqMaxCols / kWave;

__global__ __launch_bounds__(kLsqBlock) void lsq_kernel(int s, const int* __restrict__ dc_dev, int dc_host,
                                                        double* __restrict__ C, double* __restrict__ g,
                                                        double kappa_max, double* __restrict__ y,
                                                        double* __restrict__ dout, int* __restrict__ iout) {
    extern __shared__ double v[];  // s doubles: tail of the current reflector
    __shared__ double tmp[kLsqWaves];
    __shared__ double red[1];
    __shared__ double bc[3];
    __shared__ int ibc[1];
    const int dc = dc_dev ? *dc_dev : dc_host;
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
            const double zi = __shfl(mine, i & (kWave - 1), kWave);
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

}  // namespace

hipError_t launch_lsq(int s, const int* dc_dev, int dc_host, double* C, double* g, double kappa_max,
                      double* y, double* dout, int* iout, hipStream_t stream) {
    lsq_kernel<<<1, kLsqBlock, sizeof(double) * s, stream>>>(s, dc_dev, dc_host, C, g, kappa_max, y, dout, iout);
    return hipGetLastError();
}

}  // namespace sg
