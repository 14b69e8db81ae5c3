// Streaming truncated-Arnoldi basis kernel: instances, launch shape and launch
// (kernel in stream_kernel.hpp).
#include "stream_kernel.hpp"

namespace sg {

using namespace stream_detail;

namespace {

template <typename TC>
int ring_of(int P, bool hst) {
    if (hst) return 0;
    switch (P) {
        case 4: return ring_slots<TC, 4, false>();
        case 8: return ring_slots<TC, 8, false>();
        case 16: return ring_slots<TC, 16, false>();
        default: return 0;
    }
}

template <typename TC, typename TS, int NR>
const void* pick_stream(int P, bool hst) {
    if (hst) return reinterpret_cast<const void*>(stream_kernel<TC, TS, NR, 4, true>);
    switch (P) {
        case 4: return reinterpret_cast<const void*>(stream_kernel<TC, TS, NR, 4, false>);
        case 8: return reinterpret_cast<const void*>(stream_kernel<TC, TS, NR, 8, false>);
        case 16: return reinterpret_cast<const void*>(stream_kernel<TC, TS, NR, 16, false>);
        default: return nullptr;
    }
}

template <int NR>
const void* pick_prec(int precision, int P, bool hst) {
    if (precision == SGMRES_PREC_FP64) return pick_stream<double, double, NR>(P, hst);
    if (precision == SGMRES_PREC_FP32) return pick_stream<float, float, NR>(P, hst);
    if (precision == SGMRES_PREC_BF16_BASIS) return pick_stream<float, bf16_t, NR>(P, hst);
    return nullptr;
}

const void* pick(int nr, int precision, int P, bool hst) {
    switch (nr) {
        case 1: return pick_prec<1>(precision, P, hst);
        case 32: return pick_prec<32>(precision, P, hst);
        default: return nullptr;
    }
}

}  // namespace

hipError_t stream_configure(int64_t n, int nr, int k, int precision, StreamLaunch* out) {
    if (n < 1 || k < 1 || k > kStreamMaxK) return hipErrorInvalidValue;
    int device = 0;
    hipError_t err = hipGetDevice(&device);
    if (err != hipSuccess) return err;
    int cus = 0, lds_max = 0;
    err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (err != hipSuccess) return err;
    err = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (err != hipSuccess) return err;
    const size_t tc_bytes = precision == SGMRES_PREC_FP64 ? 8 : 4;
    const int64_t npairs = n * nr;
    // register state with the fewest pairs per thread whose grid fits the
    // chip, else the state buffer with four pairs per thread and tile
    const int Ps[3] = {4, 8, 16};
    for (int hi = 0; hi < 2; ++hi) {
        const bool hst = hi == 1;
        for (int pi = 0; pi < (hst ? 1 : 3); ++pi) {
            const int P = hst ? 4 : Ps[pi];
            const void* fn = pick(nr, precision, P, hst);
            if (!fn) continue;
            // register state: the instance's LDS ring of the newest window
            // columns (fixed per instance), next to its static LDS
            hipFuncAttributes fa{};
            err = hipFuncGetAttributes(&fa, fn);
            if (err != hipSuccess) continue;
            const size_t slot = static_cast<size_t>(P) * kStreamBlock * tc_bytes;
            const int nl = precision == SGMRES_PREC_FP64 ? ring_of<double>(P, hst) : ring_of<float>(P, hst);
            const size_t lds = static_cast<size_t>(nl) * slot;
            if (lds + fa.sharedSizeBytes > static_cast<size_t>(lds_max)) continue;
            err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
            if (err != hipSuccess) continue;
            int per_cu = 0;
            err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kStreamBlock, lds);
            if (err != hipSuccess || per_cu < 1) continue;
            const int64_t gmax = static_cast<int64_t>(per_cu) * cus;
            const int64_t tiles = (npairs + static_cast<int64_t>(P) * kStreamBlock - 1) /
                                  (static_cast<int64_t>(P) * kStreamBlock);
            if (!hst && tiles > gmax) continue;
            out->fn = fn;
            out->NR = nr;
            out->P = P;
            out->hst = hst ? 1 : 0;
            out->grid = static_cast<int>(hst ? (tiles < gmax ? tiles : gmax) : tiles);
            out->nl = nl;
            out->lds = lds;
            return hipSuccess;
        }
    }
    return hipErrorInvalidValue;
}

hipError_t stream_launch(const StreamLaunch& L, StreamParams params, hipStream_t stream) {
    void* args[] = {&params};
    params.nl = L.nl;
    return hipLaunchCooperativeKernel(L.fn, dim3(L.grid), dim3(kStreamBlock), args, static_cast<unsigned>(L.lds),
                                      stream);
}

}  // namespace sg
