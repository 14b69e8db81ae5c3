// spmv_truncarnoldi launch plumbing and the instances that form S m_j only
// (the solve path); the instances that also form S b_j are in arnoldi_sb.hip.
#include "arnoldi_kernel.hpp"

namespace sg {

using namespace arnoldi_detail;

namespace {

using KernelFn = void (*)(ArnoldiParams);

// FP64 solve instances live here; the others in their own translation units
KernelFn pick_kernel(int block, int R, int KW, bool sketch_basis, int precision, bool halo) {
    const void* f = nullptr;
    if (halo) {
        if (sketch_basis) return nullptr;
        if (precision == SGMRES_PREC_FP64) f = arnoldi_pick_halo_f64(block, R, KW);
        else if (precision == SGMRES_PREC_FP32) f = arnoldi_pick_halo_f32(block, R, KW);
        else if (precision == SGMRES_PREC_BF16_BASIS) f = arnoldi_pick_halo_bf16(block, R, KW);
        return reinterpret_cast<KernelFn>(const_cast<void*>(f));
    }
    if (precision == SGMRES_PREC_FP32) f = sketch_basis ? nullptr : arnoldi_pick_f32(block, R, KW);
    else if (precision == SGMRES_PREC_BF16_BASIS) f = sketch_basis ? nullptr : arnoldi_pick_bf16(block, R, KW);
    else if (precision == SGMRES_PREC_FP64)
        f = sketch_basis ? arnoldi_pick_sb(block, R, KW) : arnoldi_pick<false, double, double>(block, R, KW);
    return reinterpret_cast<KernelFn>(const_cast<void*>(f));
}

}  // namespace

size_t arnoldi_lds_bytes(int block, int R, int s, int k, int zeta) {
    const int nw = block / kWave;
    const int RB = R * block;
    return sizeof(double) * static_cast<size_t>(arnoldi_vals_doubles(RB, zeta) + nw * kRedSlots + kRedSlots + 2 * k + 3) +
           sizeof(int) * static_cast<size_t>(2 * s + 2) +
           sizeof(uint16_t) * static_cast<size_t>(sketch_lists_len(zeta * RB, s, true));
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

    const int blocks_try[3] = {1024, 512, 256};
    const int rows_try[4] = {1, 2, 4, 8};
    // candidates in order of preference; the first whose grid fits the chip wins
    {
        for (int bi = 0; bi < 3; ++bi) {
            const int block = blocks_try[bi];
            if (shape.block && block != shape.block) continue;
            for (int ri = 0; ri < 4; ++ri) {
                const int R = rows_try[ri];
                if (shape.rows_per_thread && R != shape.rows_per_thread) continue;
                int KW = 0;
                if (kw_need <= 4) KW = 4;
                else if (kw_need <= 8) KW = 8;
                if (KW * R > 32) KW = 0;  // keep the register window within 64 VGPRs
                if (shape.force_global_window) KW = 0;
                const size_t lds = arnoldi_lds_bytes(block, R, shape.s, shape.k, shape.zeta);
                if (lds > static_cast<size_t>(lds_max)) continue;
                KernelFn fn = pick_kernel(block, R, KW, shape.sketch_basis != 0, shape.precision, shape.halo != 0);
                if (!fn) continue;
                err = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
                if (err != hipSuccess) continue;
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
    }
    return hipErrorInvalidValue;
}

size_t sync_words_bytes() { return sizeof(SyncWords); }

hipError_t arnoldi_launch(const ArnoldiLaunch& L, ArnoldiParams params, hipStream_t stream) {
    void* args[] = {&params};
    return hipLaunchCooperativeKernel(L.fn, dim3(L.grid), dim3(L.block), args,
                                      static_cast<unsigned>(L.lds), stream);
}

}  // namespace sg
