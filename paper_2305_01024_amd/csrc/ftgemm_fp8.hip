// ftgemm_fp8.hip -- kernel entry points and variant table of the FP8 kernels
// (the tile computation is in ftgemm_fp8.hpp).
#include "ftgemm_fp8.hpp"

namespace ftgemm_impl {
namespace {

// The 128 x 128 tile (41 KB of LDS) fits several workgroups per compute
// unit; asking for two wavefronts per SIMD keeps its kernels at 256 VGPRs.
template <int BM, int BN>
constexpr int kMinWavesFP8 = (BM == 128 && BN == 128) ? 2 : 1;
template <int BM, int BN, int BK, int WM, int WN, int FT, bool INJ>
__global__ __launch_bounds__(64 * WM * WN, (kMinWavesFP8<BM, BN>)) void ftgemm_fp8_kernel(LaunchArgs a) {
    __shared__ fp8::SmemFP8<BM, BN, BK, WM, WN> sm;
    const int ntm = (a.M + BM - 1) / BM;
    fp8::tile<BM, BN, BK, WM, WN, FT, INJ>(a, blockIdx.x % ntm, blockIdx.x / ntm, sm);
}

// Recomputes the tiles a launch of the same variant queued (FT levels only).
template <int BM, int BN, int BK, int WM, int WN, int FT>
__global__ __launch_bounds__(64 * WM * WN) void ftgemm_fp8_retry_kernel(LaunchArgs a) {
    __shared__ fp8::SmemFP8<BM, BN, BK, WM, WN> sm;
    const int ntm = (a.M + BM - 1) / BM;
    abft::retry_queue(a, ntm, [&](int tm, int tn) { fp8::tile<BM, BN, BK, WM, WN, FT, false>(a, tm, tn, sm); });
}

template <int BM, int BN, int BK, int WM, int WN>
hipError_t launch_shape_fp8_retry(const LaunchArgs& a, int grid, hipStream_t s) {
    const dim3 g((unsigned)grid), block(64 * WM * WN);
    if (a.ft_level == 1) hipLaunchKernelGGL((ftgemm_fp8_retry_kernel<BM, BN, BK, WM, WN, 1>), g, block, 0, s, a);
    else hipLaunchKernelGGL((ftgemm_fp8_retry_kernel<BM, BN, BK, WM, WN, 2>), g, block, 0, s, a);
    return hipGetLastError();
}

template <int BM, int BN, int BK, int WM, int WN>
hipError_t launch_shape_fp8(bool inject, const LaunchArgs& a, hipStream_t s) {
    const int ntm = (a.M + BM - 1) / BM, ntn = (a.N + BN - 1) / BN;
    const dim3 grid((unsigned)(ntm * ntn)), block(64 * WM * WN);
#define FTGEMM_LAUNCH(FTL, INJL) \
    hipLaunchKernelGGL((ftgemm_fp8_kernel<BM, BN, BK, WM, WN, FTL, INJL>), grid, block, 0, s, a)
    if (inject) {
        if (a.ft_level == 0) FTGEMM_LAUNCH(0, true);
        else if (a.ft_level == 1) FTGEMM_LAUNCH(1, true);
        else FTGEMM_LAUNCH(2, true);
    } else {
        if (a.ft_level == 0) FTGEMM_LAUNCH(0, false);
        else if (a.ft_level == 1) FTGEMM_LAUNCH(1, false);
        else FTGEMM_LAUNCH(2, false);
    }
#undef FTGEMM_LAUNCH
    return hipGetLastError();
}

constexpr Variant kVariantsFP8[] = {
    {256, 256, 64, 256, 256},
    {128, 128, 64, 128, 128},
};
// default-selection cost model (aligned with kVariantsFP8; MI355X, 8192^3 rates in TFLOP/s)
constexpr VariantModel kModelsFP8[] = {
    {1, 8, 1410.0f, 512.0f},
    {2, 4, 919.0f, 336.0f},
};

}  // namespace

int fp8_variant_count() { return sizeof(kVariantsFP8) / sizeof(kVariantsFP8[0]); }
Variant fp8_variant(int idx) { return kVariantsFP8[idx]; }
VariantModel fp8_variant_model(int idx) { return kModelsFP8[idx]; }
int fp8_find_variant(int m_tile, int n_tile, int k_step, int check_m, int check_n) {
    for (int v = 0; v < fp8_variant_count(); ++v) {
        const Variant& x = kVariantsFP8[v];
        if (x.m_tile == m_tile && x.n_tile == n_tile && x.k_step == k_step && x.check_m == check_m &&
            x.check_n == check_n)
            return v;
    }
    return -1;
}

hipError_t launch_fp8(int idx, bool inject, const LaunchArgs& a, hipStream_t s) {
    switch (idx) {
        case 0: return launch_shape_fp8<256, 256, 64, 2, 4>(inject, a, s);
        case 1: return launch_shape_fp8<128, 128, 64, 2, 2>(inject, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fp8_retry(int idx, const LaunchArgs& a, int grid, hipStream_t s) {
    switch (idx) {
        case 0: return launch_shape_fp8_retry<256, 256, 64, 2, 4>(a, grid, s);
        case 1: return launch_shape_fp8_retry<128, 128, 64, 2, 2>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ftgemm_impl
