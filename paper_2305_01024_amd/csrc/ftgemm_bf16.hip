// ftgemm_bf16.hip -- kernel entry points and variant table of the BF16 kernels
// (the tile computation is in ftgemm_bf16.hpp).
#include "ftgemm_bf16.hpp"

namespace ftgemm_impl {
namespace {

// The 128 x 128 tile (79 KB of LDS) fits two workgroups per compute unit;
// asking for two wavefronts per SIMD holds its FT kernels to 256 VGPRs
// (unbounded they take 284, one wavefront per SIMD).
template <int BM, int BN, int FT>
constexpr int kMinWavesBF16 = (BM == 128 && BN == 128 && FT > 0) ? 2 : 1;
template <int BM, int BN, int BK, int WM, int WN, int FT, bool INJ>
__global__ __launch_bounds__(64 * WM * WN, (kMinWavesBF16<BM, BN, FT>)) void ftgemm_bf16_kernel(LaunchArgs a) {
    __shared__ bf16::SmemBF16<BM, BN, BK, WM, WN> sm;
    const int ntm = (a.M + BM - 1) / BM;
    bf16::tile<BM, BN, BK, WM, WN, FT, INJ>(a, blockIdx.x % ntm, blockIdx.x / ntm, sm);
}

// Recomputes the tiles a launch of the same variant queued (FT levels only).
template <int BM, int BN, int BK, int WM, int WN, int FT>
__global__ __launch_bounds__(64 * WM * WN) void ftgemm_bf16_retry_kernel(LaunchArgs a) {
    __shared__ bf16::SmemBF16<BM, BN, BK, WM, WN> sm;
    const int ntm = (a.M + BM - 1) / BM;
    abft::retry_queue(a, ntm, [&](int tm, int tn) { bf16::tile<BM, BN, BK, WM, WN, FT, false>(a, tm, tn, sm); });
}

template <int BM, int BN, int BK, int WM, int WN>
hipError_t launch_shape_bf16_retry(const LaunchArgs& a, int grid, hipStream_t s) {
    const dim3 g((unsigned)grid), block(64 * WM * WN);
    if (a.ft_level == 1) hipLaunchKernelGGL((ftgemm_bf16_retry_kernel<BM, BN, BK, WM, WN, 1>), g, block, 0, s, a);
    else hipLaunchKernelGGL((ftgemm_bf16_retry_kernel<BM, BN, BK, WM, WN, 2>), g, block, 0, s, a);
    return hipGetLastError();
}

template <int BM, int BN, int BK, int WM, int WN>
hipError_t launch_shape_bf16(bool inject, const LaunchArgs& a, hipStream_t s) {
    const int ntm = (a.M + BM - 1) / BM, ntn = (a.N + BN - 1) / BN;
    const dim3 grid((unsigned)(ntm * ntn)), block(64 * WM * WN);
#define FTGEMM_LAUNCH(FTL, INJL) \
    hipLaunchKernelGGL((ftgemm_bf16_kernel<BM, BN, BK, WM, WN, FTL, INJL>), grid, block, 0, s, a)
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

constexpr Variant kVariantsBF16[] = {
    {256, 256, 64, 256, 256},
    {128, 128, 64, 128, 128},
};
// default-selection cost model (aligned with kVariantsBF16; MI355X, 8192^3)
constexpr VariantModel kModelsBF16[] = {
    {1, 8, 994.0f, 505.0f},
    {2, 4, 786.0f, 337.0f},
};

}  // namespace

int bf16_variant_count() { return sizeof(kVariantsBF16) / sizeof(kVariantsBF16[0]); }
Variant bf16_variant(int idx) { return kVariantsBF16[idx]; }
VariantModel bf16_variant_model(int idx) { return kModelsBF16[idx]; }
int bf16_find_variant(int m_tile, int n_tile, int k_step, int check_m, int check_n) {
    for (int v = 0; v < bf16_variant_count(); ++v) {
        const Variant& x = kVariantsBF16[v];
        if (x.m_tile == m_tile && x.n_tile == n_tile && x.k_step == k_step && x.check_m == check_m &&
            x.check_n == check_n)
            return v;
    }
    return -1;
}

hipError_t launch_bf16(int idx, bool inject, const LaunchArgs& a, hipStream_t s) {
    switch (idx) {
        case 0: return launch_shape_bf16<256, 256, 64, 2, 4>(inject, a, s);
        case 1: return launch_shape_bf16<128, 128, 64, 2, 2>(inject, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bf16_retry(int idx, const LaunchArgs& a, int grid, hipStream_t s) {
    switch (idx) {
        case 0: return launch_shape_bf16_retry<256, 256, 64, 2, 4>(a, grid, s);
        case 1: return launch_shape_bf16_retry<128, 128, 64, 2, 2>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ftgemm_impl
