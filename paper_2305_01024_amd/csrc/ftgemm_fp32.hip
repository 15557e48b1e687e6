// ftgemm_fp32.hip -- kernel entry points and variant table of the FP32 kernels
// (the tile computation is in ftgemm_fp32.hpp).
#include "ftgemm_fp32.hpp"

namespace ftgemm_impl {
namespace {

template <int BM, int BN, int BK, int WM, int WN, int FT, bool INJ>
__global__ __launch_bounds__(64 * WM * WN) void ftgemm_f32_kernel(LaunchArgs a) {
    __shared__ f32::Smem<BM, BN, BK, WM, WN> sm;
    const int ntm = (a.M + BM - 1) / BM;
    f32::tile<BM, BN, BK, WM, WN, FT, INJ>(a, blockIdx.x % ntm, blockIdx.x / ntm, sm);
}

// Recomputes the tiles a launch of the same variant queued (FT levels only).
template <int BM, int BN, int BK, int WM, int WN, int FT>
__global__ __launch_bounds__(64 * WM * WN) void ftgemm_f32_retry_kernel(LaunchArgs a) {
    __shared__ f32::Smem<BM, BN, BK, WM, WN> sm;
    const int ntm = (a.M + BM - 1) / BM;
    abft::retry_queue(a, ntm, [&](int tm, int tn) { f32::tile<BM, BN, BK, WM, WN, FT, false>(a, tm, tn, sm); });
}

__global__ void scale_kernel(float* C, int64_t ldc, int32_t M, int32_t N, float beta) {
    const int64_t total = (int64_t)M * N;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = x / M, i = x % M;
        float* p = C + j * ldc + i;
        *p = (beta == 0.0f) ? 0.0f : beta * *p;
    }
}

// ---------------------------------------------------------------------------
// variant table
// ---------------------------------------------------------------------------
struct VariantDef {
    Variant v;
    int wm, wn;
};
constexpr VariantDef kVariants[] = {
    {{256, 256, 32}, 2, 4},
    {{256, 128, 32}, 2, 2},
    {{128, 256, 32}, 1, 4},
    {{128, 128, 32}, 2, 2},
    {{64, 64, 32}, 1, 1},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <int BM, int BN, int BK, int WM, int WN>
hipError_t launch_shape(bool inject, const LaunchArgs& a, hipStream_t s) {
    const int ntm = (a.M + BM - 1) / BM, ntn = (a.N + BN - 1) / BN;
    const dim3 grid((unsigned)(ntm * ntn)), block(64 * WM * WN);
#define FTGEMM_LAUNCH(FTL, INJL) \
    hipLaunchKernelGGL((ftgemm_f32_kernel<BM, BN, BK, WM, WN, FTL, INJL>), grid, block, 0, s, a)
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

template <int BM, int BN, int BK, int WM, int WN>
hipError_t launch_shape_retry(const LaunchArgs& a, int grid, hipStream_t s) {
    const dim3 g((unsigned)grid), block(64 * WM * WN);
    if (a.ft_level == 1) hipLaunchKernelGGL((ftgemm_f32_retry_kernel<BM, BN, BK, WM, WN, 1>), g, block, 0, s, a);
    else hipLaunchKernelGGL((ftgemm_f32_retry_kernel<BM, BN, BK, WM, WN, 2>), g, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace

int fp32_variant_count() { return kNumVariants; }
Variant fp32_variant(int idx) { return kVariants[idx].v; }
int fp32_find_variant(int m_tile, int n_tile, int k_step) {
    for (int v = 0; v < kNumVariants; ++v) {
        const Variant& x = kVariants[v].v;
        if (x.m_tile == m_tile && x.n_tile == n_tile && x.k_step == k_step) return v;
    }
    return -1;
}

hipError_t launch_fp32(int idx, bool inject, const LaunchArgs& a, hipStream_t s) {
    switch (idx) {
        case 0: return launch_shape<256, 256, 32, 2, 4>(inject, a, s);
        case 1: return launch_shape<256, 128, 32, 2, 2>(inject, a, s);
        case 2: return launch_shape<128, 256, 32, 1, 4>(inject, a, s);
        case 3: return launch_shape<128, 128, 32, 2, 2>(inject, a, s);
        case 4: return launch_shape<64, 64, 32, 1, 1>(inject, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fp32_retry(int idx, const LaunchArgs& a, int grid, hipStream_t s) {
    switch (idx) {
        case 0: return launch_shape_retry<256, 256, 32, 2, 4>(a, grid, s);
        case 1: return launch_shape_retry<256, 128, 32, 2, 2>(a, grid, s);
        case 2: return launch_shape_retry<128, 256, 32, 1, 4>(a, grid, s);
        case 3: return launch_shape_retry<128, 128, 32, 2, 2>(a, grid, s);
        case 4: return launch_shape_retry<64, 64, 32, 1, 1>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_scale(float* C, int64_t ldc, int32_t M, int32_t N, float beta, hipStream_t s) {
    const int64_t total = (int64_t)M * N;
    const int blocks = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
    hipLaunchKernelGGL(scale_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, C, ldc, M, N, beta);
    return hipGetLastError();
}

}  // namespace ftgemm_impl
