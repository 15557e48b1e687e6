// ftgemm_fp32.hip -- kernel entry points and variant table of the FP32 kernels
// (the tile computation is in ftgemm_fp32.hpp).
#include <algorithm>

#include "ftgemm_fp32.hpp"

namespace ftgemm_impl {
namespace {

// WAVE: wavefront-tile checks (FT levels only).  The 128 x 128 tile's LDS
// (79 KB) leaves room for two workgroups per compute unit; asking for two
// wavefronts per SIMD holds its FT kernels to 256 VGPRs, which they fit in
// without spilling in the main loop (the plain kernel is there already).
template <int BM, int BN, int FT>
constexpr int kMinWaves = (BM == 128 && BN == 128 && FT > 0) ? 2 : 1;
template <int BM, int BN, int BK, int WM, int WN, int FT, bool INJ, bool WAVE = false>
__global__ __launch_bounds__(64 * WM * WN, (kMinWaves<BM, BN, FT>)) void ftgemm_f32_kernel(LaunchArgs a) {
    __shared__ f32::Smem<BM, BN, BK, WM, WN, WAVE> sm;
    const int ntm = (a.M + BM - 1) / BM;
    f32::tile<BM, BN, BK, WM, WN, FT, INJ, WAVE>(a, blockIdx.x % ntm, blockIdx.x / ntm, sm);
}

// Recomputes the tiles a launch of the same variant queued (FT levels only).
template <int BM, int BN, int BK, int WM, int WN, int FT, bool WAVE = false>
__global__ __launch_bounds__(64 * WM * WN) void ftgemm_f32_retry_kernel(LaunchArgs a) {
    __shared__ f32::Smem<BM, BN, BK, WM, WN, WAVE> sm;
    const int ntm = (a.M + BM - 1) / BM;
    abft::retry_queue(a, ntm, [&](int tm, int tn) { f32::tile<BM, BN, BK, WM, WN, FT, false, WAVE>(a, tm, tn, sm); });
}

__global__ void zero_u32_kernel(uint32_t* p, int n) {
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) p[x] = 0u;
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
// compute-tile checks first (automatic selection walks them in order), then
// the wavefront-tile check (check tile = one wave's 64 x 64 sub-tile).  The
// 256 x 256 tile has no wavefront-check variant: its 8 wavefronts hold 128
// accumulators each at two wavefronts per SIMD, and the four reference
// checksums per row owner do not fit beside them without spilling.
constexpr Variant kVariants[] = {
    {256, 256, 32, 256, 256},
    {256, 128, 32, 256, 128},
    {128, 256, 32, 128, 256},
    {128, 128, 32, 128, 128},
    {64, 64, 32, 64, 64},
    {128, 128, 32, 64, 64},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
// aligned with kVariants (the wavefront-check variant is never auto-selected)
constexpr VariantModel kModels[] = {
    {1, 8, 137.4f, 123.3f}, {1, 4, 117.4f, 99.1f}, {1, 4, 118.4f, 95.8f}, {2, 4, 137.0f, 113.1f},
    {4, 1, 111.1f, 81.9f}, {2, 4, 137.0f, 96.2f},
};
static_assert(sizeof(kModels) / sizeof(kModels[0]) == kNumVariants, "one model entry per variant");

// Level 0 of a wavefront-check variant runs the plain kernel of its tile.
template <int BM, int BN, int BK, int WM, int WN, bool WAVE = false>
hipError_t launch_shape(bool inject, const LaunchArgs& a, hipStream_t s) {
    const int ntm = (a.M + BM - 1) / BM, ntn = (a.N + BN - 1) / BN;
    const dim3 grid((unsigned)(ntm * ntn)), block(64 * WM * WN);
#define FTGEMM_LAUNCH(FTL, INJL, WV) \
    hipLaunchKernelGGL((ftgemm_f32_kernel<BM, BN, BK, WM, WN, FTL, INJL, WV>), grid, block, 0, s, a)
    if (inject) {
        if (a.ft_level == 0) FTGEMM_LAUNCH(0, true, false);
        else if (a.ft_level == 1) FTGEMM_LAUNCH(1, true, WAVE);
        else FTGEMM_LAUNCH(2, true, WAVE);
    } else {
        if (a.ft_level == 0) FTGEMM_LAUNCH(0, false, false);
        else if (a.ft_level == 1) FTGEMM_LAUNCH(1, false, WAVE);
        else FTGEMM_LAUNCH(2, false, WAVE);
    }
#undef FTGEMM_LAUNCH
    return hipGetLastError();
}

template <int BM, int BN, int BK, int WM, int WN, bool WAVE = false>
hipError_t launch_shape_retry(const LaunchArgs& a, int grid, hipStream_t s) {
    const dim3 g((unsigned)grid), block(64 * WM * WN);
    if (a.ft_level == 1) hipLaunchKernelGGL((ftgemm_f32_retry_kernel<BM, BN, BK, WM, WN, 1, WAVE>), g, block, 0, s, a);
    else hipLaunchKernelGGL((ftgemm_f32_retry_kernel<BM, BN, BK, WM, WN, 2, WAVE>), g, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace

int fp32_variant_count() { return kNumVariants; }
VariantModel fp32_variant_model(int idx) { return kModels[idx]; }
Variant fp32_variant(int idx) { return kVariants[idx]; }
int fp32_find_variant(int m_tile, int n_tile, int k_step, int check_m, int check_n) {
    for (int v = 0; v < kNumVariants; ++v) {
        const Variant& x = kVariants[v];
        if (x.m_tile == m_tile && x.n_tile == n_tile && x.k_step == k_step && x.check_m == check_m &&
            x.check_n == check_n)
            return v;
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
        case 5: return launch_shape<128, 128, 32, 2, 2, true>(inject, a, s);
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
        case 5: return launch_shape_retry<128, 128, 32, 2, 2, true>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)std::max(1, std::min(64, (n + 255) / 256))), dim3(256), 0, s,
                       p, n);
    return hipGetLastError();
}

hipError_t launch_scale(float* C, int64_t ldc, int32_t M, int32_t N, float beta, hipStream_t s) {
    const int64_t total = (int64_t)M * N;
    const int blocks = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
    hipLaunchKernelGGL(scale_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, C, ldc, M, N, beta);
    return hipGetLastError();
}

}  // namespace ftgemm_impl
