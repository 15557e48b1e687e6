// ftgemm_batched.hip -- many independent FT-GEMMs in one persistent launch.
//
// A grid of resident 256-thread workgroups walks a list of (problem, tile)
// work items, ordered by decreasing cost on the host so that the static
// round-robin assignment (item = workgroup + grid * i) stays balanced.  Each
// item runs the same tile computation as the single-problem kernels (the
// threadblock-level online ABFT of section 4.2.3, with its own encode,
// checksum update, checks and correction), on the item's problem: one tile
// shape per problem, picked on the host.  The LDS of the tile variants is
// one union.  A plan with FP8 problems launches the instantiation that also
// holds the FP8 tile (F8); the others leave it out and keep the register
// allocation of the FP32 and BF16 paths as it is without it.
#include "ftgemm_bf16.hpp"
#include "ftgemm_fp32.hpp"
#include "ftgemm_fp8.hpp"

namespace ftgemm_impl {
namespace {

constexpr int kBatchThreads = 256;

struct NoLds {};
template <bool F8>
union BatchSmem {
    f32::Smem<128, 128, 32, 2, 2> f32_128;
    f32::Smem<64, 64, 64, 2, 2> f32_64;
    bf16::SmemBF16<128, 128, 64, 2, 2> bf16_128;
    std::conditional_t<F8, fp8::SmemFP8<128, 128, 64, 2, 2>, NoLds> fp8_128;
};

constexpr Variant kBatchVariantTable[kBatchVariants] = {
    {128, 128, 32, 128, 128}, {64, 64, 64, 64, 64}, {128, 128, 64, 128, 128}, {128, 128, 64, 128, 128}};
constexpr int kBatchVariantDtype[kBatchVariants] = {FTGEMM_F32, FTGEMM_F32, FTGEMM_BF16, FTGEMM_F8E4M3};

// C = beta * C on one 128 x 128 tile (problems with k == 0 or alpha == 0)
__device__ void scale_tile(const BatchProblem& p, int tm, int tn) {
    for (int x = threadIdx.x; x < 128 * 128; x += kBatchThreads) {
        const int i = tm * 128 + (x & 127), j = tn * 128 + (x >> 7);
        if (i < p.M && j < p.N) {
            float* c = p.C + (size_t)j * p.ldc + i;
            *c = (p.beta == 0.0f) ? 0.0f : p.beta * *c;
        }
    }
}

template <int FT, bool INJ, bool F8>
__global__ __launch_bounds__(kBatchThreads, 2) void ftgemm_batched_kernel(BatchArgs b) {
    __shared__ BatchSmem<F8> sm;
    for (int it = blockIdx.x; it < b.n_items; it += gridDim.x) {
        const BatchItem item = b.items[it];
        const BatchProblem& p = b.probs[item.problem];
        const int tm = item.tile % p.ntm, tn = item.tile / p.ntm;
        if (p.variant < 0) {
            scale_tile(p, tm, tn);
            continue;
        }
        LaunchArgs a;
        a.A = static_cast<const float*>(p.A);
        a.B = static_cast<const float*>(p.B);
        a.C = p.C;
        a.lda = p.lda;
        a.ldb = p.ldb;
        a.ldc = p.ldc;
        a.M = p.M;
        a.N = p.N;
        a.K = p.K;
        a.alpha = p.alpha;
        a.beta = p.beta;
        a.scale = p.scale;
        a.tol_c = b.tol_c;
        a.check_interval = b.ft_level == 1 ? 0x7fffffff : p.check_interval;   // detect-only: after the last step
        a.ft_level = b.ft_level;
        a.problem = item.problem;
        a.events = b.events;
        a.counters = b.counters;
        a.event_cap = b.event_cap;
        a.faults = b.faults;
        a.n_faults = b.n_faults;
        a.fault_log = b.fault_log;
        a.fault_log_cap = b.fault_log_cap;
        a.retry = nullptr;   // no recompute in the batched launch
        a.retry_tiles = nullptr;
        a.retry_pass = 0;
        switch (p.variant) {
            case 0: f32::tile<128, 128, 32, 2, 2, FT, INJ>(a, tm, tn, sm.f32_128); break;
            case 1: f32::tile<64, 64, 64, 2, 2, FT, INJ>(a, tm, tn, sm.f32_64); break;
            default:
                if constexpr (F8) {
                    if (p.variant == 3) {
                        fp8::tile<128, 128, 64, 2, 2, FT, INJ>(a, tm, tn, sm.fp8_128);
                        break;
                    }
                }
                bf16::tile<128, 128, 64, 2, 2, FT, INJ>(a, tm, tn, sm.bf16_128);
                break;
        }
        __syncthreads();   // the next item reuses the LDS
    }
}

template <int FT, bool INJ>
hipError_t launch_level(const BatchArgs& b, int grid, bool fp8, hipStream_t s) {
    if (fp8) hipLaunchKernelGGL((ftgemm_batched_kernel<FT, INJ, true>), dim3((unsigned)grid), dim3(kBatchThreads), 0, s, b);
    else hipLaunchKernelGGL((ftgemm_batched_kernel<FT, INJ, false>), dim3((unsigned)grid), dim3(kBatchThreads), 0, s, b);
    return hipGetLastError();
}

}  // namespace

Variant batch_variant(int v) { return kBatchVariantTable[v]; }
int batch_variant_dtype(int v) { return kBatchVariantDtype[v]; }

int batch_resident_blocks(int device, bool fp8) {
    int per_cu = 0, cus = 0;
    const hipError_t e = fp8 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ftgemm_batched_kernel<2, false, true>,
                                                                             kBatchThreads, 0)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ftgemm_batched_kernel<2, false, false>,
                                                                             kBatchThreads, 0);
    if (e != hipSuccess) per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) cus = 256;
    return std::max(1, per_cu) * std::max(1, cus);
}

hipError_t launch_batched(const BatchArgs& b, bool inject, int grid, bool fp8, hipStream_t s) {
    if (b.n_items <= 0) return hipSuccess;
    if (inject) {
        if (b.ft_level == 0) return launch_level<0, true>(b, grid, fp8, s);
        if (b.ft_level == 1) return launch_level<1, true>(b, grid, fp8, s);
        return launch_level<2, true>(b, grid, fp8, s);
    }
    if (b.ft_level == 0) return launch_level<0, false>(b, grid, fp8, s);
    if (b.ft_level == 1) return launch_level<1, false>(b, grid, fp8, s);
    return launch_level<2, false>(b, grid, fp8, s);
}

}  // namespace ftgemm_impl
