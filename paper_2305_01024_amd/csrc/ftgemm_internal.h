// ftgemm_internal.h -- launch interface between the C ABI (ftgemm_api.cpp)
// and the gfx950 kernels (ftgemm_fp32.hip, ftgemm_bf16.hip, ftgemm_fp8.hip).
// Not installed, not part of the ABI.
#pragma once

#include <stdint.h>
#include <hip/hip_runtime.h>
#include "ftgemm.h"

namespace ftgemm_impl {

// Device-side counters, one block per handle (index into `counters`).
enum Counter : int {
    CNT_EVENTS = 0,        // events appended (may exceed capacity)
    CNT_DETECTED = 1,
    CNT_CORRECTED = 2,
    CNT_UNCORRECTABLE = 3,
    CNT_CHECKSUM_ONLY = 4,
    CNT_FAULTS = 5,        // faults applied by the injection hook
    CNT_RECOMPUTED = 6,    // tiles recomputed by the retry launch
    CNT_RECOMPUTE_FAILED = 7,  // retried tiles whose own checks still flagged a fault
    CNT_CHECKS = 8,        // checks performed (one per check tile and check step)
    CNT_NONFINITE = 9,     // check tiles reported once for non-finite operands
    CNT_N = 10
};

// Maximum fault sites one tile may hold in the injection build.
constexpr int kMaxFaultsPerTile = 32;

struct LaunchArgs {
    const float* A;
    const float* B;
    float* C;
    int64_t lda, ldb, ldc;
    int32_t M, N, K;
    float alpha, beta;
    float scale;                 // per-tensor dequantisation scale_a * scale_b (1 for FP32)
    float tol_c;                 // threshold factor c
    int32_t check_interval;      // g, in k-steps
    int32_t ft_level;            // 0, 1, 2
    int32_t problem;             // problem index reported in events
    ftgemm_event_t* events;      // device event log
    uint32_t* counters;          // device counters[CNT_N]
    int32_t event_cap;
    const ftgemm_fault_t* faults;    // device fault sites (injection build) or nullptr
    int32_t n_faults;
    ftgemm_fault_log_t* fault_log;   // device applied-fault log
    int32_t fault_log_cap;
    // Recompute of tainted tiles (nullptr / 0: off).  Main launch: a tainted
    // tile appends tm + ntm * tn to retry_tiles (retry[0] counts) instead of
    // writing C.  Retry launch (retry_pass = 1): recomputes the queued tiles;
    // its last workgroup clears retry[0..1].
    uint32_t* retry;             // [0] queued tiles, [1] retry workgroups finished
    int32_t* retry_tiles;        // capacity >= number of tiles of the launch
    int32_t retry_pass;
};

// A compiled kernel variant: compute tile, k-step and check tile (the
// compute tile itself, or the sub-tile of one wavefront).
struct Variant {
    int m_tile, n_tile, k_step, check_m, check_n;
};

// Kernel variants compiled for FP32 operands, in preference order.
int fp32_variant_count();
Variant fp32_variant(int idx);
// Default-selection cost model of an FP32 variant: workgroups resident per
// compute unit, wavefronts per workgroup, and the throughput (TFLOP/s) of its
// plain and online FT kernels with every compute unit full (measured on
// MI355X at 8192^3).
struct VariantModel {
    int wg_per_cu, waves_per_wg;
    float tflops_plain, tflops_ft;
};
VariantModel fp32_variant_model(int idx);
int fp32_find_variant(int m_tile, int n_tile, int k_step, int check_m, int check_n);

// Launch the FP32 kernel variant `idx` (A, B as float).  `inject` selects the instantiation
// carrying the fault-injection hook.  Returns a hipError_t.
hipError_t launch_fp32(int idx, bool inject, const LaunchArgs& a, hipStream_t stream);
// Retry launch of variant `idx` over the tiles queued in a.retry_tiles, `grid` workgroups.
hipError_t launch_fp32_retry(int idx, const LaunchArgs& a, int grid, hipStream_t stream);

// Kernel variants for BF16 operands (A, B as bfloat16 codes).
int bf16_variant_count();
Variant bf16_variant(int idx);
VariantModel bf16_variant_model(int idx);
int bf16_find_variant(int m_tile, int n_tile, int k_step, int check_m, int check_n);
hipError_t launch_bf16(int idx, bool inject, const LaunchArgs& a, hipStream_t stream);
hipError_t launch_bf16_retry(int idx, const LaunchArgs& a, int grid, hipStream_t stream);

// Kernel variants for FP8 E4M3 operands (A, B as 8-bit codes).
int fp8_variant_count();
Variant fp8_variant(int idx);
VariantModel fp8_variant_model(int idx);
int fp8_find_variant(int m_tile, int n_tile, int k_step, int check_m, int check_n);
hipError_t launch_fp8(int idx, bool inject, const LaunchArgs& a, hipStream_t stream);
hipError_t launch_fp8_retry(int idx, const LaunchArgs& a, int grid, hipStream_t stream);

// ---- FP64 (A, B, C as double) ----
struct F64Args {
    const double* A;
    const double* B;
    double* C;
    int64_t lda, ldb, ldc;
    int32_t M, N, K;
    double alpha, beta;
    float tol_c;                 // threshold factor c
    int32_t check_interval;      // g, in k-steps
    int32_t ft_level;            // 0, 1, 2
    int32_t problem;             // problem index reported in events (0)
    ftgemm_event_t* events;
    uint32_t* counters;
    int32_t event_cap;
    const ftgemm_fault_t* faults;
    int32_t n_faults;
    ftgemm_fault_log_t* fault_log;
    int32_t fault_log_cap;
};
int fp64_variant_count();
Variant fp64_variant(int idx);
int fp64_find_variant(int m_tile, int n_tile, int k_step, int check_m, int check_n);
hipError_t launch_fp64(int idx, bool inject, const F64Args& a, hipStream_t stream);
hipError_t launch_scale64(double* C, int64_t ldc, int32_t M, int32_t N, double beta, hipStream_t stream);

// ---- double complex through two binary64 products (ftgemm_complex.hip) ----
// A (m x k complex) -> A' = (Re A, -Im A) and A'' = (Im A, Re A) interleaved
// along k (m x 2k real, leading dimension m)
hipError_t launch_zrepack(const double* A, int64_t lda, int32_t M, int32_t K, double* Ap, double* App,
                          hipStream_t stream);
// C = alpha (Pr + i Pi) + beta C, alpha / beta host (re, im) pairs
hipError_t launch_zepilogue(double* C, int64_t ldc, int32_t M, int32_t N, const double* Pr, const double* Pi,
                            const double* alpha, const double* beta, hipStream_t stream);
hipError_t launch_zscale(double* C, int64_t ldc, int32_t M, int32_t N, const double* beta, hipStream_t stream);

// ---- batched persistent launch ----
// Device descriptor of one problem of a batched call.
struct BatchProblem {
    const void* A;
    const void* B;
    float* C;
    int64_t lda, ldb, ldc;
    int32_t M, N, K;
    int32_t variant;             // batched tile variant, or -1: C = beta * C only (k == 0 or alpha == 0)
    float alpha, beta, scale;
    int32_t check_interval;      // in k-steps of the variant
    int32_t ntm;                 // tiles along m
    int32_t pad_;
};

// One work item: tile `tile` (tm + ntm * tn) of problem `problem`.
struct BatchItem {
    int32_t problem, tile;
};

struct BatchArgs {
    const BatchProblem* probs;
    const BatchItem* items;
    int32_t n_items;
    int32_t ft_level;
    float tol_c;
    int32_t event_cap;
    ftgemm_event_t* events;
    uint32_t* counters;
    const ftgemm_fault_t* faults;    // injection build only
    int32_t n_faults;
    int32_t fault_log_cap;
    ftgemm_fault_log_t* fault_log;
};

// Tile variants of the batched kernel (one 256-thread workgroup per tile):
// 0 = FP32 128 x 128 x 32, 1 = FP32 64 x 64 x 64, 2 = BF16 128 x 128 x 64,
// 3 = FP8 128 x 128 x 64 (only in the instantiation launched for plans with
// FP8 problems).
constexpr int kBatchVariants = 4;
Variant batch_variant(int v);
int batch_variant_dtype(int v);
// Workgroups of the batched kernel that are resident on the device at once.
int batch_resident_blocks(int device, bool fp8);
hipError_t launch_batched(const BatchArgs& b, bool inject, int grid, bool fp8, hipStream_t stream);

// ---- non-fused ABFT (the same checks around the plain kernel, one launch per step) ----
constexpr int kNonFusedTile = 256;   // check tile, rows and columns
struct NonFusedArgs {
    const float* A;
    const float* B;
    float* C;
    int64_t lda, ldb, ldc;
    int32_t M, N, K;
    float tol_c;
    float* W;      // [ntm][K]  e^T A per row tile
    float* V;      // [ntn][K]  B e per column tile
    float* R;      // [ntn][M]  row references
    float* S;      // [ntm][N]  column references
    float* na2;    // [M]       prefix ||a_i||^2
    float* nb2;    // [N]       prefix ||b_j||^2
    unsigned* tile_flag;   // [ntm * ntn] tile reported for non-finite operands
    ftgemm_event_t* events;
    int32_t event_cap;
    uint32_t* counters;
    const ftgemm_fault_t* faults;    // kstep = chunk index; applied to C after that chunk's GEMM
    int32_t n_faults;
    ftgemm_fault_log_t* fault_log;
    int32_t fault_log_cap;
};
hipError_t launch_nonfused_encode(const NonFusedArgs& n, hipStream_t stream);
// reference update, fault hook and check after chunk c = k indices [k0, k1)
hipError_t launch_nonfused_chunk(const NonFusedArgs& n, int c, int k0, int k1, hipStream_t stream);

// C = beta * C (beta == 0 writes zeros without reading C).
hipError_t launch_scale(float* C, int64_t ldc, int32_t M, int32_t N, float beta, hipStream_t stream);
// p[0 .. n) = 0 by a kernel (no memset node, so it replays correctly inside a HIP graph).
hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t stream);

// Device memory a run uses besides its operands: the counters, the event log,
// the fault sites and applied-fault log of the injection build, and the
// recompute queue (retry[0..1] zero between calls; retry_tiles holds
// retry_cap tile indices).  A handle owns one; ftgemm_run_noalloc uses a
// static one.
struct RunWorkspace {
    uint32_t* counters;
    ftgemm_event_t* events;
    int32_t event_cap;
    const ftgemm_fault_t* faults;
    int32_t n_faults;
    ftgemm_fault_log_t* fault_log;
    int32_t fault_log_cap;
    uint32_t* retry;
    int32_t* retry_tiles;
    int64_t retry_cap;
};

// Body of ftgemm_run and ftgemm_run_noalloc on the current device (defined in
// ftgemm_api.cpp).  `h` may be null.
int run_common(ftgemm_ctx* h, int dtype, float scale, RunWorkspace ws, int64_t m, int64_t n, int64_t k,
               float alpha, const void* A, int64_t lda, const void* B, int64_t ldb, float beta, float* C,
               int64_t ldc, int ft_level, float tol, hipStream_t stream, ftgemm_report_t* report);

}  // namespace ftgemm_impl
