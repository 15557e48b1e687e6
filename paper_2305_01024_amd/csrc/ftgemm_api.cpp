// ftgemm_api.cpp -- the C ABI declared in include/ftgemm.h: handle lifetime,
// argument checks, BLAS quick returns, kernel selection and launch, event log
// and fault-injection plumbing.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ftgemm_internal.h"

using namespace ftgemm_impl;

struct ftgemm_ctx {
    int device = 0;
    int dtype = FTGEMM_F32;
    float scale_a = 1.f, scale_b = 1.f;
    bool forced = false;
    ftgemm_config_t cfg{};
    ftgemm_event_t* d_events = nullptr;
    int event_cap = 0;
    uint32_t* d_counters = nullptr;
    ftgemm_fault_t* d_faults = nullptr;
    int n_faults = 0, fault_cap = 0;
    ftgemm_fault_log_t* d_flog = nullptr;
    int flog_cap = 0;
    // recompute queue: d_retry[0] queued tiles, d_retry[1] retry workgroups done
    uint32_t* d_retry = nullptr;
    int32_t* d_retry_tiles = nullptr;
    int retry_cap = 0;
    // workspace of ftgemm_run_nonfused
    float* d_nf = nullptr;
    int64_t nf_cap = 0;
    // workspace of ftgemm_run_z64 (doubles)
    double* d_z = nullptr;
    int64_t z_cap = 0;
    // configurations picked by ftgemm_tune, per (m, n, k, ft_level)
    std::vector<ftgemm_tuned_t> tuned;
    // batched plan of the last ftgemm_batched call
    std::vector<ftgemm_problem_t> plan_probs;
    std::vector<ftgemm_config_t> plan_cfg;
    bool plan_valid = false;
    BatchProblem* d_bprobs = nullptr;
    int bprobs_cap = 0;
    BatchItem* d_bitems = nullptr;
    int bitems_cap = 0;
    int n_items = 0;
    int grid = 0;
    bool plan_fp8 = false;   // the plan has FP8 problems: launch the kernel that holds the FP8 tile
    // cost model of the batched tile variants: multiply-adds per second
    double batch_rate[kBatchVariants] = {4.0e13, 2.0e13, 1.6e14, 1.7e14};
};

namespace {

constexpr int kEventCap = 16384;
constexpr int kFaultLogCap = 16384;
constexpr int kNumCUs = 256;

#define FT_HIP(call)                                   \
    do {                                               \
        if ((call) != hipSuccess) return FTGEMM_HIP_ERROR; \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int default_interval(int k_step) { return std::max(1, 256 / std::max(1, k_step)); }

// ft_level without / with the recompute flag
int base_level(int ft_level) { return ft_level & ~FTGEMM_FT_RECOMPUTE; }
bool wants_recompute(int ft_level) { return (ft_level & FTGEMM_FT_RECOMPUTE) != 0; }

int variant_count(int dtype) {
    return dtype == FTGEMM_BF16 ? bf16_variant_count() : dtype == FTGEMM_F8E4M3 ? fp8_variant_count()
           : (dtype == FTGEMM_F64 || dtype == FTGEMM_C64) ? fp64_variant_count() : fp32_variant_count();
}
Variant variant_at(int dtype, int v) {
    return dtype == FTGEMM_BF16 ? bf16_variant(v) : dtype == FTGEMM_F8E4M3 ? fp8_variant(v)
           : (dtype == FTGEMM_F64 || dtype == FTGEMM_C64) ? fp64_variant(v) : fp32_variant(v);
}
// A check shape of 0 stands for the compute tile's.
ftgemm_config_t normalized(ftgemm_config_t c) {
    if (c.check_m == 0) c.check_m = c.m_tile;
    if (c.check_n == 0) c.check_n = c.n_tile;
    return c;
}
int find_variant(int dtype, const ftgemm_config_t& c0) {
    const ftgemm_config_t c = normalized(c0);
    return dtype == FTGEMM_BF16     ? bf16_find_variant(c.m_tile, c.n_tile, c.k_step, c.check_m, c.check_n)
           : dtype == FTGEMM_F8E4M3 ? fp8_find_variant(c.m_tile, c.n_tile, c.k_step, c.check_m, c.check_n)
           : (dtype == FTGEMM_F64 || dtype == FTGEMM_C64)
                                    ? fp64_find_variant(c.m_tile, c.n_tile, c.k_step, c.check_m, c.check_n)
                                    : fp32_find_variant(c.m_tile, c.n_tile, c.k_step, c.check_m, c.check_n);
}
bool compute_tile_check(const Variant& x) { return x.check_m == x.m_tile && x.check_n == x.n_tile; }
bool dtype_supported(int dtype) {
    return dtype == FTGEMM_F32 || dtype == FTGEMM_BF16 || dtype == FTGEMM_F8E4M3 || dtype == FTGEMM_F64 ||
           dtype == FTGEMM_C64;
}

// Modelled time of an FP32 variant on an m x n output (the k extent is common
// to all variants and left out): the tiles run in waves of
// kNumCUs * wg_per_cu workgroups, and a full wave takes the time its work
// needs at the variant's full-load rate.  A last, partial wave with fewer
// wavefronts per SIMD than a full one takes the fraction of a full wave that
// its wavefronts per SIMD need, but at least kPartialWave (a wavefront that
// has its SIMD to itself runs faster, not proportionally: a 128x128
// workgroup alone on a compute unit takes ~0.65 of the time it takes beside
// another); a 64x64 workgroup is one wavefront, so a partial wave of it
// still takes a full wave's time.
double modelled_time(const Variant& x, const VariantModel& mdl, int64_t m, int64_t n, bool ft) {
    constexpr double kPartialWave = 0.65;
    constexpr int kSimdsPerCU = 4;
    const int64_t tiles = ((m + x.m_tile - 1) / x.m_tile) * ((n + x.n_tile - 1) / x.n_tile);
    const int64_t slots = (int64_t)kNumCUs * mdl.wg_per_cu;
    const double wave = (double)slots * x.m_tile * x.n_tile / (ft ? mdl.tflops_ft : mdl.tflops_plain);
    const int64_t full = tiles / slots, rem = tiles - full * slots;
    double t = (double)full * wave;
    if (rem > 0) {
        auto per_simd = [&](int64_t wg_per_cu) {
            return (wg_per_cu * mdl.waves_per_wg + kSimdsPerCU - 1) / kSimdsPerCU;
        };
        const double frac = (double)per_simd((rem + kNumCUs - 1) / kNumCUs) / (double)per_simd(mdl.wg_per_cu);
        t += wave * std::max(kPartialWave, frac);
    }
    return t;
}

// FP32, BF16 and FP8: the compute-tile variant with the least modelled time
// (ties: the earlier, larger tile); FP64 and double complex: their one
// variant.  A check every 256 k.
int select_variant(int dtype, int64_t m, int64_t n, int ft_level, ftgemm_config_t* out) {
    const int nv = variant_count(dtype);
    int pick = -1;
    double best = 0.0;
    for (int v = 0; v < nv; ++v) {
        const Variant x = variant_at(dtype, v);
        if (!compute_tile_check(x)) continue;
        if (dtype != FTGEMM_F32 && dtype != FTGEMM_BF16 && dtype != FTGEMM_F8E4M3) {
            pick = v;
            break;
        }
        const VariantModel mdl = dtype == FTGEMM_BF16     ? bf16_variant_model(v)
                                 : dtype == FTGEMM_F8E4M3 ? fp8_variant_model(v)
                                                          : fp32_variant_model(v);
        const double t = modelled_time(x, mdl, std::max<int64_t>(m, 1), std::max<int64_t>(n, 1),
                                       base_level(ft_level) > 0);
        if (pick < 0 || t < best * (1.0 - 1e-9)) {
            pick = v;
            best = t;
        }
    }
    const Variant x = variant_at(dtype, pick);
    out->m_tile = x.m_tile;
    out->n_tile = x.n_tile;
    out->k_step = x.k_step;
    out->check_interval = default_interval(x.k_step);
    out->check_m = x.check_m;
    out->check_n = x.check_n;
    return FTGEMM_OK;
}

bool find_tuned(const ftgemm_ctx* h, int64_t m, int64_t n, int64_t k, int ft_level, ftgemm_config_t* out) {
    for (const ftgemm_tuned_t& t : h->tuned)
        if (t.m == m && t.n == n && t.k == k && t.ft_level == ft_level) {
            *out = t.config;
            return true;
        }
    return false;
}

bool dims_ok(int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb, int64_t ldc) {
    return m >= 0 && m <= INT32_MAX && n >= 0 && n <= INT32_MAX && k >= 0 && k <= INT32_MAX &&
           lda >= std::max<int64_t>(1, m) && ldb >= std::max<int64_t>(1, k) && ldc >= std::max<int64_t>(1, m);
}

// Per-problem checks of a batched call; returns the index of the first bad problem or -1.
int first_bad_problem(int count, const ftgemm_problem_t* probs) {
    for (int p = 0; p < count; ++p) {
        const ftgemm_problem_t& q = probs[p];
        if (q.dtype != FTGEMM_F32 && q.dtype != FTGEMM_BF16 && q.dtype != FTGEMM_F8E4M3) return p;
        if (q.reserved_ != 0 || !dims_ok(q.m, q.n, q.k, q.lda, q.ldb, q.ldc)) return p;
        if (q.m > 0 && q.n > 0 && !q.C) return p;
        if (q.m > 0 && q.n > 0 && q.k > 0 && q.alpha != 0.f && (!q.A || !q.B)) return p;
        if (q.dtype != FTGEMM_F32 && !(q.scale_a > 0.f && q.scale_b > 0.f)) return p;
    }
    return -1;
}

// Tile variant of the batched kernel for a problem: the one with the least
// modelled time (padded multiply-adds over the variant's measured rate).
int pick_batch_variant(const ftgemm_ctx* h, const ftgemm_problem_t& q) {
    int best = -1;
    double best_t = 0.0;
    for (int v = 0; v < kBatchVariants; ++v) {
        if (batch_variant_dtype(v) != q.dtype) continue;
        const Variant x = batch_variant(v);
        const double padded = (double)((q.m + x.m_tile - 1) / x.m_tile) * x.m_tile *
                              (double)((q.n + x.n_tile - 1) / x.n_tile) * x.n_tile *
                              (double)((q.k + x.k_step - 1) / x.k_step) * x.k_step;
        const double t = padded / h->batch_rate[v];
        if (best < 0 || t < best_t) {
            best = v;
            best_t = t;
        }
    }
    return best;
}

template <class T>
int grow(T** buf, int* cap, int need) {
    if (need <= *cap) return FTGEMM_OK;
    if (*buf) (void)hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
    if (hipMalloc(buf, sizeof(T) * (size_t)need) != hipSuccess) return FTGEMM_NO_MEMORY;
    *cap = need;
    return FTGEMM_OK;
}

// Build the device plan of a batched call: per-problem descriptors and the
// cost-ordered (problem, tile) list.
int build_plan(ftgemm_ctx* h, int count, const ftgemm_problem_t* probs) {
    std::vector<BatchProblem> bp((size_t)count);
    std::vector<ftgemm_config_t> cfgs((size_t)count, ftgemm_config_t{0, 0, 0, 0, 0, 0});
    struct Work { double cost; BatchItem item; };
    std::vector<Work> work;
    for (int p = 0; p < count; ++p) {
        const ftgemm_problem_t& q = probs[p];
        BatchProblem& d = bp[(size_t)p];
        std::memset(&d, 0, sizeof(d));
        d.A = q.A;
        d.B = q.B;
        d.C = q.C;
        d.lda = q.lda;
        d.ldb = q.ldb;
        d.ldc = q.ldc;
        d.M = (int32_t)q.m;
        d.N = (int32_t)q.n;
        d.K = (int32_t)q.k;
        d.alpha = q.alpha;
        d.beta = q.beta;
        d.scale = q.dtype == FTGEMM_F32 ? 1.0f : q.scale_a * q.scale_b;
        if (q.m == 0 || q.n == 0) {
            d.variant = -1;
            d.ntm = 1;
            continue;
        }
        int bm = 128, bn = 128;
        double per_tile = 1.0;
        if (q.k == 0 || q.alpha == 0.f) {
            d.variant = -1;
        } else {
            d.variant = pick_batch_variant(h, q);
            const Variant x = batch_variant(d.variant);
            bm = x.m_tile;
            bn = x.n_tile;
            d.check_interval = default_interval(x.k_step);
            cfgs[(size_t)p] = {x.m_tile, x.n_tile, x.k_step, d.check_interval, x.check_m, x.check_n};
            const int64_t nk = (q.k + x.k_step - 1) / x.k_step;
            per_tile = (double)bm * bn * (double)(nk * x.k_step) / h->batch_rate[d.variant];
        }
        d.ntm = (int32_t)((q.m + bm - 1) / bm);
        const int64_t ntn = (q.n + bn - 1) / bn;
        for (int64_t t = 0; t < (int64_t)d.ntm * ntn; ++t) work.push_back({per_tile, {p, (int32_t)t}});
    }
    std::stable_sort(work.begin(), work.end(), [](const Work& x, const Work& y) { return x.cost > y.cost; });
    std::vector<BatchItem> items(work.size());
    for (size_t i = 0; i < work.size(); ++i) items[i] = work[i].item;
    if (grow(&h->d_bprobs, &h->bprobs_cap, std::max(1, count)) != FTGEMM_OK) return FTGEMM_NO_MEMORY;
    if (grow(&h->d_bitems, &h->bitems_cap, std::max<int>(1, (int)items.size())) != FTGEMM_OK) return FTGEMM_NO_MEMORY;
    if (count > 0)
        FT_HIP(hipMemcpy(h->d_bprobs, bp.data(), sizeof(BatchProblem) * (size_t)count, hipMemcpyHostToDevice));
    if (!items.empty())
        FT_HIP(hipMemcpy(h->d_bitems, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice));
    h->n_items = (int)items.size();
    h->plan_fp8 = false;
    for (const BatchProblem& d : bp) h->plan_fp8 = h->plan_fp8 || (d.variant >= 0 && batch_variant_dtype(d.variant) == FTGEMM_F8E4M3);
    h->grid = std::max(1, std::min(h->n_items, batch_resident_blocks(h->device, h->plan_fp8)));
    h->plan_probs.assign(probs, probs + count);
    h->plan_cfg = cfgs;
    h->plan_valid = true;
    return FTGEMM_OK;
}

bool same_plan(const ftgemm_ctx* h, int count, const ftgemm_problem_t* probs) {
    return h->plan_valid && (int)h->plan_probs.size() == count &&
           (count == 0 || std::memcmp(h->plan_probs.data(), probs, sizeof(ftgemm_problem_t) * (size_t)count) == 0);
}

// Counters and events of the last launch into the report.  Every count,
// `checks` included, is taken on the device.
int fill_report(const RunWorkspace& ws, hipStream_t stream, ftgemm_report_t* report, bool recompute = false) {
    FT_HIP(hipStreamSynchronize(stream));
    uint32_t cnt[CNT_N];
    FT_HIP(hipMemcpy(cnt, ws.counters, sizeof(cnt), hipMemcpyDeviceToHost));
    report->checks = cnt[CNT_CHECKS];
    report->detected = cnt[CNT_DETECTED];
    report->corrected = cnt[CNT_CORRECTED];
    report->uncorrectable = cnt[CNT_UNCORRECTABLE];
    report->checksum_only = cnt[CNT_CHECKSUM_ONLY];
    report->nonfinite_input = cnt[CNT_NONFINITE];
    report->recomputed = cnt[CNT_RECOMPUTED];
    report->recompute_failed = cnt[CNT_RECOMPUTE_FAILED];
    const uint32_t logged = std::min<uint32_t>(cnt[CNT_EVENTS], (uint32_t)ws.event_cap);
    const uint32_t copy = report->events ? std::min<uint32_t>(logged, report->cap_events) : 0;
    if (copy > 0)
        FT_HIP(hipMemcpy(report->events, ws.events, sizeof(ftgemm_event_t) * copy, hipMemcpyDeviceToHost));
    report->n_events = copy;
    if (cnt[CNT_EVENTS] > copy && report->events) return FTGEMM_LOG_OVERFLOW;
    if (recompute ? report->recompute_failed > 0 : report->uncorrectable > 0) return FTGEMM_UNCORRECTABLE;
    return report->nonfinite_input > 0 ? FTGEMM_NONFINITE_INPUT : FTGEMM_OK;
}

// The device memory of a handle as a run's workspace.
RunWorkspace workspace_of(const ftgemm_ctx* h) {
    RunWorkspace ws{};
    ws.counters = h->d_counters;
    ws.events = h->d_events;
    ws.event_cap = h->event_cap;
    ws.faults = h->n_faults > 0 ? h->d_faults : nullptr;
    ws.n_faults = h->n_faults;
    ws.fault_log = h->d_flog;
    ws.fault_log_cap = h->flog_cap;
    ws.retry = h->d_retry;
    ws.retry_tiles = h->d_retry_tiles;
    ws.retry_cap = h->retry_cap;
    return ws;
}
int fill_report(ftgemm_ctx* h, hipStream_t stream, ftgemm_report_t* report, bool recompute = false) {
    return fill_report(workspace_of(h), stream, report, recompute);
}

// Zero the report's outputs (the caller's events and cap_events stay).
void reset_report(ftgemm_report_t* report) {
    if (!report) return;
    report->checks = report->detected = report->corrected = 0;
    report->uncorrectable = report->checksum_only = report->nonfinite_input = 0;
    report->n_events = 0;
    report->bad_arg = 0;
    report->tol_used = 0.f;
    report->bad_problem = -1;
    report->recomputed = report->recompute_failed = 0;
    std::memset(&report->config, 0, sizeof(report->config));
}

}  // namespace

namespace ftgemm_impl {

// Body of ftgemm_run and ftgemm_run_noalloc: argument checks, BLAS quick
// returns, configuration, the launches and the report, on the workspace `ws`
// and the current device.  `h` (may be null) supplies a forced or tuned
// configuration and grows its own recompute queue; without a handle the
// queue must already hold every tile (FTGEMM_NO_MEMORY otherwise).
int run_common(ftgemm_ctx* h, int dtype, float scale, RunWorkspace ws, int64_t m, int64_t n, int64_t k,
               float alpha, const void* A, int64_t lda, const void* B, int64_t ldb, float beta, float* C,
               int64_t ldc, int ft_level, float tol, hipStream_t stream, ftgemm_report_t* report) {
    int32_t bad = 0;
    if (ftgemm_validate(m, n, k, lda, ldb, ldc, ft_level, tol, &bad) != FTGEMM_OK) {
        if (report) report->bad_arg = bad;
        return FTGEMM_INVALID;
    }
    if (!dtype_supported(dtype) || dtype == FTGEMM_F64 || dtype == FTGEMM_C64)
        return FTGEMM_UNSUPPORTED;   // binary64: ftgemm_run_f64, complex: ftgemm_run_z64
    const float c = tol > 0.f ? tol : 2.0f;
    if (report) report->tol_used = c;
    if (m == 0 || n == 0) return FTGEMM_OK;
    if (!C) {
        if (report) report->bad_arg = 11;
        return FTGEMM_INVALID;
    }
    if (k == 0 || alpha == 0.f) {
        FT_HIP(launch_scale(C, ldc, (int32_t)m, (int32_t)n, beta, stream));
        if (report) FT_HIP(hipStreamSynchronize(stream));
        return FTGEMM_OK;
    }
    if (!A || !B) {
        if (report) report->bad_arg = !A ? 6 : 8;
        return FTGEMM_INVALID;
    }

    const bool recompute = wants_recompute(ft_level);
    ft_level = base_level(ft_level);
    ftgemm_config_t cfg;
    if (h && h->forced) cfg = h->cfg;
    else if (!(h && find_tuned(h, m, n, k, ft_level, &cfg))) select_variant(dtype, m, n, ft_level, &cfg);
    const int variant = find_variant(dtype, cfg);
    if (variant < 0) return FTGEMM_UNSUPPORTED;
    const int64_t ntiles = ((m + cfg.m_tile - 1) / cfg.m_tile) * ((n + cfg.n_tile - 1) / cfg.n_tile);
    if (recompute) {
        if (h) {
            if (grow(&h->d_retry_tiles, &h->retry_cap, (int)ntiles) != FTGEMM_OK) return FTGEMM_NO_MEMORY;
            ws.retry_tiles = h->d_retry_tiles;
            ws.retry_cap = h->retry_cap;
        } else if (ntiles > ws.retry_cap) {
            return FTGEMM_NO_MEMORY;
        }
    }

    const bool inject = ws.n_faults > 0;
    if (report || inject) FT_HIP(launch_zero_u32(ws.counters, CNT_N, stream));

    LaunchArgs a{};
    a.A = static_cast<const float*>(A);
    a.B = static_cast<const float*>(B);
    a.C = C;
    a.lda = lda;
    a.ldb = ldb;
    a.ldc = ldc;
    a.M = (int32_t)m;
    a.N = (int32_t)n;
    a.K = (int32_t)k;
    a.alpha = alpha;
    a.beta = beta;
    a.scale = scale;
    a.tol_c = c;
    a.check_interval = ft_level == 1 ? INT32_MAX : cfg.check_interval;   // detect-only: after the last step
    a.ft_level = ft_level;
    a.problem = 0;
    a.events = ws.events;
    a.counters = ws.counters;
    a.event_cap = ws.event_cap;
    a.faults = inject ? ws.faults : nullptr;
    a.n_faults = inject ? ws.n_faults : 0;
    a.fault_log = ws.fault_log;
    a.fault_log_cap = ws.fault_log_cap;
    a.retry = recompute ? ws.retry : nullptr;
    a.retry_tiles = recompute ? ws.retry_tiles : nullptr;
    a.retry_pass = 0;
    if (dtype == FTGEMM_BF16) FT_HIP(launch_bf16(variant, inject, a, stream));
    else if (dtype == FTGEMM_F8E4M3) FT_HIP(launch_fp8(variant, inject, a, stream));
    else FT_HIP(launch_fp32(variant, inject, a, stream));
    if (recompute) {
        // the queued tiles again, without injection; one workgroup per compute
        // unit at most, each walking the queue
        LaunchArgs r = a;
        r.retry_pass = 1;
        r.faults = nullptr;
        r.n_faults = 0;
        const int grid = (int)std::min<int64_t>(ntiles, kNumCUs);
        if (dtype == FTGEMM_BF16) FT_HIP(launch_bf16_retry(variant, r, grid, stream));
        else if (dtype == FTGEMM_F8E4M3) FT_HIP(launch_fp8_retry(variant, r, grid, stream));
        else FT_HIP(launch_fp32_retry(variant, r, grid, stream));
    }

    if (!report) return FTGEMM_OK;
    report->config = cfg;
    return fill_report(ws, stream, report, recompute);
}

}  // namespace ftgemm_impl

extern "C" {

const char* ftgemm_status_string(int s) {
    switch (s) {
        case FTGEMM_OK: return "ok";
        case FTGEMM_UNCORRECTABLE: return "uncorrectable fault pattern in at least one tile";
        case FTGEMM_NONFINITE_INPUT: return "operands hold Inf or NaN: the tiles that read them were not checked";
        case FTGEMM_INVALID: return "invalid argument";
        case FTGEMM_UNSUPPORTED: return "unsupported dtype, level, configuration or device";
        case FTGEMM_HIP_ERROR: return "HIP runtime error";
        case FTGEMM_NO_MEMORY: return "out of memory";
        case FTGEMM_LOG_OVERFLOW: return "event log overflow";
        default: return "unknown status";
    }
}

int ftgemm_validate(int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb, int64_t ldc,
                    int ft_level, float tol, int32_t* bad_arg) {
    int bad = 0;
    if (m < 0 || m > INT32_MAX) bad = 2;
    else if (n < 0 || n > INT32_MAX) bad = 3;
    else if (k < 0 || k > INT32_MAX) bad = 4;
    else if (lda < std::max<int64_t>(1, m)) bad = 7;
    else if (ldb < std::max<int64_t>(1, k)) bad = 9;
    else if (ldc < std::max<int64_t>(1, m)) bad = 12;
    else if (base_level(ft_level) < 0 || base_level(ft_level) > 2 ||
             (wants_recompute(ft_level) && base_level(ft_level) == 0)) bad = 13;
    else if (!(tol == tol) || tol > 1e30f) bad = 14;   // NaN or absurd
    if (bad_arg) *bad_arg = bad;
    return bad ? FTGEMM_INVALID : FTGEMM_OK;
}

int ftgemm_select_config(int dtype, int64_t m, int64_t n, int64_t k, int ft_level, ftgemm_config_t* config) {
    (void)k;
    if (!config) return FTGEMM_INVALID;
    if (!dtype_supported(dtype)) return FTGEMM_UNSUPPORTED;
    return select_variant(dtype, m, n, ft_level, config);
}

int ftgemm_create(ftgemm_t* handle, int dtype, int device) {
    if (!handle) return FTGEMM_INVALID;
    *handle = nullptr;
    if (!dtype_supported(dtype)) return FTGEMM_UNSUPPORTED;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FTGEMM_UNSUPPORTED;
    hipDeviceProp_t prop;
    FT_HIP(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FTGEMM_UNSUPPORTED;
    DeviceGuard g(device);
    ftgemm_ctx* h = new (std::nothrow) ftgemm_ctx();
    if (!h) return FTGEMM_NO_MEMORY;
    h->device = device;
    h->dtype = dtype;
    h->event_cap = kEventCap;
    h->flog_cap = kFaultLogCap;
    if (hipMalloc(&h->d_events, sizeof(ftgemm_event_t) * kEventCap) != hipSuccess ||
        hipMalloc(&h->d_counters, sizeof(uint32_t) * CNT_N) != hipSuccess ||
        hipMalloc(&h->d_flog, sizeof(ftgemm_fault_log_t) * kFaultLogCap) != hipSuccess ||
        hipMalloc(&h->d_retry, sizeof(uint32_t) * 2) != hipSuccess) {
        ftgemm_destroy(h);
        return FTGEMM_NO_MEMORY;
    }
    if (hipMemset(h->d_counters, 0, sizeof(uint32_t) * CNT_N) != hipSuccess ||
        hipMemset(h->d_retry, 0, sizeof(uint32_t) * 2) != hipSuccess) {
        ftgemm_destroy(h);
        return FTGEMM_HIP_ERROR;
    }
    *handle = h;
    return FTGEMM_OK;
}

int ftgemm_destroy(ftgemm_t h) {
    if (!h) return FTGEMM_INVALID;
    {
        DeviceGuard g(h->device);
        if (h->d_events) (void)hipFree(h->d_events);
        if (h->d_counters) (void)hipFree(h->d_counters);
        if (h->d_faults) (void)hipFree(h->d_faults);
        if (h->d_flog) (void)hipFree(h->d_flog);
        if (h->d_bprobs) (void)hipFree(h->d_bprobs);
        if (h->d_bitems) (void)hipFree(h->d_bitems);
        if (h->d_retry) (void)hipFree(h->d_retry);
        if (h->d_retry_tiles) (void)hipFree(h->d_retry_tiles);
        if (h->d_nf) (void)hipFree(h->d_nf);
        if (h->d_z) (void)hipFree(h->d_z);
    }
    delete h;
    return FTGEMM_OK;
}

int ftgemm_set_scales(ftgemm_t h, float scale_a, float scale_b) {
    if (!h || !(scale_a > 0.f) || !(scale_b > 0.f)) return FTGEMM_INVALID;
    h->scale_a = scale_a;
    h->scale_b = scale_b;
    return FTGEMM_OK;
}

int ftgemm_set_config(ftgemm_t h, const ftgemm_config_t* c) {
    if (!h) return FTGEMM_INVALID;
    if (!c) {
        h->forced = false;
        return FTGEMM_OK;
    }
    if (c->check_interval < 1 || c->check_m < 0 || c->check_n < 0) return FTGEMM_INVALID;
    if (find_variant(h->dtype, *c) < 0) return FTGEMM_UNSUPPORTED;
    h->cfg = normalized(*c);
    h->forced = true;
    return FTGEMM_OK;
}

int ftgemm_set_injection(ftgemm_t h, const ftgemm_fault_t* faults, int n) {
    if (!h || n < 0 || (n > 0 && !faults)) return FTGEMM_INVALID;
    for (int q = 0; q < n; ++q) {
        const ftgemm_fault_t& f = faults[q];
        if (f.tile_m < 0 || f.tile_n < 0 || f.kstep < 0 || f.row < 0 || f.col < 0 || f.problem < 0)
            return FTGEMM_INVALID;
        if (f.kind != FTGEMM_FAULT_ADD && f.kind != FTGEMM_FAULT_XOR) return FTGEMM_INVALID;
        const float top_bit = (h->dtype == FTGEMM_F64 || h->dtype == FTGEMM_C64) ? 63.f : 31.f;
        if (f.kind == FTGEMM_FAULT_XOR && !(f.payload >= 0.f && f.payload <= top_bit)) return FTGEMM_INVALID;
    }
    DeviceGuard g(h->device);
    if (n > h->fault_cap) {
        if (h->d_faults) (void)hipFree(h->d_faults);
        h->d_faults = nullptr;
        h->fault_cap = 0;
        if (hipMalloc(&h->d_faults, sizeof(ftgemm_fault_t) * (size_t)n) != hipSuccess) {
            h->n_faults = 0;
            return FTGEMM_NO_MEMORY;
        }
        h->fault_cap = n;
    }
    if (n > 0) FT_HIP(hipMemcpy(h->d_faults, faults, sizeof(ftgemm_fault_t) * (size_t)n, hipMemcpyHostToDevice));
    h->n_faults = n;
    return FTGEMM_OK;
}

int ftgemm_get_injection_log(ftgemm_t h, ftgemm_fault_log_t* out, int cap, int* n) {
    if (!h || cap < 0 || (cap > 0 && !out)) return FTGEMM_INVALID;
    DeviceGuard g(h->device);
    uint32_t cnt[CNT_N];
    FT_HIP(hipMemcpy(cnt, h->d_counters, sizeof(cnt), hipMemcpyDeviceToHost));
    const int applied = (int)cnt[CNT_FAULTS];
    const int copy = std::min(std::min(applied, cap), h->flog_cap);
    if (copy > 0) FT_HIP(hipMemcpy(out, h->d_flog, sizeof(ftgemm_fault_log_t) * (size_t)copy, hipMemcpyDeviceToHost));
    if (n) *n = copy;
    return applied > copy ? FTGEMM_LOG_OVERFLOW : FTGEMM_OK;
}

int ftgemm_run(ftgemm_t h, int64_t m, int64_t n, int64_t k, float alpha, const void* A, int64_t lda,
               const void* B, int64_t ldb, float beta, float* C, int64_t ldc, int ft_level, float tol,
               hipStream_t stream, ftgemm_report_t* report) {
    reset_report(report);
    if (!h) {
        if (report) report->bad_arg = 1;
        return FTGEMM_INVALID;
    }
    DeviceGuard g(h->device);
    const float scale = h->dtype == FTGEMM_F32 ? 1.0f : h->scale_a * h->scale_b;
    return run_common(h, h->dtype, scale, workspace_of(h), m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                      ft_level, tol, stream, report);
}

int ftgemm_run_f64(ftgemm_t h, int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int ft_level, double tol,
                   hipStream_t stream, ftgemm_report_t* report) {
    int32_t bad = 0;
    reset_report(report);
    if (!h) {
        if (report) report->bad_arg = 1;
        return FTGEMM_INVALID;
    }
    if (ftgemm_validate(m, n, k, lda, ldb, ldc, ft_level, (float)std::min(tol, 1e31), &bad) != FTGEMM_OK) {
        if (report) report->bad_arg = bad;
        return FTGEMM_INVALID;
    }
    if (h->dtype != FTGEMM_F64 || wants_recompute(ft_level)) return FTGEMM_UNSUPPORTED;
    const float c = tol > 0.0 ? (float)tol : 2.0f;
    if (report) report->tol_used = c;
    if (m == 0 || n == 0) return FTGEMM_OK;
    if (!C) {
        if (report) report->bad_arg = 11;
        return FTGEMM_INVALID;
    }
    DeviceGuard g(h->device);
    if (k == 0 || alpha == 0.0) {
        FT_HIP(launch_scale64(C, ldc, (int32_t)m, (int32_t)n, beta, stream));
        if (report) FT_HIP(hipStreamSynchronize(stream));
        return FTGEMM_OK;
    }
    if (!A || !B) {
        if (report) report->bad_arg = !A ? 6 : 8;
        return FTGEMM_INVALID;
    }
    ftgemm_config_t cfg;
    if (h->forced) cfg = h->cfg;
    else select_variant(FTGEMM_F64, m, n, ft_level, &cfg);
    const int variant = find_variant(FTGEMM_F64, cfg);
    if (variant < 0) return FTGEMM_UNSUPPORTED;

    const bool inject = h->n_faults > 0;
    if (report || inject) FT_HIP(launch_zero_u32(h->d_counters, CNT_N, stream));
    F64Args a{};
    a.A = A;
    a.B = B;
    a.C = C;
    a.lda = lda;
    a.ldb = ldb;
    a.ldc = ldc;
    a.M = (int32_t)m;
    a.N = (int32_t)n;
    a.K = (int32_t)k;
    a.alpha = alpha;
    a.beta = beta;
    a.tol_c = c;
    a.check_interval = ft_level == 1 ? INT32_MAX : cfg.check_interval;   // detect-only: after the last step
    a.ft_level = ft_level;
    a.problem = 0;
    a.events = h->d_events;
    a.counters = h->d_counters;
    a.event_cap = h->event_cap;
    a.faults = inject ? h->d_faults : nullptr;
    a.n_faults = inject ? h->n_faults : 0;
    a.fault_log = h->d_flog;
    a.fault_log_cap = h->flog_cap;
    FT_HIP(launch_fp64(variant, inject, a, stream));
    if (!report) return FTGEMM_OK;
    report->config = cfg;
    return fill_report(h, stream, report);
}

int ftgemm_run_z64(ftgemm_t h, int64_t m, int64_t n, int64_t k, const double* alpha, const void* A, int64_t lda,
                   const void* B, int64_t ldb, const double* beta, void* C, int64_t ldc, int ft_level, double tol,
                   hipStream_t stream, ftgemm_report_t* report) {
    int32_t bad = 0;
    reset_report(report);
    if (!h) {
        if (report) report->bad_arg = 1;
        return FTGEMM_INVALID;
    }
    if (ftgemm_validate(m, n, k, lda, ldb, ldc, ft_level, (float)std::min(tol, 1e31), &bad) != FTGEMM_OK) {
        if (report) report->bad_arg = bad;
        return FTGEMM_INVALID;
    }
    if (!alpha || !beta) {
        if (report) report->bad_arg = !alpha ? 5 : 10;
        return FTGEMM_INVALID;
    }
    // the real products have 2k inner indices
    if (2 * k > INT32_MAX) {
        if (report) report->bad_arg = 4;
        return FTGEMM_INVALID;
    }
    if (h->dtype != FTGEMM_C64 || wants_recompute(ft_level)) return FTGEMM_UNSUPPORTED;
    const float c = tol > 0.0 ? (float)tol : 2.0f;
    if (report) report->tol_used = c;
    if (m == 0 || n == 0) return FTGEMM_OK;
    if (!C) {
        if (report) report->bad_arg = 11;
        return FTGEMM_INVALID;
    }
    DeviceGuard g(h->device);
    double* Cz = static_cast<double*>(C);
    if (k == 0 || (alpha[0] == 0.0 && alpha[1] == 0.0)) {
        FT_HIP(launch_zscale(Cz, ldc, (int32_t)m, (int32_t)n, beta, stream));
        if (report) FT_HIP(hipStreamSynchronize(stream));
        return FTGEMM_OK;
    }
    if (!A || !B) {
        if (report) report->bad_arg = !A ? 6 : 8;
        return FTGEMM_INVALID;
    }
    ftgemm_config_t cfg;
    if (h->forced) cfg = h->cfg;
    else select_variant(FTGEMM_C64, m, n, ft_level, &cfg);
    const int variant = find_variant(FTGEMM_C64, cfg);
    if (variant < 0) return FTGEMM_UNSUPPORTED;

    // workspace: A', A'' (m x 2k each), then the real and imaginary accumulators (m x n each)
    const int64_t need = 4 * m * k + 2 * m * n;
    if (need > h->z_cap) {
        if (h->d_z) (void)hipFree(h->d_z);
        h->d_z = nullptr;
        h->z_cap = 0;
        if (hipMalloc(&h->d_z, sizeof(double) * (size_t)need) != hipSuccess) return FTGEMM_NO_MEMORY;
        h->z_cap = need;
    }
    double* Ap = h->d_z;
    double* App = Ap + 2 * m * k;
    double* Pr = App + 2 * m * k;
    double* Pi = Pr + m * n;
    FT_HIP(launch_zrepack(static_cast<const double*>(A), lda, (int32_t)m, (int32_t)k, Ap, App, stream));

    const bool inject = h->n_faults > 0;
    if (report || inject) FT_HIP(launch_zero_u32(h->d_counters, CNT_N, stream));
    F64Args a{};
    a.B = static_cast<const double*>(B);   // B' = B's (re, im) storage as a real 2k x n matrix
    a.lda = m;
    a.ldb = 2 * ldb;
    a.ldc = m;
    a.M = (int32_t)m;
    a.N = (int32_t)n;
    a.K = (int32_t)(2 * k);
    a.alpha = 1.0;
    a.beta = 0.0;
    a.tol_c = c;
    a.check_interval = ft_level == 1 ? INT32_MAX : cfg.check_interval;   // detect-only: after the last step
    a.ft_level = ft_level;
    a.events = h->d_events;
    a.counters = h->d_counters;
    a.event_cap = h->event_cap;
    a.faults = inject ? h->d_faults : nullptr;
    a.n_faults = inject ? h->n_faults : 0;
    a.fault_log = h->d_flog;
    a.fault_log_cap = h->flog_cap;
    for (int comp = 0; comp < 2; ++comp) {   // real part, then imaginary part
        a.A = comp == 0 ? Ap : App;
        a.C = comp == 0 ? Pr : Pi;
        a.problem = comp;
        FT_HIP(launch_fp64(variant, inject, a, stream));
    }
    FT_HIP(launch_zepilogue(Cz, ldc, (int32_t)m, (int32_t)n, Pr, Pi, alpha, beta, stream));
    if (!report) return FTGEMM_OK;
    report->config = cfg;
    return fill_report(h, stream, report);
}

int ftgemm_run_nonfused(ftgemm_t h, int64_t m, int64_t n, int64_t k, float alpha, const void* A, int64_t lda,
                        const void* B, int64_t ldb, float beta, float* C, int64_t ldc, int check_k, float tol,
                        hipStream_t stream, ftgemm_report_t* report) {
    int32_t bad = 0;
    reset_report(report);
    if (!h) bad = 1;
    else if (ftgemm_validate(m, n, k, lda, ldb, ldc, FTGEMM_FT_CORRECT, tol, &bad) != FTGEMM_OK) {}
    else if (check_k < 0) bad = 13;
    if (bad) {
        if (report) report->bad_arg = bad;
        return FTGEMM_INVALID;
    }
    if (h->dtype != FTGEMM_F32 || alpha != 1.0f || beta != 0.0f) return FTGEMM_UNSUPPORTED;
    const float c = tol > 0.f ? tol : 2.0f;
    if (report) report->tol_used = c;
    if (m == 0 || n == 0) return FTGEMM_OK;
    if (!C) {
        if (report) report->bad_arg = 11;
        return FTGEMM_INVALID;
    }
    DeviceGuard g(h->device);
    if (k == 0) {
        FT_HIP(launch_scale(C, ldc, (int32_t)m, (int32_t)n, 0.0f, stream));
        if (report) FT_HIP(hipStreamSynchronize(stream));
        return FTGEMM_OK;
    }
    if (!A || !B) {
        if (report) report->bad_arg = !A ? 6 : 8;
        return FTGEMM_INVALID;
    }
    const int64_t T = kNonFusedTile;
    const int64_t ntm = (m + T - 1) / T, ntn = (n + T - 1) / T;
    const int64_t ck = check_k > 0 ? check_k : 256;
    const int64_t nchunks = (k + ck - 1) / ck;
    // workspace: W [ntm][k], V [ntn][k], R [ntn][m], S [ntm][n], na2 [m], nb2 [n]
    const int64_t need = ntm * k + ntn * k + ntn * m + ntm * n + m + n + ntm * ntn;
    if (need > h->nf_cap) {
        if (h->d_nf) (void)hipFree(h->d_nf);
        h->d_nf = nullptr;
        h->nf_cap = 0;
        if (hipMalloc(&h->d_nf, sizeof(float) * (size_t)need) != hipSuccess) return FTGEMM_NO_MEMORY;
        h->nf_cap = need;
    }
    NonFusedArgs nf{};
    nf.A = static_cast<const float*>(A);
    nf.B = static_cast<const float*>(B);
    nf.C = C;
    nf.lda = lda;
    nf.ldb = ldb;
    nf.ldc = ldc;
    nf.M = (int32_t)m;
    nf.N = (int32_t)n;
    nf.K = (int32_t)k;
    nf.tol_c = c;
    nf.W = h->d_nf;
    nf.V = nf.W + ntm * k;
    nf.R = nf.V + ntn * k;
    nf.S = nf.R + ntn * m;
    nf.na2 = nf.S + ntm * n;
    nf.nb2 = nf.na2 + m;
    nf.tile_flag = reinterpret_cast<unsigned*>(nf.nb2 + n);
    nf.events = h->d_events;
    nf.event_cap = h->event_cap;
    nf.counters = h->d_counters;
    const bool inject = h->n_faults > 0;
    nf.faults = inject ? h->d_faults : nullptr;
    nf.n_faults = inject ? h->n_faults : 0;
    nf.fault_log = h->d_flog;
    nf.fault_log_cap = h->flog_cap;
    if (report || inject) FT_HIP(hipMemsetAsync(h->d_counters, 0, sizeof(uint32_t) * CNT_N, stream));
    FT_HIP(hipMemsetAsync(nf.R, 0, sizeof(float) * (size_t)(ntn * m + ntm * n + m + n + ntm * ntn), stream));
    FT_HIP(launch_nonfused_encode(nf, stream));

    // the plain kernel for the chunk shape: a configuration tuned for (m, n, chunk) at
    // level 0 if the handle has one, else the default
    ftgemm_config_t cfg;
    if (!find_tuned(h, m, n, std::min<int64_t>(ck, k), FTGEMM_FT_OFF, &cfg)) select_variant(FTGEMM_F32, m, n, FTGEMM_FT_OFF, &cfg);
    const int variant = find_variant(FTGEMM_F32, cfg);
    if (variant < 0) return FTGEMM_UNSUPPORTED;
    LaunchArgs a{};
    a.C = C;
    a.lda = lda;
    a.ldb = ldb;
    a.ldc = ldc;
    a.M = (int32_t)m;
    a.N = (int32_t)n;
    a.alpha = 1.0f;
    a.scale = 1.0f;
    a.tol_c = c;
    a.check_interval = 1;
    a.ft_level = 0;
    a.events = h->d_events;
    a.counters = h->d_counters;
    a.event_cap = h->event_cap;
    a.fault_log = h->d_flog;
    a.fault_log_cap = h->flog_cap;
    for (int64_t q = 0; q < nchunks; ++q) {
        const int64_t k0 = q * ck, k1 = std::min(k, k0 + ck);
        a.A = static_cast<const float*>(A) + k0 * lda;
        a.B = static_cast<const float*>(B) + k0;
        a.K = (int32_t)(k1 - k0);
        a.beta = q == 0 ? 0.0f : 1.0f;
        FT_HIP(launch_fp32(variant, false, a, stream));
        FT_HIP(launch_nonfused_chunk(nf, (int)q, (int)k0, (int)k1, stream));
    }
    if (!report) return FTGEMM_OK;
    report->config = ftgemm_config_t{(int32_t)T, (int32_t)T, (int32_t)ck, 1, (int32_t)T, (int32_t)T};
    return fill_report(h, stream, report);
}

int ftgemm_batched(ftgemm_t h, int count, const ftgemm_problem_t* probs, int ft_level, float tol,
                   hipStream_t stream, ftgemm_report_t* report) {
    reset_report(report);
    int bad = 0;
    if (!h) bad = 1;
    else if (count < 0 || (count > 0 && !probs)) bad = 2;
    else if (ft_level < 0 || ft_level > 2) bad = 4;
    else if (!(tol == tol) || tol > 1e30f) bad = 5;
    if (bad) {
        if (report) report->bad_arg = bad;
        return FTGEMM_INVALID;
    }
    const int bp = first_bad_problem(count, probs);
    if (bp >= 0) {
        if (report) {
            report->bad_arg = 3;
            report->bad_problem = bp;
        }
        return FTGEMM_INVALID;
    }
    const float c = tol > 0.f ? tol : 2.0f;
    if (report) report->tol_used = c;
    DeviceGuard g(h->device);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    FT_HIP(hipStreamIsCapturing(stream, &cap));
    const bool capturing = cap != hipStreamCaptureStatusNone;
    const bool inject = h->n_faults > 0;
    if (capturing && (report || inject)) {
        if (report) report->bad_arg = 7;
        return FTGEMM_INVALID;
    }
    if (!same_plan(h, count, probs)) {
        if (capturing) {
            if (report) report->bad_arg = 3;
            return FTGEMM_INVALID;
        }
        const int st = build_plan(h, count, probs);
        if (st != FTGEMM_OK) {
            h->plan_valid = false;
            return st;
        }
    }
    if (report || inject) FT_HIP(launch_zero_u32(h->d_counters, CNT_N, stream));
    BatchArgs b{};
    b.probs = h->d_bprobs;
    b.items = h->d_bitems;
    b.n_items = h->n_items;
    b.ft_level = ft_level;
    b.tol_c = c;
    b.event_cap = h->event_cap;
    b.events = h->d_events;
    b.counters = h->d_counters;
    b.faults = inject ? h->d_faults : nullptr;
    b.n_faults = inject ? h->n_faults : 0;
    b.fault_log_cap = h->flog_cap;
    b.fault_log = h->d_flog;
    FT_HIP(launch_batched(b, inject, h->grid, h->plan_fp8, stream));
    if (!report) return FTGEMM_OK;
    return fill_report(h, stream, report);
}

int ftgemm_batched_config(ftgemm_t h, int p, ftgemm_config_t* config) {
    if (!h || !config || !h->plan_valid || p < 0 || p >= (int)h->plan_cfg.size()) return FTGEMM_INVALID;
    *config = h->plan_cfg[(size_t)p];
    return FTGEMM_OK;
}

int ftgemm_get_tuned(ftgemm_t h, ftgemm_tuned_t* out, int cap, int* n) {
    if (!h || cap < 0 || (cap > 0 && !out)) return FTGEMM_INVALID;
    const int cnt = (int)h->tuned.size();
    for (int i = 0; i < std::min(cap, cnt); ++i) out[i] = h->tuned[(size_t)i];
    if (n) *n = cnt;
    return FTGEMM_OK;
}

int ftgemm_add_tuned(ftgemm_t h, const ftgemm_tuned_t* e) {
    if (!h || !e || e->ft_level < 0 || e->ft_level > 2 || e->config.check_interval < 1 || e->config.check_m < 0 ||
        e->config.check_n < 0)
        return FTGEMM_INVALID;
    if (find_variant(h->dtype, e->config) < 0) return FTGEMM_UNSUPPORTED;
    for (ftgemm_tuned_t& t : h->tuned)
        if (t.m == e->m && t.n == e->n && t.k == e->k && t.ft_level == e->ft_level) {
            t.config = normalized(e->config);
            return FTGEMM_OK;
        }
    h->tuned.push_back(*e);
    h->tuned.back().config = normalized(e->config);
    return FTGEMM_OK;
}

int ftgemm_tune(ftgemm_t h, int64_t m, int64_t n, int64_t k, int ft_level, int max_k_between_checks,
                hipStream_t stream, ftgemm_config_t* best) {
    if (!h || ftgemm_validate(m, n, k, std::max<int64_t>(1, m), std::max<int64_t>(1, k), std::max<int64_t>(1, m),
                              ft_level, 0.f, nullptr) != FTGEMM_OK || m == 0 || n == 0 || k == 0 ||
        max_k_between_checks < 0)
        return FTGEMM_INVALID;
    if (!dtype_supported(h->dtype) || h->dtype == FTGEMM_F64 || h->dtype == FTGEMM_C64) return FTGEMM_UNSUPPORTED;
    ft_level = base_level(ft_level);   // configurations are kept per level; recompute does not change them
    const int kmax = max_k_between_checks > 0 ? max_k_between_checks : 256;
    const size_t esz = h->dtype == FTGEMM_F32 ? 4 : h->dtype == FTGEMM_BF16 ? 2 : 1;
    DeviceGuard g(h->device);
    void *A = nullptr, *B = nullptr, *C = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int st = FTGEMM_OK;
    ftgemm_config_t pick{};
    const bool was_forced = h->forced;
    const ftgemm_config_t was_cfg = h->cfg;
    if (hipMalloc(&A, esz * (size_t)m * (size_t)k) != hipSuccess || hipMalloc(&B, esz * (size_t)k * (size_t)n) != hipSuccess ||
        hipMalloc(&C, 4 * (size_t)m * (size_t)n) != hipSuccess) {
        st = FTGEMM_NO_MEMORY;
    } else if (hipMemsetAsync(A, 0, esz * (size_t)m * (size_t)k, stream) != hipSuccess ||
               hipMemsetAsync(B, 0, esz * (size_t)k * (size_t)n, stream) != hipSuccess ||
               hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        st = FTGEMM_HIP_ERROR;
    } else {
        // candidates: every variant with check intervals 1, 2, 4, ... within the
        // cap (at level 0 only the compute-tile variants: the others run the same kernel)
        std::vector<ftgemm_config_t> cand;
        const int nv = variant_count(h->dtype);
        for (int v = 0; v < nv; ++v) {
            const Variant x = variant_at(h->dtype, v);
            if (ft_level == 0 && !compute_tile_check(x)) continue;
            const int64_t nk = (k + x.k_step - 1) / x.k_step;
            for (int gi = 1;; gi *= 2) {
                if (gi > 1 && ((int64_t)gi * x.k_step > kmax || gi > nk || ft_level != 2)) break;
                cand.push_back({x.m_tile, x.n_tile, x.k_step, gi, x.check_m, x.check_n});
            }
        }
        ftgemm_config_t dflt;
        select_variant(h->dtype, m, n, ft_level, &dflt);
        if (ft_level == 2)   // the default interval may exceed the cap: clamp it like the candidates
            while (dflt.check_interval > 1 && (int64_t)dflt.check_interval * dflt.k_step > kmax) dflt.check_interval /= 2;
        auto once = [&]() {
            return ftgemm_run(h, m, n, k, 1.0f, A, std::max<int64_t>(1, m), B, std::max<int64_t>(1, k), 0.0f,
                              static_cast<float*>(C), std::max<int64_t>(1, m), ft_level, 0.f, stream, nullptr);
        };
        // interleaved rounds (so drift affects every candidate alike), median per candidate
        constexpr int kRounds = 5;
        std::vector<std::vector<float>> t(cand.size());
        for (int r = -1; r < kRounds && st == FTGEMM_OK; ++r) {
            for (size_t c = 0; c < cand.size() && st == FTGEMM_OK; ++c) {
                h->cfg = cand[c];
                h->forced = true;
                float ms = 0.f;
                if (hipEventRecord(e0, stream) != hipSuccess || once() != FTGEMM_OK ||
                    hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    st = FTGEMM_HIP_ERROR;
                    break;
                }
                if (r >= 0) t[c].push_back(ms);   // round -1 warms every candidate up
            }
        }
        if (st == FTGEMM_OK) {
            auto median = [](std::vector<float> v) {
                std::sort(v.begin(), v.end());
                return v[v.size() / 2];
            };
            int best = -1;
            float best_ms = 0.f;
            for (size_t c = 0; c < cand.size(); ++c)
                if (std::memcmp(&cand[c], &dflt, sizeof(dflt)) == 0) {
                    best = (int)c;
                    best_ms = median(t[c]);
                }
            for (size_t c = 0; c < cand.size(); ++c) {
                const float ms = median(t[c]);
                if (best < 0 || ms < 0.98f * best_ms) {   // replace the incumbent only on a clear win
                    best = (int)c;
                    best_ms = ms;
                }
            }
            pick = cand[(size_t)best];
        }
    }
    h->forced = was_forced;
    h->cfg = was_cfg;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(stream);
    if (A) (void)hipFree(A);
    if (B) (void)hipFree(B);
    if (C) (void)hipFree(C);
    if (st != FTGEMM_OK) return st;
    ftgemm_tuned_t e{m, n, k, ft_level, pick};
    ftgemm_add_tuned(h, &e);
    if (best) *best = pick;
    return FTGEMM_OK;
}

int ftgemm_tune_batched(ftgemm_t h, hipStream_t stream, double* rates) {
    if (!h) return FTGEMM_INVALID;
    DeviceGuard g(h->device);
    constexpr int kProbs = 64, kDim = 512;
    void *A = nullptr, *B = nullptr, *C = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int st = FTGEMM_OK;
    const size_t ab = 4 * (size_t)kDim * kDim, cb = 4 * (size_t)kDim * kDim;
    double measured[kBatchVariants] = {};
    const bool had_plan = h->plan_valid;
    if (hipMalloc(&A, ab * kProbs) != hipSuccess || hipMalloc(&B, ab * kProbs) != hipSuccess ||
        hipMalloc(&C, cb * kProbs) != hipSuccess) {
        st = FTGEMM_NO_MEMORY;
    } else if (hipMemsetAsync(A, 0, ab * kProbs, stream) != hipSuccess || hipMemsetAsync(B, 0, ab * kProbs, stream) != hipSuccess ||
               hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        st = FTGEMM_HIP_ERROR;
    } else {
        // each variant alone: force it by giving the model a single admissible rate
        double saved[kBatchVariants];
        for (int u = 0; u < kBatchVariants; ++u) saved[u] = h->batch_rate[u];
        for (int v = 0; v < kBatchVariants && st == FTGEMM_OK; ++v) {
            for (int u = 0; u < kBatchVariants; ++u) h->batch_rate[u] = (u == v) ? 1.0 : 1e-30;
            std::vector<ftgemm_problem_t> probs(kProbs);
            for (int p = 0; p < kProbs; ++p) {
                ftgemm_problem_t& q = probs[(size_t)p];
                std::memset(&q, 0, sizeof(q));
                q.dtype = batch_variant_dtype(v);
                q.m = q.n = q.k = kDim;
                q.lda = q.ldb = q.ldc = kDim;
                q.alpha = 1.f;
                q.beta = 0.f;
                q.scale_a = q.scale_b = 1.f;
                q.A = static_cast<char*>(A) + ab * p;
                q.B = static_cast<char*>(B) + ab * p;
                q.C = reinterpret_cast<float*>(static_cast<char*>(C) + cb * p);
            }
            h->plan_valid = false;
            if (ftgemm_batched(h, kProbs, probs.data(), 2, 0.f, stream, nullptr) != FTGEMM_OK) {
                st = FTGEMM_HIP_ERROR;
                break;
            }
            float ms = 0.f;
            const int reps = 5;
            if (hipEventRecord(e0, stream) != hipSuccess) { st = FTGEMM_HIP_ERROR; break; }
            for (int r = 0; r < reps; ++r) ftgemm_batched(h, kProbs, probs.data(), 2, 0.f, stream, nullptr);
            if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.f)) { st = FTGEMM_HIP_ERROR; break; }
            measured[v] = (double)kProbs * kDim * kDim * kDim * reps / (ms * 1e-3);
        }
        for (int u = 0; u < kBatchVariants; ++u) h->batch_rate[u] = st == FTGEMM_OK ? measured[u] : saved[u];
    }
    (void)had_plan;
    h->plan_valid = false;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(stream);
    if (A) (void)hipFree(A);
    if (B) (void)hipFree(B);
    if (C) (void)hipFree(C);
    if (st == FTGEMM_OK && rates)
        for (int u = 0; u < kBatchVariants; ++u) rates[u] = measured[u];
    return st;
}

}  // extern "C"
