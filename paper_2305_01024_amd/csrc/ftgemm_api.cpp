// ftgemm_api.cpp -- the C ABI declared in include/ftgemm.h: handle lifetime,
// argument checks, BLAS quick returns, kernel selection and launch, event log
// and fault-injection plumbing.
#include <algorithm>
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

int variant_count(int dtype) { return dtype == FTGEMM_BF16 ? bf16_variant_count() : fp32_variant_count(); }
Variant variant_at(int dtype, int v) { return dtype == FTGEMM_BF16 ? bf16_variant(v) : fp32_variant(v); }
int find_variant(int dtype, const ftgemm_config_t& c) {
    return dtype == FTGEMM_BF16 ? bf16_find_variant(c.m_tile, c.n_tile, c.k_step)
                                : fp32_find_variant(c.m_tile, c.n_tile, c.k_step);
}
bool dtype_supported(int dtype) { return dtype == FTGEMM_F32 || dtype == FTGEMM_BF16; }

// Largest compiled tile that still gives every compute unit a workgroup,
// else the smallest tile; a check every 256 k.
int select_variant(int dtype, int64_t m, int64_t n, ftgemm_config_t* out) {
    const int nv = variant_count(dtype);
    int pick = nv - 1;
    for (int v = 0; v < nv; ++v) {
        const Variant x = variant_at(dtype, v);
        const int64_t tiles = ((m + x.m_tile - 1) / x.m_tile) * ((n + x.n_tile - 1) / x.n_tile);
        if (tiles >= kNumCUs) { pick = v; break; }
    }
    const Variant x = variant_at(dtype, pick);
    out->m_tile = x.m_tile;
    out->n_tile = x.n_tile;
    out->k_step = x.k_step;
    out->check_interval = default_interval(x.k_step);
    return FTGEMM_OK;
}

}  // namespace

extern "C" {

const char* ftgemm_status_string(int s) {
    switch (s) {
        case FTGEMM_OK: return "ok";
        case FTGEMM_UNCORRECTABLE: return "uncorrectable fault pattern in at least one tile";
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
    else if (ft_level < 0 || ft_level > 2) bad = 13;
    else if (!(tol == tol) || tol > 1e30f) bad = 14;   // NaN or absurd
    if (bad_arg) *bad_arg = bad;
    return bad ? FTGEMM_INVALID : FTGEMM_OK;
}

int ftgemm_select_config(int dtype, int64_t m, int64_t n, int64_t k, int ft_level, ftgemm_config_t* config) {
    (void)k;
    (void)ft_level;
    if (!config) return FTGEMM_INVALID;
    if (!dtype_supported(dtype)) return FTGEMM_UNSUPPORTED;
    return select_variant(dtype, m, n, config);
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
        hipMalloc(&h->d_flog, sizeof(ftgemm_fault_log_t) * kFaultLogCap) != hipSuccess) {
        ftgemm_destroy(h);
        return FTGEMM_NO_MEMORY;
    }
    if (hipMemset(h->d_counters, 0, sizeof(uint32_t) * CNT_N) != hipSuccess) {
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
    if (c->check_interval < 1) return FTGEMM_INVALID;
    if (find_variant(h->dtype, *c) < 0) return FTGEMM_UNSUPPORTED;
    h->cfg = *c;
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
        if (f.kind == FTGEMM_FAULT_XOR && !(f.payload >= 0.f && f.payload <= 31.f)) return FTGEMM_INVALID;
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
    if (n) *n = applied;
    return FTGEMM_OK;
}

int ftgemm_run(ftgemm_t h, int64_t m, int64_t n, int64_t k, float alpha, const void* A, int64_t lda,
               const void* B, int64_t ldb, float beta, float* C, int64_t ldc, int ft_level, float tol,
               hipStream_t stream, ftgemm_report_t* report) {
    int32_t bad = 0;
    if (report) {
        report->checks = report->detected = report->corrected = 0;
        report->uncorrectable = report->checksum_only = 0;
        report->n_events = 0;
        report->bad_arg = 0;
        report->tol_used = 0.f;
        std::memset(&report->config, 0, sizeof(report->config));
    }
    if (!h) {
        if (report) report->bad_arg = 1;
        return FTGEMM_INVALID;
    }
    if (ftgemm_validate(m, n, k, lda, ldb, ldc, ft_level, tol, &bad) != FTGEMM_OK) {
        if (report) report->bad_arg = bad;
        return FTGEMM_INVALID;
    }
    if (!dtype_supported(h->dtype)) return FTGEMM_UNSUPPORTED;
    const float c = tol > 0.f ? tol : 2.0f;
    if (report) report->tol_used = c;
    if (m == 0 || n == 0) return FTGEMM_OK;
    if (!C) {
        if (report) report->bad_arg = 11;
        return FTGEMM_INVALID;
    }
    DeviceGuard g(h->device);
    if (k == 0 || alpha == 0.f) {
        FT_HIP(launch_scale(C, ldc, (int32_t)m, (int32_t)n, beta, stream));
        if (report) FT_HIP(hipStreamSynchronize(stream));
        return FTGEMM_OK;
    }
    if (!A || !B) {
        if (report) report->bad_arg = !A ? 6 : 8;
        return FTGEMM_INVALID;
    }

    ftgemm_config_t cfg;
    if (h->forced) cfg = h->cfg;
    else select_variant(h->dtype, m, n, &cfg);
    const int variant = find_variant(h->dtype, cfg);
    if (variant < 0) return FTGEMM_UNSUPPORTED;

    const bool inject = h->n_faults > 0;
    if (report || inject) FT_HIP(hipMemsetAsync(h->d_counters, 0, sizeof(uint32_t) * CNT_N, stream));

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
    a.scale = h->dtype == FTGEMM_F32 ? 1.0f : h->scale_a * h->scale_b;
    a.tol_c = c;
    a.check_interval = cfg.check_interval;
    a.ft_level = ft_level;
    a.problem = 0;
    a.events = h->d_events;
    a.counters = h->d_counters;
    a.event_cap = h->event_cap;
    a.faults = inject ? h->d_faults : nullptr;
    a.n_faults = inject ? h->n_faults : 0;
    a.fault_log = h->d_flog;
    a.fault_log_cap = h->flog_cap;
    if (h->dtype == FTGEMM_BF16) FT_HIP(launch_bf16(variant, inject, a, stream));
    else FT_HIP(launch_fp32(variant, inject, a, stream));

    if (!report) return FTGEMM_OK;

    FT_HIP(hipStreamSynchronize(stream));
    uint32_t cnt[CNT_N];
    FT_HIP(hipMemcpy(cnt, h->d_counters, sizeof(cnt), hipMemcpyDeviceToHost));
    const int64_t ntiles = ((m + cfg.m_tile - 1) / cfg.m_tile) * ((n + cfg.n_tile - 1) / cfg.n_tile);
    const int64_t nk = (k + cfg.k_step - 1) / cfg.k_step;
    const int64_t per_tile = ft_level == 2 ? (nk + cfg.check_interval - 1) / cfg.check_interval
                           : ft_level == 1 ? 1 : 0;
    report->checks = (uint64_t)(ntiles * per_tile);
    report->detected = cnt[CNT_DETECTED];
    report->corrected = cnt[CNT_CORRECTED];
    report->uncorrectable = cnt[CNT_UNCORRECTABLE];
    report->checksum_only = cnt[CNT_CHECKSUM_ONLY];
    report->config = cfg;
    const uint32_t logged = std::min<uint32_t>(cnt[CNT_EVENTS], (uint32_t)h->event_cap);
    const uint32_t copy = report->events ? std::min<uint32_t>(logged, report->cap_events) : 0;
    if (copy > 0)
        FT_HIP(hipMemcpy(report->events, h->d_events, sizeof(ftgemm_event_t) * copy, hipMemcpyDeviceToHost));
    report->n_events = copy;
    if (cnt[CNT_EVENTS] > copy && report->events) return FTGEMM_LOG_OVERFLOW;
    return report->uncorrectable > 0 ? FTGEMM_UNCORRECTABLE : FTGEMM_OK;
}

}  // extern "C"
