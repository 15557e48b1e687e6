// ftgemm_noalloc.hip -- ftgemm_run_noalloc: ftgemm_run without a handle and
// without any allocation, for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops).
//
// The device memory a run needs besides its operands -- the counters, the
// event log and the recompute queue -- lives in one file-scope device array,
// `scratch`, of fixed size.  Each device the library runs on holds its own copy
// until the process ends; its address on a device is taken once, with that
// device current, by hipGetSymbolAddress (the array's name in host code is a
// host-side stand-in, never a device address), and only that address is
// handed to kernels and copies.  Every call on a device shares that device's
// array: the counters and the recompute queue are cleared by a kernel at the
// start of each call, and calls that overlap on one device race.
#include <cstring>
#include <mutex>

#include "ftgemm_internal.h"

namespace ftgemm_impl {
namespace {

constexpr int kNaEvents = 1024;          // event log entries
constexpr int kNaRetryTiles = 16384;     // recompute queue: output tiles of one call
constexpr int kNaMaxDevices = 64;

// Layout of the scratch array (byte offsets).
constexpr size_t kOffCounters = 0;                                        // uint32_t[CNT_N]
constexpr size_t kOffRetry = 256;                                         // uint32_t[2]
constexpr size_t kOffEvents = 512;                                        // ftgemm_event_t[kNaEvents]
constexpr size_t kOffRetryTiles = kOffEvents + sizeof(ftgemm_event_t) * kNaEvents;   // int32_t[kNaRetryTiles]
constexpr size_t kScratchBytes = kOffRetryTiles + sizeof(int32_t) * kNaRetryTiles;  // 128.5 KiB
static_assert(sizeof(uint32_t) * CNT_N <= kOffRetry - kOffCounters, "counter block");
static_assert(kOffEvents % 256 == 0 && kOffRetryTiles % 256 == 0, "256-byte aligned blocks");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
unsigned char* g_addr[kNaMaxDevices] = {};   // device address of `scratch`, per device
bool g_gfx950[kNaMaxDevices] = {};

// Set-up on the current device (once): the address of its copy of the array
// and whether it is a gfx950.  Returns FTGEMM_OK or an error status.
int device_scratch(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kNaMaxDevices) return FTGEMM_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return FTGEMM_HIP_ERROR;
        g_gfx950[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FTGEMM_HIP_ERROR;
        g_addr[dev] = static_cast<unsigned char*>(p);
    }
    if (!g_gfx950[dev]) return FTGEMM_UNSUPPORTED;
    *out = g_addr[dev];
    return FTGEMM_OK;
}

}  // namespace

}  // namespace ftgemm_impl

using namespace ftgemm_impl;

extern "C" int ftgemm_run_noalloc(int dtype, int64_t m, int64_t n, int64_t k, float alpha, const void* A,
                                  int64_t lda, const void* B, int64_t ldb, float beta, float* C, int64_t ldc,
                                  int ft_level, float tol, hipStream_t stream, ftgemm_report_t* report) {
    if (report) {
        report->checks = report->detected = report->corrected = 0;
        report->uncorrectable = report->checksum_only = report->nonfinite_input = 0;
        report->n_events = 0;
        report->bad_arg = 0;
        report->tol_used = 0.f;
        report->bad_problem = -1;
        report->recomputed = report->recompute_failed = 0;
        std::memset(&report->config, 0, sizeof(report->config));
    }
    if (dtype != FTGEMM_F32 && dtype != FTGEMM_BF16 && dtype != FTGEMM_F8E4M3) return FTGEMM_UNSUPPORTED;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return FTGEMM_HIP_ERROR;
    unsigned char* base = nullptr;
    const int st = device_scratch(dev, &base);
    if (st != FTGEMM_OK) return st;
    RunWorkspace ws{};
    ws.counters = reinterpret_cast<uint32_t*>(base + kOffCounters);
    ws.events = reinterpret_cast<ftgemm_event_t*>(base + kOffEvents);
    ws.event_cap = kNaEvents;
    ws.faults = nullptr;
    ws.n_faults = 0;
    ws.fault_log = nullptr;
    ws.fault_log_cap = 0;
    ws.retry = reinterpret_cast<uint32_t*>(base + kOffRetry);
    ws.retry_tiles = reinterpret_cast<int32_t*>(base + kOffRetryTiles);
    ws.retry_cap = kNaRetryTiles;
    // the recompute queue's two counters start at zero (the retry launch's
    // last workgroup also clears them, but an earlier call may have stopped
    // between its two launches)
    if ((ft_level & FTGEMM_FT_RECOMPUTE) && launch_zero_u32(ws.retry, 2, stream) != hipSuccess)
        return FTGEMM_HIP_ERROR;
    return run_common(nullptr, dtype, 1.0f, ws, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, ft_level, tol,
                      stream, report);
}
