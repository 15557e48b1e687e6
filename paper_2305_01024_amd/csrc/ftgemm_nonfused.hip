// ftgemm_nonfused.hip -- the same threadblock-level ABFT as the fused kernels
// (256 x 256 check tiles, a check every check interval, locate at the
// row/column intersection, correct by reconstruction), but not fused: every
// step is its own launch, the way ABFT is applied around a library GEMM.
//   encode      W = e^T A per row tile, V = B e per column tile  (section 2.2 Eq. 1-2)
//   per k-chunk (one check interval):
//     GEMM      C += A[:, chunk] B[chunk, :]  (the plain FP32 kernel, FT compiled out)
//     update    R += A[:, chunk] V[chunk], S += W[chunk] B[chunk, :], prefix norms (Eq. 4)
//     check     row and column sums of C read back from memory against R and S
// It exists to measure what fusing saves (the comparisons of sections 5.2-5.4):
// the check reads C from HBM after every chunk and the chunk GEMMs re-read
// and re-write it, where the fused kernels keep the tile in registers.
#include <algorithm>

#include "ftgemm_abft.hpp"

namespace ftgemm_impl {
namespace {

using abft::ReduceScatter;
using abft::wave_sum;

constexpr int T = kNonFusedTile;

// W[tm * K + k] = sum of A[i][k] over the rows of row tile tm.
// grid (ceil(K / 4), ntm), 256 threads: wave w takes k = 4 blockIdx.x + w, lanes take rows.
__global__ void nf_encode_a(const float* A, int64_t lda, int M, int K, float* W) {
    const int lane = threadIdx.x & 63, k = blockIdx.x * 4 + (threadIdx.x >> 6), tm = blockIdx.y;
    if (k >= K) return;   // wave-uniform
    float s = 0.f;
    for (int r = lane; r < T; r += 64) {
        const int i = tm * T + r;
        if (i < M) s += A[(size_t)k * lda + i];
    }
    s = wave_sum(s);
    if (lane == 0) W[(size_t)tm * K + k] = s;
}

// V[tn * K + k] = sum of B[k][j] over the columns of column tile tn.
// grid (ceil(K / 256), ntn), 256 threads: one k per thread (coalesced along k).
__global__ void nf_encode_b(const float* B, int64_t ldb, int N, int K, float* V) {
    const int k = blockIdx.x * 256 + threadIdx.x, tn = blockIdx.y;
    if (k >= K) return;
    const int j1 = min(N, (tn + 1) * T);
    float s = 0.f;
    for (int j = tn * T; j < j1; ++j) s += B[(size_t)j * ldb + k];
    V[(size_t)tn * K + k] = s;
}

// Row references of one chunk: R[tn * M + i] += sum_k A[i][k] V[tn][k] for 32 column
// tiles per block row, and (block row 0) na2[i] += sum_k A[i][k]^2.
// grid (ceil(M / 64), ceil(ntn / 32), ksplit), 64 threads, one row per thread; the k range of
// the chunk is split over blockIdx.z and summed with atomics.
__global__ void nf_update_rows(const float* A, int64_t lda, int M, int K, int k0, int k1, int ntn,
                               const float* V, float* R, float* na2) {
    const int i = blockIdx.x * 64 + threadIdx.x, tn0 = blockIdx.y * 32;
    const int span = (k1 - k0 + gridDim.z - 1) / gridDim.z;
    const int ka = k0 + blockIdx.z * span, kb = min(k1, ka + span);
    const bool valid = i < M;
    const int nt = min(32, ntn - tn0);
    float acc[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) acc[q] = 0.f;
    float nn = 0.f;
    // eight k per iteration: the eight loads of A are in flight together
    int k = ka;
    for (; k + 8 <= kb; k += 8) {
        float x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = valid ? A[(size_t)(k + u) * lda + i] : 0.f;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            nn = fmaf(x[u], x[u], nn);
#pragma unroll
            for (int q = 0; q < 32; ++q)
                if (q < nt) acc[q] = fmaf(x[u], V[(size_t)(tn0 + q) * K + k + u], acc[q]);
        }
    }
    for (; k < kb; ++k) {
        const float x = valid ? A[(size_t)k * lda + i] : 0.f;
        nn = fmaf(x, x, nn);
#pragma unroll
        for (int q = 0; q < 32; ++q)
            if (q < nt) acc[q] = fmaf(x, V[(size_t)(tn0 + q) * K + k], acc[q]);
    }
    if (!valid) return;
#pragma unroll
    for (int q = 0; q < 32; ++q)
        if (q < nt) atomicAdd(&R[(size_t)(tn0 + q) * M + i], acc[q]);
    if (blockIdx.y == 0) atomicAdd(&na2[i], nn);
}

// Column references of one chunk: S[tm * N + j] += sum_k W[tm][k] B[k][j] and
// nb2[j] += sum_k B[k][j]^2.  One wave per column (lanes along k, coalesced), 32 row tiles
// per pass; the 32 lane partials are reduce-scattered so that lane 2q holds tile q.
// grid (N, ceil(ntm / 32)), 64 threads.
__global__ void nf_update_cols(const float* B, int64_t ldb, int N, int K, int k0, int k1, int ntm,
                               const float* W, float* S, float* nb2) {
    const int j = blockIdx.x, lane = threadIdx.x, tm0 = blockIdx.y * 32;
    const int nt = min(32, ntm - tm0);
    float acc[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) acc[q] = 0.f;
    float nn = 0.f;
    for (int k = k0 + lane; k < k1; k += 64) {
        const float x = B[(size_t)j * ldb + k];
        nn = fmaf(x, x, nn);
#pragma unroll
        for (int q = 0; q < 32; ++q)
            if (q < nt) acc[q] = fmaf(x, W[(size_t)(tm0 + q) * K + k], acc[q]);
    }
    ReduceScatter<32, 5, 0>::run(acc, lane);
    const int q = (lane >> 1) & 31;
    if ((lane & 1) == 0 && q < nt) S[(size_t)(tm0 + q) * N + j] += acc[0];
    nn = wave_sum(nn);
    if (blockIdx.y == 0 && lane == 0) nb2[j] += nn;
}

// Faults of chunk c hit C after that chunk's GEMM (the test hook of this path).
__global__ void nf_inject(float* C, int64_t ldc, int M, int N, const ftgemm_fault_t* faults, int n_faults, int c,
                          ftgemm_fault_log_t* flog, int flog_cap, uint32_t* counters) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_faults) return;
    const ftgemm_fault_t f = faults[q];
    if (f.kstep != c || f.problem != 0) return;
    const int i = f.tile_m * T + f.row, j = f.tile_n * T + f.col;
    if (i >= M || j >= N || f.row >= T || f.col >= T) return;
    float* p = C + (size_t)j * ldc + i;
    const float old = *p;
    const float nv = f.kind == FTGEMM_FAULT_XOR ? abft::bitflip(old, (int)f.payload) : old + f.payload;
    *p = nv;
    const unsigned slot = atomicAdd(&counters[CNT_FAULTS], 1u);
    if ((int)slot < flog_cap) {
        ftgemm_fault_log_t L;
        L.problem = 0; L.tile_m = f.tile_m; L.tile_n = f.tile_n; L.kstep = c; L.row = f.row; L.col = f.col;
        L.kind = f.kind; L.check_step = c; L.old_v = old; L.new_v = nv;
        L.r_row = L.r_col = L.tau_row = L.tau_col = 0.f;
        L.delta = (double)nv - (double)old;
        flog[slot] = L;
    }
}

struct CheckShared {
    float colpart[4][T];
    float nsum[2][4];
    int nr, nc, fr, fc;
    float rres, rtau, cres, ctau, rref;
    float excl[4];
};

// Check of tile (blockIdx.x % ntm, blockIdx.x / ntm) after kp k indices (chunk c):
// row sums (thread t = row t, coalesced along the column) and column sums (a wave
// reduction per column) of C against R and S with the FP32 roundoff threshold of the
// fused kernels; one row and one column flagged: C[i][j] = R_i - sum_{j' != j} C[i][j'];
// other patterns re-base the flagged checksums and are logged.  256 threads.
// A tile whose norm sums are not finite (an Inf or NaN operand in the k
// prefix) is reported once (tile_flag remembers it across chunks) and not
// decided on.
__global__ __launch_bounds__(256) void nf_check(float* C, int64_t ldc, int M, int N, int ntm, int kp, int c,
                                                float tol_c, float* R, float* S, const float* na2, const float* nb2,
                                                unsigned* tile_flag, ftgemm_event_t* events, int event_cap,
                                                uint32_t* counters) {
    __shared__ CheckShared sh;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int tm = blockIdx.x % ntm, tn = blockIdx.x / ntm;
    const int i0 = tm * T, j0 = tn * T;
    const int mI = min(T, M - i0), nJ = min(T, N - j0);
    if (t == 0) { sh.nr = sh.nc = 0; sh.fr = sh.fc = T; }
    // (1) one pass over the tile, 16 columns at a time: the row sum in each
    // thread, the 16 column sums of the wave by one reduce-scatter over its 64
    // lanes (lane l keeps column (l >> 2) & 15)
    float rs = 0.f;
    for (int jb = 0; jb < nJ; jb += 16) {
        float x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            x[u] = (t < mI && jb + u < nJ) ? C[(size_t)(j0 + jb + u) * ldc + i0 + t] : 0.f;
#pragma unroll
        for (int u = 0; u < 16; ++u) rs += x[u];
        ReduceScatter<16, 5, 0>::run(x, lane);
        const int u = (lane >> 2) & 15;
        if ((lane & 3) == 0 && jb + u < nJ) sh.colpart[w][jb + u] = x[0];
    }
    // (2) norms for the thresholds
    const float na = t < mI ? sqrtf(na2[i0 + t]) : 0.f;
    const float nb = t < nJ ? sqrtf(nb2[j0 + t]) : 0.f;
    const float wa = wave_sum(na), wb = wave_sum(nb);
    if (lane == 0) { sh.nsum[0][w] = wa; sh.nsum[1][w] = wb; }
    __syncthreads();
    const float sa = sh.nsum[0][0] + sh.nsum[0][1] + sh.nsum[0][2] + sh.nsum[0][3];
    const float sb = sh.nsum[1][0] + sh.nsum[1][1] + sh.nsum[1][2] + sh.nsum[1][3];
    if (t == 0) atomicAdd(&counters[CNT_CHECKS], 1u);
    if (!(__builtin_isfinite(sa) && __builtin_isfinite(sb))) {
        if (t == 0 && tile_flag[blockIdx.x] == 0u) {
            tile_flag[blockIdx.x] = 1u;
            const unsigned e = atomicAdd(&counters[CNT_EVENTS], 1u);
            atomicAdd(&counters[CNT_NONFINITE], 1u);
            if ((int)e < event_cap) {
                ftgemm_event_t E;
                E.problem = 0; E.tile_m = tm; E.tile_n = tn; E.kstep = c; E.row = -1; E.col = -1;
                E.kind = FTGEMM_EV_NONFINITE; E.n_rows = 0; E.n_cols = 0; E.pad_ = 0;
                E.value_before = E.value_after = 0.f;
                E.r_row = E.r_col = E.tau_row = E.tau_col = 0.f;
                events[e] = E;
            }
        }
        return;
    }
    const float base = tol_c * 2.0f * abft::kUnitRoundoff;
    bool rf = false, cf = false;
    float rres = 0.f, rtau = 0.f, cres = 0.f, ctau = 0.f, rref = 0.f;
    float* rp = &R[(size_t)tn * M + i0 + t];
    float* sp = &S[(size_t)tm * N + j0 + t];
    if (t < mI) {
        rref = *rp;
        rres = rs - rref;
        rtau = base * (float)(kp + nJ + 1) * na * sb;
        rf = !(fabsf(rres) <= rtau);
    }
    float csum = 0.f;
    if (t < nJ) {
        csum = sh.colpart[0][t] + sh.colpart[1][t] + sh.colpart[2][t] + sh.colpart[3][t];
        cres = csum - *sp;
        ctau = base * (float)(kp + mI + 1) * nb * sa;
        cf = !(fabsf(cres) <= ctau);
    }
    if (rf) { atomicAdd(&sh.nr, 1); atomicMin(&sh.fr, t); }
    if (cf) { atomicAdd(&sh.nc, 1); atomicMin(&sh.fc, t); }
    __syncthreads();
    const int nr = sh.nr, nc = sh.nc, fr = sh.fr, fc = sh.fc;
    if (nr + nc == 0) return;
    if (rf && t == fr) { sh.rres = rres; sh.rtau = rtau; sh.rref = rref; }
    if (cf && t == fc) { sh.cres = cres; sh.ctau = ctau; }
    __syncthreads();
    if (nr == 1 && nc == 1) {
        // sum of row fr without element fc, then rebuild the element from the row checksum
        float part = 0.f;
        for (int jj = t; jj < nJ; jj += 256)
            if (jj != fc) part += C[(size_t)(j0 + jj) * ldc + i0 + fr];
        part = wave_sum(part);
        if (lane == 0) sh.excl[w] = part;
        __syncthreads();
        if (t == 0) {
            const float excl = sh.excl[0] + sh.excl[1] + sh.excl[2] + sh.excl[3];
            float* p = C + (size_t)(j0 + fc) * ldc + i0 + fr;
            const float oldv = *p, newv = sh.rref - excl;
            *p = newv;
            const unsigned e = atomicAdd(&counters[CNT_EVENTS], 1u);
            atomicAdd(&counters[CNT_DETECTED], 1u);
            atomicAdd(&counters[CNT_CORRECTED], 1u);
            if ((int)e < event_cap) {
                ftgemm_event_t E;
                E.problem = 0; E.tile_m = tm; E.tile_n = tn; E.kstep = c; E.row = fr; E.col = fc;
                E.kind = FTGEMM_EV_CORRECTED; E.n_rows = 1; E.n_cols = 1; E.pad_ = 0;
                E.value_before = oldv; E.value_after = newv;
                E.r_row = sh.rres; E.r_col = sh.cres; E.tau_row = sh.rtau; E.tau_col = sh.ctau;
                events[e] = E;
            }
        }
        return;
    }
    // re-base the flagged checksums on C and log the pattern
    if (rf) *rp = rs;
    if (cf) *sp = csum;
    if (t == 0) {
        const int kind = (nr == 1 && nc == 0) ? FTGEMM_EV_CHECKSUM_ROW
                       : (nr == 0 && nc == 1) ? FTGEMM_EV_CHECKSUM_COL : FTGEMM_EV_UNCORRECTABLE;
        const unsigned e = atomicAdd(&counters[CNT_EVENTS], 1u);
        atomicAdd(&counters[CNT_DETECTED], 1u);
        if (kind == FTGEMM_EV_UNCORRECTABLE) atomicAdd(&counters[CNT_UNCORRECTABLE], 1u);
        else atomicAdd(&counters[CNT_CHECKSUM_ONLY], 1u);
        if ((int)e < event_cap) {
            ftgemm_event_t E;
            E.problem = 0; E.tile_m = tm; E.tile_n = tn; E.kstep = c;
            E.row = nr ? fr : -1; E.col = nc ? fc : -1; E.kind = kind; E.n_rows = nr; E.n_cols = nc; E.pad_ = 0;
            E.value_before = E.value_after = 0.f;
            E.r_row = nr ? sh.rres : 0.f; E.tau_row = nr ? sh.rtau : 0.f;
            E.r_col = nc ? sh.cres : 0.f; E.tau_col = nc ? sh.ctau : 0.f;
            events[e] = E;
        }
    }
}

}  // namespace

hipError_t launch_nonfused_encode(const NonFusedArgs& n, hipStream_t s) {
    const int ntm = (n.M + T - 1) / T, ntn = (n.N + T - 1) / T;
    hipLaunchKernelGGL(nf_encode_a, dim3((unsigned)((n.K + 3) / 4), (unsigned)ntm), dim3(256), 0, s,
                       n.A, n.lda, n.M, n.K, n.W);
    hipLaunchKernelGGL(nf_encode_b, dim3((unsigned)((n.K + 255) / 256), (unsigned)ntn), dim3(256), 0, s,
                       n.B, n.ldb, n.N, n.K, n.V);
    return hipGetLastError();
}

hipError_t launch_nonfused_chunk(const NonFusedArgs& n, int c, int k0, int k1, hipStream_t s) {
    const int ntm = (n.M + T - 1) / T, ntn = (n.N + T - 1) / T;
    const int ksplit = std::max(1, std::min(8, 1024 / std::max(1, ((n.M + 63) / 64) * ((ntn + 31) / 32))));
    hipLaunchKernelGGL(nf_update_rows, dim3((unsigned)((n.M + 63) / 64), (unsigned)((ntn + 31) / 32), (unsigned)ksplit),
                       dim3(64), 0, s, n.A, n.lda, n.M, n.K, k0, k1, ntn, n.V, n.R, n.na2);
    hipLaunchKernelGGL(nf_update_cols, dim3((unsigned)n.N, (unsigned)((ntm + 31) / 32)), dim3(64), 0, s,
                       n.B, n.ldb, n.N, n.K, k0, k1, ntm, n.W, n.S, n.nb2);
    if (n.n_faults > 0)
        hipLaunchKernelGGL(nf_inject, dim3((unsigned)((n.n_faults + 255) / 256)), dim3(256), 0, s, n.C, n.ldc, n.M,
                           n.N, n.faults, n.n_faults, c, n.fault_log, n.fault_log_cap, n.counters);
    hipLaunchKernelGGL(nf_check, dim3((unsigned)(ntm * ntn)), dim3(256), 0, s, n.C, n.ldc, n.M, n.N, ntm, k1, c,
                       n.tol_c, n.R, n.S, n.na2, n.nb2, n.tile_flag, n.events, n.event_cap, n.counters);
    return hipGetLastError();
}

}  // namespace ftgemm_impl
