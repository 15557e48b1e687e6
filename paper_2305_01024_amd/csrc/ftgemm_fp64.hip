// ftgemm_fp64.hip -- FP64 online ABFT GEMM for gfx950 (MI355X).
//
// C = alpha * A * B + beta * C in binary64, A, B, C column-major, on the FP64
// matrix cores (v_mfma_f64_16x16x4_f64).  A workgroup of 256 threads (four
// wavefronts, a 2 x 2 grid of 64 x 64 sub-tiles, each 4 x 4 blocks of
// 16 x 16) computes a 128 x 128 tile, k-steps of 16 staged through
// double-buffered LDS, both panels k-major (A as loaded, B transposed on the
// way in), so every operand a lane supplies is one consecutive 16-lane row of
// a panel.  The MFMA computes the transposed block P^T = B^T A^T: lane l
// supplies B[k0 + l / 16][j0 + l % 16] and A[i0 + l % 16][k0 + l / 16] and
// holds P[i0 + l % 16][j0 + 4 q + l / 16] in component q (the instruction's
// lane layout, measured on the device), so a lane owns one row of C per block
// and stores along i are coalesced.  (The SIMT form of the paper, 8 x 8
// v_fma_f64 micro-tiles per thread, ran this tile at 40.2 TFLOP/s plain and
// 29.9 online at 8192^3; this form at 56.6 and 39.1.)
//
// Fault tolerance, threadblock-level (section 4.2.3), online (section 2.2,
// Eq. 4), all in FP64:
//   * encodings of each staged panel (Eq. 1-2) from the staging registers:
//       w[k] = sum_i A[i,k]: every wave holds one whole column of the A panel
//       per load slot, reduced across the wave;
//       v[k] = sum_j B[k,j]: a lane reduction per wave, then one LDS atomic
//       add per wave (three rotating slots);
//     the lane reductions use DPP moves and permlane swaps on the two
//     32-bit halves of each double (no LDS round trip);
//   * reference checksums (Eq. 3-4): threads 0..127 own rows (R_i, ||a_i||^2),
//     threads 128..255 own columns (S_j, ||b_j||^2);
//   * a check every `check_interval` k-steps and after the last: row and
//     column sums of the accumulator blocks (lane exchanges in a wave, LDS
//     across the wave grid), residuals against R and S, the threshold with
//     u = 2^-53;
//     one flagged row and one flagged column: the element at their
//     intersection is rebuilt from the row checksum (section 4.2.1, 5.3);
//     other patterns are logged and the flagged checksums re-based.
#include <hip/hip_runtime.h>

#include <cmath>

#include "ftgemm_internal.h"

namespace ftgemm_impl {
namespace {

constexpr int BM = 128, BN = 128, BK = 16, NT = 256;   // tile, k-step, threads
constexpr int LP = BM + 2;            // LDS row pitch in doubles (16-byte aligned rows, staggered banks)
constexpr double kU64 = 1.1102230246251565e-16;   // 2^-53, unit roundoff of binary64
constexpr int kMaxF64Faults = 32;

struct F64Lds {
    double As[2][BK][LP];         // A panel, k-major (i contiguous)
    double Bs[2][BK][LP];         // B panel, k-major (j contiguous)
    double wsum[2][BK];           // e^T A of the panel
    double vsum[3][BK];           // B e of the panel (added across waves, 3 rotating slots)
    double rowpart[2][BM];        // row sums per wave column
    double colpart[2][BN];        // column sums per wave row
    double excl[2];               // correction: row sum without the faulty element, per wave column
    double nsum[4];               // per-wave sums of ||a_i|| (waves 0, 1) and ||b_j|| (waves 2, 3)
    int census[4][4];             // per wave: #rows, first row, #cols, first col flagged
    double bc[5];                 // first flagged row: R, r, tau; first flagged column: r, tau
    ftgemm_fault_t fault[kMaxF64Faults];
    int fslot[kMaxF64Faults];
    int nf;
    int nonfinite;                // the tile was reported for non-finite operands
    unsigned nchecks;             // checks of this tile (added to the launch's counter at its end)
};

// Lane exchanges of a double on its two 32-bit halves.  dpp64<CTRL>: the
// value of the DPP-selected lane.  swap_sum64<BIT>: own value plus that of
// lane l ^ (1 << BIT) for BIT = 4 or 5 (v_permlane16/32_swap with both
// operands the value itself returns the own value in one result and the
// partner's in the other, so their sum is the pair's sum).
// (Only controls whose source lane is always valid are used, so the moves
// need no old value.)
template <int CTRL>
__device__ __forceinline__ double dpp64(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int BIT>
__device__ __forceinline__ double swap_sum64(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
    unsigned a0, a1, b0, b1;
    if constexpr (BIT == 4) {
        const auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        a0 = rl[0]; a1 = rl[1]; b0 = rh[0]; b1 = rh[1];
    } else {
        const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        a0 = rl[0]; a1 = rl[1]; b0 = rh[0]; b1 = rh[1];
    }
    const double d0 = __longlong_as_double((long long)(((unsigned long long)b0 << 32) | a0));
    const double d1 = __longlong_as_double((long long)(((unsigned long long)b1 << 32) | a1));
    return d0 + d1;
}
// Butterfly level on lane bit 4 or 5 of two doubles: lanes whose bit is
// clear keep `lo`, lanes whose bit is set keep `hi`, and every lane gets its
// kept value plus its partner's (lane l ^ (1 << BIT)); one swap per 32-bit
// half, as in swap_sum64.
template <int BIT>
__device__ __forceinline__ double swap_add64(double lo, double hi) {
    const unsigned long long ul = (unsigned long long)__double_as_longlong(lo);
    const unsigned long long uh = (unsigned long long)__double_as_longlong(hi);
    unsigned a0, a1, b0, b1;
    if constexpr (BIT == 4) {
        const auto rl = __builtin_amdgcn_permlane16_swap((unsigned)ul, (unsigned)uh, false, false);
        const auto rh = __builtin_amdgcn_permlane16_swap((unsigned)(ul >> 32), (unsigned)(uh >> 32), false, false);
        a0 = rl[0]; a1 = rl[1]; b0 = rh[0]; b1 = rh[1];
    } else {
        const auto rl = __builtin_amdgcn_permlane32_swap((unsigned)ul, (unsigned)uh, false, false);
        const auto rh = __builtin_amdgcn_permlane32_swap((unsigned)(ul >> 32), (unsigned)(uh >> 32), false, false);
        a0 = rl[0]; a1 = rl[1]; b0 = rh[0]; b1 = rh[1];
    }
    const double d0 = __longlong_as_double((long long)(((unsigned long long)b0 << 32) | a0));
    const double d1 = __longlong_as_double((long long)(((unsigned long long)b1 << 32) | a1));
    return d0 + d1;
}
// Sum over the 16 lanes of a row (lane bits 0..3), in every lane of it.
// Ascending levels: after bits 0 .. b-1 are summed, the partners
// quad_perm [3,2,1,0] (l ^ 3) and row_half_mirror (l ^ 7 within 8) hold the
// same value as l ^ 2 and l ^ 4.
__device__ __forceinline__ double row_sum64(double x) {
    x += dpp64<0xB1>(x);    // quad_perm [1,0,3,2]: l ^ 1
    x += dpp64<0x1B>(x);    // quad_perm [3,2,1,0]
    x += dpp64<0x141>(x);   // row_half_mirror
    return x + dpp64<0x128>(x);   // row_ror:8: l ^ 8
}
// Sum over the 64 lanes of a wave, in every lane.
__device__ __forceinline__ double wave_sum64(double x) {
    return swap_sum64<5>(swap_sum64<4>(row_sum64(x)));
}

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double flip64(double v, int bit) {
    return __longlong_as_double(__double_as_longlong(v) ^ (long long)(1ull << (bit & 63)));
}

// Per-lane indices of the thread.  lanes() passes threadIdx.x through an
// empty asm, so what the staging and the check derive from them (offsets,
// addresses) is computed where it is used rather than hoisted out of the
// k-loop, where it would hold a register, or a spill slot reloaded at every
// step, for the whole loop.
struct Lanes {
    int tid, lane, li, lg, own;
};
__device__ __forceinline__ Lanes lanes() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    Lanes L;
    L.tid = t;
    L.lane = t & 63;
    L.li = t & 15;
    L.lg = (t >> 4) & 3;
    L.own = t & (BM - 1);   // owned tile row (threads 0..127) or column (128..255)
    return L;
}

// One 128 x 128 tile (tm, tn).  FT: 0 plain, 1 detect-only, 2 online.
template <int FT, bool INJ>
__device__ void tile64(const F64Args& a, int tm, int tn, F64Lds& s) {
    // the wavefront index is uniform: scalar registers hold it and what is derived from it
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave & 1, wn = wave >> 1, li = lane & 15, lg = lane >> 4;
    const int i0 = tm * BM, j0 = tn * BN;
    const int mI = min(BM, a.M - i0), nJ = min(BN, a.N - j0);
    const int nk = (a.K + BK - 1) / BK;
    const bool row_owner = wave < BM / 64;        // threads 0..127 own rows (uniform per wave)
    const int own = tid & (BM - 1);               // owned tile row or column

    f64x4 accm[4][4];   // matrix-core blocks [bj][bi]
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) accm[bj][bi] = f64x4{0.0, 0.0, 0.0, 0.0};
    double ref = 0.0, nrm2 = 0.0;   // R_i or S_j, ||a_i||^2 or ||b_j||^2 over the k prefix

    int fnext = 0, flogged = 0;
    if constexpr (INJ) {
        if (tid == 0) s.nf = 0;
        __syncthreads();
        for (int q = tid; q < a.n_faults; q += NT) {
            const ftgemm_fault_t f = a.faults[q];
            if (f.problem == a.problem && f.tile_m == tm && f.tile_n == tn && f.row < BM && f.col < BN) {
                const int x = atomicAdd(&s.nf, 1);
                if (x < kMaxF64Faults) { s.fault[x] = f; s.fslot[x] = -1; }
            }
        }
        __syncthreads();
        if (tid == 0) {   // order by k-step
            const int n = min(s.nf, kMaxF64Faults);
            s.nf = n;
            for (int x = 1; x < n; ++x) {
                const ftgemm_fault_t f = s.fault[x];
                int y = x - 1;
                while (y >= 0 && s.fault[y].kstep > f.kstep) { s.fault[y + 1] = s.fault[y]; --y; }
                s.fault[y + 1] = f;
            }
        }
    }

    // ---- staging: each thread holds 4 pairs of A (rows 2p, 2p+1 of column k = 4 r + wave)
    // and 4 pairs of B (k = 2 (tid % 8), +1 of column j = tid / 8 + 32 r) ----
    double ra[4][2], rb[4][2];
    // Interior panels (the whole k-step inside K, the whole tile inside M or
    // N, 16-byte aligned pairs): one 16-byte buffer load per pair, with the
    // per-lane byte offset fixed for the whole k-loop, the per-step origin in
    // the scalar resource base and the per-slot offset in a scalar register,
    // so the loop carries no vector address arithmetic or bounds selects.
    const bool vecA = ((reinterpret_cast<uintptr_t>(a.A) & 15) == 0) && ((a.lda & 1) == 0) &&
                      (int64_t)BK * a.lda * 8 < (int64_t(1) << 31);
    const bool vecB = ((reinterpret_cast<uintptr_t>(a.B) & 15) == 0) && ((a.ldb & 1) == 0) &&
                      (int64_t)BN * a.ldb * 8 < (int64_t(1) << 31);
    constexpr int kRsrcWord3 = 0x00020000;   // raw 32-bit data format
    auto load = [&](int t) {
        const Lanes L = lanes();
        const int voffA = 16 * L.lane;                                      // rows 2 lane, 2 lane + 1
        const int voffB = ((L.tid / 8) * (int)a.ldb + 2 * (L.tid % 8)) * 8;  // k pair 2 (tid % 8) of column tid / 8
        const int k0 = t * BK;
        const bool fullk = k0 + BK <= a.K;
        // the edge paths take their k origin through an empty asm so that the
        // loop optimiser cannot turn their per-element pointers into
        // induction variables advanced on every step of the interior path
        int k0e = k0;
        asm volatile("" : "+s"(k0e));
        if (vecA && fullk && mI == BM) {
            const auto rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(a.A + i0 + (size_t)k0 * a.lda),
                                                              (short)0, 0x7fffffff, kRsrcWord3);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const f64x2 v = __builtin_bit_cast(
                    f64x2, __builtin_amdgcn_raw_buffer_load_b128(rs, voffA, (4 * r + wave) * (int)a.lda * 8, 0));
                ra[r][0] = v[0];
                ra[r][1] = v[1];
            }
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gk = k0e + 4 * r + wave, i = 2 * L.lane;
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const bool in = gk < a.K && i + e < mI;
                    const double* p = in ? a.A + (size_t)gk * a.lda + (i0 + i + e) : a.A;
                    const double x = *p;
                    ra[r][e] = in ? x : 0.0;
                }
            }
        }
        if (vecB && fullk && nJ == BN) {
            const auto rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(a.B + (size_t)j0 * a.ldb + k0),
                                                              (short)0, 0x7fffffff, kRsrcWord3);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const f64x2 v = __builtin_bit_cast(
                    f64x2, __builtin_amdgcn_raw_buffer_load_b128(rs, voffB, 32 * r * (int)a.ldb * 8, 0));
                rb[r][0] = v[0];
                rb[r][1] = v[1];
            }
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = L.tid / 8 + 32 * r, kk = 2 * (L.tid % 8);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const bool in = k0e + kk + e < a.K && j < nJ;
                    const double* p = in ? a.B + (size_t)(j0 + j) * a.ldb + (k0e + kk + e) : a.B;
                    const double x = *p;
                    rb[r][e] = in ? x : 0.0;
                }
            }
        }
    };
    auto store = [&](int buf, int vslot) {
        const Lanes L = lanes();
        const int lane = L.lane;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = 4 * r + wave, i = 2 * lane;
            s.As[buf][k][i] = ra[r][0];
            s.As[buf][k][i + 1] = ra[r][1];
            const int j = L.tid / 8 + 32 * r, kk = 2 * (L.tid % 8);
            s.Bs[buf][kk][j] = rb[r][0];
            s.Bs[buf][kk + 1][j] = rb[r][1];
        }
        if constexpr (FT > 0) {
            // e^T A: wave `wave` holds all 128 rows of columns 4 r + wave,
            // r = 0..3; a reduce-scatter over the wave (bit 5 halves the four
            // column sums, bit 4 halves them again, bits 0..3 finish) leaves
            // column r = 2 bit5 + bit4 in each row of 16 lanes
            double x[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) x[r] = ra[r][0] + ra[r][1];
            const double y0 = swap_add64<5>(x[0], x[2]), y1 = swap_add64<5>(x[1], x[3]);
            const double w = row_sum64(swap_add64<4>(y0, y1));
            if ((lane & 15) == 0) s.wsum[buf][4 * ((lane >> 4) & 3) + wave] = w;
            // B e: the thread's 4 columns of its k pair, then a reduce-scatter
            // over the 8 lanes of the wave with the same k pair (lane bits
            // 3..5): on bit 3 lanes with the bit clear keep k and those with
            // it set keep k + 1, each adding what its partner l ^ 8 sends;
            // bits 4 and 5 finish, and the waves add in LDS
            double v0 = rb[0][0], v1 = rb[0][1];
#pragma unroll
            for (int r = 1; r < 4; ++r) { v0 += rb[r][0]; v1 += rb[r][1]; }
            const bool upper = (lane & 8) != 0;
            const double keep = upper ? v1 : v0, send = upper ? v0 : v1;
            const double v = swap_sum64<5>(swap_sum64<4>(keep + dpp64<0x128>(send)));   // row_ror:8 = l ^ 8
            if (lane < 16) atomicAdd(&s.vsum[vslot][2 * (lane & 7) + ((lane >> 3) & 1)], v);
        }
    };

    // ---- online check after k-step t (kp = k indices accumulated) ----
    auto check = [&](int t, int kp) {
        const Lanes L = lanes();
        const int tid = L.tid, lane = L.lane, li = L.li, lg = L.lg, own = L.own;
        // row sums: a lane's 16 values of a block row, then lane bits 4, 5,
        // then the two wave columns in LDS; column sums: the four blocks
        // of a lane's column, then lane bits 0..3, then the two wave rows
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) {
            double x = accm[0][bi][0];   // (sums start from their first term: an add to 0.0 is kept for -0.0)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (bj + q > 0) x += accm[bj][bi][q];
            x = swap_sum64<5>(swap_sum64<4>(x));
            if (lg == 0) s.rowpart[wn][64 * wm + 16 * bi + li] = x;
        }
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double y = accm[bj][0][q];
#pragma unroll
                for (int bi = 1; bi < 4; ++bi) y += accm[bj][bi][q];
                y = row_sum64(y);
                if (li == 0) s.colpart[wm][64 * wn + 16 * bj + 4 * q + lg] = y;
            }
        const double nv = sqrt(nrm2);
        const double ws = wave_sum64(nv);
        if (lane == 0) s.nsum[wave] = ws;
        __syncthreads();

        const double sa = s.nsum[0] + s.nsum[1], sb = s.nsum[2] + s.nsum[3];
        // An Inf or NaN operand in the k prefix makes the norm sums (uniform
        // values) non-finite: nothing is flagged and the tile is reported once.
        const bool finite = __builtin_amdgcn_readfirstlane((__builtin_isfinite(sa) && __builtin_isfinite(sb)) ? 1 : 0) != 0;
        if (tid == 0) {
            s.nchecks += 1u;
            if (!finite && !s.nonfinite) {
                s.nonfinite = 1;
                const unsigned e = atomicAdd(&a.counters[CNT_EVENTS], 1u);
                atomicAdd(&a.counters[CNT_NONFINITE], 1u);
                if ((int)e < a.event_cap) {
                    ftgemm_event_t E;
                    E.problem = a.problem; E.tile_m = tm; E.tile_n = tn; E.kstep = t; E.row = -1; E.col = -1;
                    E.kind = FTGEMM_EV_NONFINITE; E.n_rows = 0; E.n_cols = 0; E.pad_ = 0;
                    E.value_before = E.value_after = 0.f;
                    E.r_row = E.r_col = E.tau_row = E.tau_col = 0.f;
                    a.events[e] = E;
                }
            }
        }
        const double base = (double)a.tol_c * 2.0 * kU64;
        double res = 0.0, tau = 0.0;
        bool flag = false;
        if (finite && row_owner && own < mI) {
            res = (s.rowpart[0][own] + s.rowpart[1][own]) - ref;
            tau = base * (double)(kp + nJ + 1) * nv * sb;
            flag = !(fabs(res) <= tau);
        } else if (finite && !row_owner && own < nJ) {
            res = (s.colpart[0][own] + s.colpart[1][own]) - ref;
            tau = base * (double)(kp + mI + 1) * nv * sa;
            flag = !(fabs(res) <= tau);
        }
        // owners are in index order within a wave: the first flagged line is
        // the lowest flagged lane's
        const unsigned long long b = __ballot(flag);
        if (lane == 0) {
            const int first = b ? (tid + (int)__builtin_ctzll(b)) - (row_owner ? 0 : BM) : -1;
            s.census[wave][0] = row_owner ? __popcll(b) : 0;
            s.census[wave][1] = row_owner ? first : -1;
            s.census[wave][2] = row_owner ? 0 : __popcll(b);
            s.census[wave][3] = row_owner ? -1 : first;
        }
        if constexpr (INJ) {   // complete the log entries this check is the first to see
            for (int q = flogged; q < fnext; ++q) {
                const int slot = s.fslot[q];
                if (slot < 0 || slot >= a.fault_log_cap) continue;
                if (row_owner && own == s.fault[q].row) {
                    a.fault_log[slot].r_row = (float)res; a.fault_log[slot].tau_row = (float)tau;
                }
                if (!row_owner && own == s.fault[q].col) {
                    a.fault_log[slot].r_col = (float)res; a.fault_log[slot].tau_col = (float)tau;
                }
                if (tid == 0) a.fault_log[slot].check_step = t;
            }
            flogged = fnext;
        }
        __syncthreads();
        int nr = 0, ncl = 0, fr = -1, fc = -1;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            nr += s.census[w][0];
            ncl += s.census[w][2];
            if (s.census[w][1] >= 0 && (fr < 0 || s.census[w][1] < fr)) fr = s.census[w][1];
            if (s.census[w][3] >= 0 && (fc < 0 || s.census[w][3] < fc)) fc = s.census[w][3];
        }
        if (nr + ncl == 0) return;

        // rare path (uniform branch)
        const bool online = (FT == 2) || a.ft_level == 2;
        const bool correct = online && nr == 1 && ncl == 1;
        if (row_owner && own == fr) { s.bc[0] = ref; s.bc[1] = res; s.bc[2] = tau; }
        if (!row_owner && own == fc) { s.bc[3] = res; s.bc[4] = tau; }
        __syncthreads();
        if (correct) {
            // P_ij = R_i - sum_{j' != j} P_ij'
            double oldv = 0.0, newv = 0.0;
            bool owner = false;
            // row fr: lanes li = fr % 16 of the two waves of wave row fr / 64,
            // block row (fr % 64) / 16; partials over lane bits 4, 5, then LDS
            const int fbi = (fr & 63) >> 4, fbj = (fc & 63) >> 4, fq = (fc & 15) >> 2;
            const bool in_row = wm == (fr >> 6) && li == (fr & 15);
            owner = in_row && wn == (fc >> 6) && lg == (fc & 3);
            // (per-lane selects over every element, no branches: branches on the
            // block index would make the compiler copy the accumulators)
            double part = 0.0;
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const bool mine = in_row && bi == fbi;
                        const bool hit = owner && bi == fbi && bj == fbj && q == fq;
                        part += (mine && !hit) ? accm[bj][bi][q] : 0.0;
                        oldv = hit ? accm[bj][bi][q] : oldv;
                    }
            part = swap_sum64<5>(swap_sum64<4>(part));
            if (wm == (fr >> 6) && lane == (fr & 15)) s.excl[wn] = part;
            __syncthreads();
            newv = s.bc[0] - (s.excl[0] + s.excl[1]);
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        accm[bj][bi][q] = (owner && bi == fbi && bj == fbj && q == fq) ? newv : accm[bj][bi][q];
            if (owner) {
                const unsigned e = atomicAdd(&a.counters[CNT_EVENTS], 1u);
                atomicAdd(&a.counters[CNT_DETECTED], 1u);
                atomicAdd(&a.counters[CNT_CORRECTED], 1u);
                if ((int)e < a.event_cap) {
                    ftgemm_event_t E;
                    E.problem = a.problem; E.tile_m = tm; E.tile_n = tn; E.kstep = t; E.row = fr; E.col = fc;
                    E.kind = FTGEMM_EV_CORRECTED; E.n_rows = 1; E.n_cols = 1; E.pad_ = 0;
                    E.value_before = (float)oldv; E.value_after = (float)newv;
                    E.r_row = (float)s.bc[1]; E.tau_row = (float)s.bc[2];
                    E.r_col = (float)s.bc[3]; E.tau_col = (float)s.bc[4];
                    a.events[e] = E;
                }
            }
        } else {
            const int kind = !online ? FTGEMM_EV_DETECTED
                           : (nr == 1 && ncl == 0) ? FTGEMM_EV_CHECKSUM_ROW
                           : (nr == 0 && ncl == 1) ? FTGEMM_EV_CHECKSUM_COL
                           : FTGEMM_EV_UNCORRECTABLE;
            if (online && flag) ref += res;   // re-base on the accumulator
            if (tid == 0) {
                const unsigned e = atomicAdd(&a.counters[CNT_EVENTS], 1u);
                atomicAdd(&a.counters[CNT_DETECTED], 1u);
                if (kind == FTGEMM_EV_UNCORRECTABLE) atomicAdd(&a.counters[CNT_UNCORRECTABLE], 1u);
                if (kind == FTGEMM_EV_CHECKSUM_ROW || kind == FTGEMM_EV_CHECKSUM_COL)
                    atomicAdd(&a.counters[CNT_CHECKSUM_ONLY], 1u);
                if ((int)e < a.event_cap) {
                    ftgemm_event_t E;
                    E.problem = a.problem; E.tile_m = tm; E.tile_n = tn; E.kstep = t; E.row = fr; E.col = fc;
                    E.kind = kind; E.n_rows = nr; E.n_cols = ncl; E.pad_ = 0;
                    E.value_before = E.value_after = 0.f;
                    E.r_row = fr >= 0 ? (float)s.bc[1] : 0.f; E.tau_row = fr >= 0 ? (float)s.bc[2] : 0.f;
                    E.r_col = fc >= 0 ? (float)s.bc[3] : 0.f; E.tau_col = fc >= 0 ? (float)s.bc[4] : 0.f;
                    a.events[e] = E;
                }
            }
        }
        __syncthreads();   // s.bc is rewritten by the next check
    };

    if constexpr (FT > 0) {
        if (tid < 3 * BK) (&s.vsum[0][0])[tid] = 0.0;
        if (tid == 0) { s.nonfinite = 0; s.nchecks = 0; }
        __syncthreads();
    }
    load(0);
    store(0, 0);
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
        const int cur = t & 1;
        if (t + 1 < nk) load(t + 1);
        // slot of panel t + 2: its last reader (step t - 1) finished before this step
        if (FT > 0 && t + 2 < nk && tid < BK) s.vsum[(t + 2) % 3][tid] = 0.0;
        // the product of this k-step, four k at a time on the matrix cores
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            double bf[4], af[4];
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) bf[bj] = s.Bs[cur][4 * ks + lg][64 * wn + 16 * bj + li];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) af[bi] = s.As[cur][4 * ks + lg][64 * wm + 16 * bi + li];
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
#pragma unroll
                for (int bi = 0; bi < 4; ++bi)
                    accm[bj][bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[bj], af[bi], accm[bj][bi], 0, 0, 0);
        }
        if constexpr (FT > 0) {
            // reference checksums (Eq. 4): R_i += sum_k A[i,k] (B e)[k], S_j += sum_k (e^T A)[k] B[k,j]
#pragma unroll
            for (int k = 0; k < BK; ++k) {
                const double x = row_owner ? s.As[cur][k][own] : s.Bs[cur][k][own];
                const double y = row_owner ? s.vsum[t % 3][k] : s.wsum[cur][k];
                ref = fma(x, y, ref);
                nrm2 = fma(x, x, nrm2);
            }
        }
        if (t + 1 < nk) store(cur ^ 1, (t + 1) % 3);
        if constexpr (INJ) {   // faults of k-step t hit the accumulator after its update
            while (fnext < s.nf && s.fault[fnext].kstep == t) {
                const ftgemm_fault_t f = s.fault[fnext];
                bool owner;
                double oldv = 0.0, newv = 0.0;
                const int fbi = (f.row & 63) >> 4, fbj = (f.col & 63) >> 4, fq = (f.col & 15) >> 2;
                owner = wm == (f.row >> 6) && wn == (f.col >> 6) && li == (f.row & 15) && lg == (f.col & 3);
#pragma unroll
                for (int bj = 0; bj < 4; ++bj)
#pragma unroll
                    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const bool hit = owner && bj == fbj && bi == fbi && q == fq;
                            const double x = accm[bj][bi][q];
                            const double y = f.kind == FTGEMM_FAULT_XOR ? flip64(x, (int)f.payload)
                                                                        : x + (double)f.payload;
                            oldv = hit ? x : oldv;
                            newv = hit ? y : newv;
                            accm[bj][bi][q] = hit ? y : x;
                        }
                if (owner) {
                    const int slot = (int)atomicAdd(&a.counters[CNT_FAULTS], 1u);
                    s.fslot[fnext] = slot;
                    if (slot < a.fault_log_cap) {
                        ftgemm_fault_log_t L;
                        L.problem = a.problem; L.tile_m = tm; L.tile_n = tn; L.kstep = t;
                        L.row = f.row; L.col = f.col; L.kind = f.kind; L.check_step = -1;
                        L.old_v = (float)oldv; L.new_v = (float)newv;
                        L.r_row = L.r_col = L.tau_row = L.tau_col = 0.f;
                        L.delta = newv - oldv;
                        a.fault_log[slot] = L;
                    }
                }
                ++fnext;
            }
            __syncthreads();   // s.fslot written by the owner, read by the check
        }
        if constexpr (FT > 0) {
            if (((t + 1) % a.check_interval == 0) || t == nk - 1) check(t, min((t + 1) * BK, a.K));
        }
        __syncthreads();
    }

    if (FT > 0 && tid == 0) atomicAdd(&a.counters[CNT_CHECKS], s.nchecks);   // written before the last barrier

    // epilogue: C = alpha P + beta C (beta == 0: C is not read)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 64 * wn + 16 * bj + 4 * q + lg;
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) {
                const int i = 64 * wm + 16 * bi + li;
                if (i < mI && j < nJ) {
                    double* pc = a.C + (size_t)(j0 + j) * a.ldc + (i0 + i);
                    double v = a.alpha * accm[bj][bi][q];
                    if (a.beta != 0.0) v = fma(a.beta, *pc, v);
                    *pc = v;
                }
            }
        }
}

template <int FT, bool INJ>
__global__ __launch_bounds__(NT, 2) void ftgemm_f64_kernel(F64Args a) {
    __shared__ F64Lds s;
    const int ntm = (a.M + BM - 1) / BM;
    tile64<FT, INJ>(a, blockIdx.x % ntm, blockIdx.x / ntm, s);
}

__global__ void scale64_kernel(double* C, int64_t ldc, int32_t M, int32_t N, double beta) {
    const int64_t total = (int64_t)M * N;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = x / M, i = x % M;
        double* p = C + j * ldc + i;
        *p = (beta == 0.0) ? 0.0 : beta * *p;
    }
}

constexpr Variant kVariantsF64[] = {
    {BM, BN, BK, BM, BN},
};

}  // namespace

int fp64_variant_count() { return sizeof(kVariantsF64) / sizeof(kVariantsF64[0]); }
Variant fp64_variant(int idx) { return kVariantsF64[idx]; }
int fp64_find_variant(int m_tile, int n_tile, int k_step, int check_m, int check_n) {
    for (int v = 0; v < fp64_variant_count(); ++v) {
        const Variant& x = kVariantsF64[v];
        if (x.m_tile == m_tile && x.n_tile == n_tile && x.k_step == k_step && x.check_m == check_m &&
            x.check_n == check_n)
            return v;
    }
    return -1;
}

hipError_t launch_fp64(int idx, bool inject, const F64Args& a, hipStream_t s) {
    if (idx != 0) return hipErrorInvalidValue;
    const int ntm = (a.M + BM - 1) / BM, ntn = (a.N + BN - 1) / BN;
    const dim3 grid((unsigned)(ntm * ntn)), block(NT);
#define FTGEMM_LAUNCH(FTL, INJL) hipLaunchKernelGGL((ftgemm_f64_kernel<FTL, INJL>), grid, block, 0, s, a)
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

hipError_t launch_scale64(double* C, int64_t ldc, int32_t M, int32_t N, double beta, hipStream_t s) {
    const int64_t total = (int64_t)M * N;
    const int blocks = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
    hipLaunchKernelGGL(scale64_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, C, ldc, M, N, beta);
    return hipGetLastError();
}

}  // namespace ftgemm_impl
