// ftgemm_abft.hpp -- device code shared by every FT-GEMM kernel variant of
// the library: lane-exchange helpers, the per-thread tile geometry, the online
// check with locate/correct (section 2.2 Eq. 4, section 4.2.1, section 5.3),
// the compile-time fault-injection hook and the epilogue.
//
// All of it works on the FP32 accumulator of 32 x 32 MFMA blocks, which has
// the same lane layout for the FP32, BF16 and FP8 MFMA instructions: lane l
// holds column (l % 32) of a block and rows 8 (r / 4) + 4 (l / 32) + (r % 4)
// in register r.  The kernels compute the transposed tile P^T = B^T A^T, so a
// block's "column" is a row i of C and its "rows" are columns j of C.
#pragma once

#include <type_traits>

#include "ftgemm_internal.h"

namespace ftgemm_impl {
namespace abft {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr float kUnitRoundoff = 5.9604644775390625e-08f;  // 2^-24, binary32

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// ---------------------------------------------------------------------------
// lane exchanges (wave64)
// ---------------------------------------------------------------------------
// Partner value for the exchange level on lane bit BIT < 4, with DPP (no LDS
// round trip).  With EXACT the partner is lane l ^ (1 << BIT): quad_perm
// [1,0,3,2], quad_perm [2,3,0,1], row_shl:4 / row_shr:4 by lane, row_ror:8.
// Without it, levels 1 and 2 use quad_perm [3,2,1,0] (l ^ 3) and
// row_half_mirror (l ^ 7 within 8), one instruction each; that is valid only
// when the reduction continues down to lane bit 0: a butterfly needs the
// partner's bit BIT to differ and its higher bits to agree, and the lower
// bits are summed over later.  A reduction that stops above bit 0 keeps the
// lower bits as separate groups and needs the exact partner.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}

template <int BIT, bool EXACT>
__device__ __forceinline__ float partner(float x, int lane) {
    static_assert(BIT >= 0 && BIT < 4, "levels 4 and 5 use swap_add");
    if constexpr (BIT == 0) return dpp_mov<0xB1>(x);                        // quad_perm [1,0,3,2]
    else if constexpr (BIT == 1) return EXACT ? dpp_mov<0x4E>(x)            // quad_perm [2,3,0,1]
                                              : dpp_mov<0x1B>(x);           // quad_perm [3,2,1,0]
    else if constexpr (BIT == 2) {
        if constexpr (!EXACT) return dpp_mov<0x141>(x);                     // row_half_mirror
        const float up = dpp_mov<0x104>(x);                                 // row_shl:4: lane i + 4
        const float dn = dpp_mov<0x114>(x);                                 // row_shr:4: lane i - 4
        return (lane & 4) ? dn : up;
    } else return dpp_mov<0x128>(x);                                        // row_ror:8
}

// Butterfly level on lane bit 4 or 5 without LDS.  v_permlane16_swap_b32
// exchanges the odd 16-lane rows of its first register with the even rows of
// its second; v_permlane32_swap_b32 the upper 32 lanes of the first with the
// lower 32 of the second.  With lo = the value lanes whose bit is clear keep
// and hi = the value lanes whose bit is set keep, the two results add up, in
// every lane, to its kept value plus its partner's (lane l ^ 16 or l ^ 32).
template <int BIT>
__device__ __forceinline__ float swap_add(float lo, float hi) {
    static_assert(BIT == 4 || BIT == 5, "swap levels");
    const unsigned a = __builtin_bit_cast(unsigned, lo), b = __builtin_bit_cast(unsigned, hi);
    if constexpr (BIT == 4) {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        return __builtin_bit_cast(float, (unsigned)r[0]) + __builtin_bit_cast(float, (unsigned)r[1]);
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        return __builtin_bit_cast(float, (unsigned)r[0]) + __builtin_bit_cast(float, (unsigned)r[1]);
    }
}

// Reduce-scatter of N values over the lanes that differ only in lane bits
// BIT, BIT-1, ..., BLO.  The first log2(N) levels halve the value count, the
// rest reduce the single survivor.  Afterwards x[0] of lane l holds the sum,
// over all those lanes, of original entry sum_b bit_b(l) * (N_b / 2), where
// N_b is the count entering the halving level on bit b (for N = 1: the plain
// sum).  Example: N = 16 over bits 4..0 leaves entry (l >> 1) & 15.
template <int N, int BIT, int BLO = 0>
struct ReduceScatter {
    __device__ __forceinline__ static void run(float* x, int lane) {
        if constexpr (BIT >= BLO && BIT >= 0) {
            if constexpr (BIT >= 4) {
                if constexpr (N > 1) {
#pragma unroll
                    for (int q = 0; q < N / 2; ++q) x[q] = swap_add<BIT>(x[q], x[q + N / 2]);
                    ReduceScatter<N / 2, BIT - 1, BLO>::run(x, lane);
                } else {
                    x[0] = swap_add<BIT>(x[0], x[0]);
                    ReduceScatter<1, BIT - 1, BLO>::run(x, lane);
                }
            } else if constexpr (N > 1) {
                const bool up = ((lane >> BIT) & 1) != 0;
#pragma unroll
                for (int q = 0; q < N / 2; ++q) {
                    const float send = up ? x[q] : x[q + N / 2];
                    const float keep = up ? x[q + N / 2] : x[q];
                    x[q] = keep + partner<BIT, (BLO > 0)>(send, lane);
                }
                ReduceScatter<N / 2, BIT - 1, BLO>::run(x, lane);
            } else {
                x[0] += partner<BIT, (BLO > 0)>(x[0], lane);
                ReduceScatter<1, BIT - 1, BLO>::run(x, lane);
            }
        }
    }
};

// Sum over the 64 lanes of a wave, returned as a wave-uniform value.
__device__ __forceinline__ float wave_sum(float x) {
    float v[1] = {x};
    ReduceScatter<1, 5, 0>::run(v, 0);
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v[0])));
}

__device__ __forceinline__ float bitflip(float v, int bit) {
    return __uint_as_float(__float_as_uint(v) ^ (1u << (bit & 31)));
}

// ---------------------------------------------------------------------------
// tile geometry and per-thread roles
// ---------------------------------------------------------------------------
// A workgroup of WM x WN wavefronts computes one BM x BN tile (the check
// tile); wavefront (wm, wn) holds the TM x TN sub-tile as MI x NI blocks.
// Checksum owners: thread t < BM owns tile row t; the column owners are the
// next BN threads when there are at least BM + BN threads (SPLIT), else
// thread t < BN.  With SPLIT the role is wave-uniform.
template <int BM_, int BN_, int WM_, int WN_>
struct Geometry {
    static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_;
    static constexpr int NT = 64 * WM * WN, NW = WM * WN;
    static constexpr int TM = BM / WM, TN = BN / WN;
    static constexpr int MI = TM / 32, NI = TN / 32;
    static constexpr bool SPLIT = NT >= BM + BN;
    static constexpr int COL0 = SPLIT ? BM : 0;
    static_assert(MI >= 1 && NI >= 1, "each wavefront needs at least one 32 x 32 block");
    static_assert(!SPLIT || BM % 64 == 0, "row owners must fill whole wavefronts");
};

struct Thread {
    int tid, lane, wave, wm, wn, l32, hh;
    bool row_role;
    int my_row, my_col;     // owned tile row / column, -1 if none
    int tm, tn, i0, j0, mI, nJ;
};

// UNIFORM: the wavefront index and what derives from it are computed as
// wave-uniform values, so scalar registers hold them (the FT kernels, whose
// vector registers are full; the plain kernels schedule better without it).
template <class G, bool UNIFORM = false>
__device__ __forceinline__ Thread make_thread(const LaunchArgs& a, int tm, int tn) {
    Thread t;
    t.tid = threadIdx.x;
    t.lane = t.tid & 63;
    const int wave_u = __builtin_amdgcn_readfirstlane(t.tid >> 6);
    t.wave = UNIFORM ? wave_u : t.tid >> 6;
    t.wm = t.wave % G::WM;
    t.wn = t.wave / G::WM;
    t.l32 = t.lane & 31;
    t.hh = t.lane >> 5;
    t.row_role = !G::SPLIT || wave_u < G::BM / 64;
    t.my_row = (t.row_role && t.tid < G::BM) ? t.tid : -1;
    t.my_col = G::SPLIT ? ((!t.row_role && t.tid < G::COL0 + G::BN) ? t.tid - G::COL0 : -1)
                        : (t.tid < G::BN ? t.tid : -1);
    t.tm = tm;
    t.tn = tn;
    t.i0 = tm * G::BM;
    t.j0 = tn * G::BN;
    t.mI = min(G::BM, a.M - t.i0);
    t.nJ = min(G::BN, a.N - t.j0);
    return t;
}

// LDS scratch of the check and the injection hook
template <class G>
struct CheckLds {
    float rowpart[G::WN][G::BM];    // row sums per wave column
    float colpart[G::WM][G::BN];    // column sums per wave row
    float nsum[2][G::NW];           // per-wave sums of ||a_i|| and of ||b_j||
    int census[G::NW][4];           // per-wave (#rows, first row, #cols, first col)
    float excl[G::WN];              // correction: row sum without the faulty element
    float bc[8];                    // broadcast scratch
    float dummy[64];                // sink for stores of lanes that own no value
    ftgemm_fault_t fault[kMaxFaultsPerTile];
    int fslot[kMaxFaultsPerTile];
    int nf;
    int tainted;            // a check left the tile possibly wrong (cleared at tile start)
    int nonfinite;          // check tiles already reported for non-finite operands, one bit
                            // per check tile (bit 0: the compute tile; cleared at tile start)
    unsigned nchecks;       // checks of this tile so far (cleared at tile start); added to the
                            // launch's counter once, at the end of the tile, so that the loop
                            // carries no global atomic whose completion a later wait would see
    int nflagged;           // wavefronts that flagged a line at the current check (0 between checks)
};

// Clears the tile's check state; before the tile's first barrier.  Census
// entries rest at (0 rows, no first row, 0 columns, no first column).
template <class G>
__device__ __forceinline__ void clear_check(CheckLds<G>& s, int tid) {
    if (tid == 0) {
        s.tainted = 0;
        s.nonfinite = 0;
        s.nchecks = 0;
        s.nflagged = 0;
    }
    if (tid < G::NW) {
        s.census[tid][0] = 0;
        s.census[tid][1] = -1;
        s.census[tid][2] = 0;
        s.census[tid][3] = -1;
    }
}

// Extra LDS of the wavefront-tile check: per wave, the flag census of each
// check tile it holds owners for, and the checksum values of each check
// tile's first flagged row and column.
template <class G>
struct WaveCheckLds : CheckLds<G> {
    static constexpr int NR = G::WM > G::WN ? G::WM : G::WN;
    int wcen[G::NW][NR][2];     // (#flagged, first flagged index) per wave and check tile
    int wany[G::NW];            // the wave flagged anything
    float bw[G::NW][5];         // per check tile: R, r_row, tau_row, r_col, tau_col
    int tdec[G::NW][4];         // per check tile: #rows, #columns flagged, first row, first column
};

template <class G>
using Acc = f32x16[G::MI][G::NI];

// ---------------------------------------------------------------------------
// fault injection hook (compiled only into INJ kernels)
// ---------------------------------------------------------------------------
// Collect this tile's fault sites into LDS, ordered by (kstep, row, col).
// With WAVE the sites address wavefront check tiles: those of this compute
// tile are kept with row/col converted to the compute tile (sites outside
// their check tile are dropped) and tile_m/tile_n left as given.
template <class G, bool WAVE = false>
__device__ void gather_faults(CheckLds<G>& s, const LaunchArgs& a, const Thread& th) {
    if (th.tid == 0) s.nf = 0;
    __syncthreads();
    for (int q = th.tid; q < a.n_faults; q += G::NT) {
        ftgemm_fault_t f = a.faults[q];
        bool mine = f.problem == a.problem;
        if constexpr (WAVE) {
            mine = mine && f.tile_m / G::WM == th.tm && f.tile_n / G::WN == th.tn && f.row < G::TM && f.col < G::TN;
            f.row += (f.tile_m % G::WM) * G::TM;
            f.col += (f.tile_n % G::WN) * G::TN;
        } else {
            mine = mine && f.tile_m == th.tm && f.tile_n == th.tn;
        }
        if (mine) {
            const int x = atomicAdd(&s.nf, 1);
            if (x < kMaxFaultsPerTile) { s.fault[x] = f; s.fslot[x] = -1; }
        }
    }
    __syncthreads();
    if (th.tid == 0) {
        const int n = min(s.nf, kMaxFaultsPerTile);
        s.nf = n;
        for (int x = 1; x < n; ++x) {
            const ftgemm_fault_t f = s.fault[x];
            int y = x - 1;
            while (y >= 0 && (s.fault[y].kstep > f.kstep ||
                              (s.fault[y].kstep == f.kstep && (s.fault[y].row > f.row ||
                               (s.fault[y].row == f.row && s.fault[y].col > f.col))))) {
                s.fault[y + 1] = s.fault[y];
                --y;
            }
            s.fault[y + 1] = f;
        }
    }
}

// Faults of k-step t hit the accumulator (after that step's update): the
// element is found with uniform block branches and per-lane selects.
template <class G, bool WAVE = false>
__device__ __forceinline__ void inject(Acc<G>& acc, CheckLds<G>& s, const LaunchArgs& a, const Thread& th,
                                       int t, int& fnext) {
    while (fnext < s.nf && s.fault[fnext].kstep == t) {
        const ftgemm_fault_t f = s.fault[fnext];
        const int ir = f.row % G::TM, jr = f.col % G::TN;
        const int fbi = ir / 32, fbj = jr / 32, jj = jr % 32;
        const int freg = ((jj >> 3) << 2) | (jj & 3);
        const bool own = f.row / G::TM == th.wm && f.col / G::TN == th.wn &&
                         th.lane == ((jj >> 2) & 1) * 32 + (ir % 32);
        float oldv = 0.f, newv = 0.f;
#pragma unroll
        for (int bi = 0; bi < G::MI; ++bi)
#pragma unroll
            for (int bj = 0; bj < G::NI; ++bj) {
                if (bi == fbi && bj == fbj) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float x = acc[bi][bj][r];
                        const bool hit = own && r == freg;
                        const float y = (f.kind == FTGEMM_FAULT_XOR) ? bitflip(x, (int)f.payload) : x + f.payload;
                        oldv = hit ? x : oldv;
                        newv = hit ? y : newv;
                        acc[bi][bj][r] = hit ? y : x;
                    }
                }
            }
        if (own) {
            const int slot = (int)atomicAdd(&a.counters[CNT_FAULTS], 1u);
            s.fslot[fnext] = slot;
            if (slot < a.fault_log_cap) {
                ftgemm_fault_log_t L;
                L.problem = a.problem; L.tile_m = th.tm; L.tile_n = th.tn; L.kstep = t;
                L.row = f.row; L.col = f.col; L.kind = f.kind; L.check_step = -1;
                if constexpr (WAVE) {   // back to check-tile coordinates
                    L.tile_m = f.tile_m; L.tile_n = f.tile_n;
                    L.row = f.row % G::TM; L.col = f.col % G::TN;
                }
                L.old_v = oldv; L.new_v = newv;
                L.r_row = L.r_col = L.tau_row = L.tau_col = 0.f;
                L.delta = (double)newv - (double)oldv;
                a.fault_log[slot] = L;
            }
        }
        ++fnext;
    }
}

// ---------------------------------------------------------------------------
// online check (section 2.2: compare sums with the checksums against a
// threshold; section 4.2.1: locate at the row/column intersection and
// correct from the checksum)
// ---------------------------------------------------------------------------
// kp = number of k indices accumulated so far.  Rr/na2 are the owner's row
// checksum and ||a||^2, Sc/nb2 the column ones (the same variables may alias
// under SPLIT, where a thread owns only one of them).  Ends with a workgroup
// barrier after the census (callers use it as the end-of-step barrier).
// A check that leaves the tile possibly wrong (any flag at the detect-only
// level, an uncorrectable pattern at the online level) sets s.tainted.
// One pass over the accumulator, one 32-column block at a time: per-lane
// partial row sums (over the lane's columns) and the block's column sums over
// this wave's rows; the 16 column sums of a lane are reduce-scattered over the
// 32 lanes of its half, leaving lane pair (2x, 2x+1) with entry x.  Leaves
// s.rowpart[wn][i] = sum of row i over wave column wn's columns and
// s.colpart[wm][j] = sum of column j over wave row wm's rows (no barrier).
template <class G>
__device__ __forceinline__ void tile_sums(const Acc<G>& acc, CheckLds<G>& s, const Thread& th) {
    constexpr int MI = G::MI, NI = G::NI, TM = G::TM, TN = G::TN;
    const int lane = th.lane, l32 = th.l32, hh = th.hh, wm = th.wm, wn = th.wn;
    // (every sum starts from its first term: an add to 0.0 is not an exact
    // no-op for -0.0, so the compiler would keep it)
    float rpart[MI];
#pragma unroll
    for (int bj = 0; bj < NI; ++bj) {
        float cs[16];
#pragma unroll
        for (int bi = 0; bi < MI; ++bi) {
            float rs = 0.f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float x = acc[bi][bj][r];
                cs[r] = bi == 0 ? x : cs[r] + x;
                rs = r == 0 ? x : rs + x;
            }
            rpart[bi] = bj == 0 ? rs : rpart[bi] + rs;
        }
        ReduceScatter<16, 4, 0>::run(cs, lane);
        if ((l32 & 1) == 0) {
            const int r = l32 >> 1;
            s.colpart[wm][wn * TN + 32 * bj + 8 * (r >> 2) + 4 * hh + (r & 3)] = cs[0];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int bi = 0; bi < MI; ++bi) {
        const float rs = swap_add<5>(rpart[bi], rpart[bi]);
        if (hh == 0) s.rowpart[wn][wm * TM + 32 * bi + l32] = rs;
    }
}

// Event of a check tile whose operands hold Inf or NaN (its norm sums are not
// finite, so are its bound and references): logged once per check tile, by one
// thread, at the first check that sees it; nothing is located or corrected.
__device__ __forceinline__ void log_nonfinite(const LaunchArgs& a, int tile_m, int tile_n, int t) {
    const unsigned e = atomicAdd(&a.counters[CNT_EVENTS], 1u);
    atomicAdd(&a.counters[CNT_NONFINITE], 1u);
    if ((int)e < a.event_cap) {
        ftgemm_event_t E;
        E.problem = a.problem; E.tile_m = tile_m; E.tile_n = tile_n; E.kstep = t;
        E.row = -1; E.col = -1; E.kind = FTGEMM_EV_NONFINITE; E.n_rows = 0; E.n_cols = 0; E.pad_ = 0;
        E.value_before = E.value_after = 0.f;
        E.r_row = E.r_col = E.tau_row = E.tau_col = 0.f;
        a.events[e] = E;
    }
}

// threadIdx.x through an empty asm: per-lane offsets and addresses a k-step
// derives from it are then computed inside the step instead of being hoisted
// out of the k-loop, where they would hold registers (or spill slots,
// reloaded at every step) for the whole loop.
__device__ __forceinline__ int opaque_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// The per-lane indices, passed through an empty asm at the start of a check:
// the addresses the check derives from them are then computed inside it
// rather than hoisted out of the k-loop, where they would hold registers (or
// spill slots, reloaded at every check) for the whole loop.
__device__ __forceinline__ Thread opaque_lanes(const Thread& th) {
    Thread t = th;
    asm volatile("" : "+v"(t.tid), "+v"(t.lane), "+v"(t.l32), "+v"(t.hh), "+v"(t.my_row), "+v"(t.my_col));
    return t;
}

template <class G, int FT, bool INJ>
__device__ __forceinline__ void check(Acc<G>& acc, CheckLds<G>& s, const LaunchArgs& a, const Thread& th_loop, int t, int kp,
                                      float& Rr, float& na2, float& Sc, float& nb2, int fnext, int& flogged) {
    constexpr int MI = G::MI, NI = G::NI, TM = G::TM, TN = G::TN, WM = G::WM, WN = G::WN, NW = G::NW;
    const Thread th = opaque_lanes(th_loop);
    const int lane = th.lane, l32 = th.l32, hh = th.hh, wm = th.wm, wn = th.wn;

    // (1) row sums per wave column and column sums per wave row
    tile_sums<G>(acc, s, th);
    // (2) per-wave sums of the row and column norms for the threshold
    const float na = (th.my_row >= 0) ? sqrtf(na2) : 0.f;
    const float nb = (th.my_col >= 0) ? sqrtf(nb2) : 0.f;
    const float wna = wave_sum(na), wnb = wave_sum(nb);
    if (lane == 0) { s.nsum[0][th.wave] = wna; s.nsum[1][th.wave] = wnb; }
    __syncthreads();

    // (3) residuals, thresholds (the analytic FP32 roundoff bound), flags
    float sa = s.nsum[0][0], sb = s.nsum[1][0];
#pragma unroll
    for (int w = 1; w < NW; ++w) { sa += s.nsum[0][w]; sb += s.nsum[1][w]; }
    // An Inf or NaN operand in the k prefix makes the norm sums (uniform
    // values) non-finite: nothing is flagged and the tile is reported once.
    const bool finite = __builtin_amdgcn_readfirstlane((__builtin_isfinite(sa) && __builtin_isfinite(sb)) ? 1 : 0) != 0;
    // uniform: kept in a scalar register
    const float base = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(
                                                     __builtin_bit_cast(int, a.tol_c * 2.0f * kUnitRoundoff)));
    float rres = 0.f, cres = 0.f, taur = 0.f, tauc = 0.f;
    bool rf = false, cf = false;
    if (finite && th.my_row >= 0 && th.my_row < th.mI) {
        float x = s.rowpart[0][th.my_row];
#pragma unroll
        for (int w = 1; w < WN; ++w) x += s.rowpart[w][th.my_row];
        rres = x - Rr;
        taur = base * (float)(kp + th.nJ + 1) * na * sb;
        rf = !(fabsf(rres) <= taur);
    }
    if (finite && th.my_col >= 0 && th.my_col < th.nJ) {
        float x = s.colpart[0][th.my_col];
#pragma unroll
        for (int w = 1; w < WM; ++w) x += s.colpart[w][th.my_col];
        cres = x - Sc;
        tauc = base * (float)(kp + th.mI + 1) * nb * sa;
        cf = !(fabsf(cres) <= tauc);
    }
    // per wave: how many rows / columns are flagged and the smallest flagged
    // index (owners need not be in index order; the loops run only when
    // something is flagged)
    const unsigned long long rb = __ballot(rf), cb = __ballot(cf);
    int fr_w = -1, fc_w = -1;
    for (unsigned long long m = rb; m; m &= m - 1) {
        const int r = __builtin_amdgcn_readlane(th.my_row, __ffsll((long long)m) - 1);
        fr_w = (fr_w < 0 || r < fr_w) ? r : fr_w;
    }
    for (unsigned long long m = cb; m; m &= m - 1) {
        const int c = __builtin_amdgcn_readlane(th.my_col, __ffsll((long long)m) - 1);
        fc_w = (fc_w < 0 || c < fc_w) ? c : fc_w;
    }
    // Only a wavefront with a flag writes its census entry (the others keep
    // the cleared one) and counts itself in s.nflagged, so the common path
    // reads one word after the barrier.
    const bool wave_flagged = (rb | cb) != 0ull;
    if (lane == 0 && wave_flagged) {
        s.census[th.wave][0] = __popcll(rb);
        s.census[th.wave][1] = fr_w;
        s.census[th.wave][2] = __popcll(cb);
        s.census[th.wave][3] = fc_w;
        atomicAdd(&s.nflagged, 1);
    }
    if (th.tid == 0) {
        s.nchecks += 1u;
        if (!finite && !(s.nonfinite & 1)) {
            s.nonfinite |= 1;
            log_nonfinite(a, th.tm, th.tn, t);
        }
    }
    if constexpr (INJ) {   // complete the fault log entries this check is the first to see
        for (int q = flogged; q < fnext; ++q) {
            const int slot = s.fslot[q];
            if (slot < 0 || slot >= a.fault_log_cap) continue;
            if (th.my_row == s.fault[q].row) { a.fault_log[slot].r_row = rres; a.fault_log[slot].tau_row = taur; }
            if (th.my_col == s.fault[q].col) { a.fault_log[slot].r_col = cres; a.fault_log[slot].tau_col = tauc; }
            if (th.tid == 0) a.fault_log[slot].check_step = t;
        }
        flogged = fnext;
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s.nflagged) == 0) return;

    // rare path: something was flagged (uniform branch)
    int nr = 0, ncl = 0, fr = -1, fc = -1;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        nr += s.census[w][0];
        ncl += s.census[w][2];
        const int r = s.census[w][1], c = s.census[w][3];
        if (r >= 0 && (fr < 0 || r < fr)) fr = r;
        if (c >= 0 && (fc < 0 || c < fc)) fc = c;
    }

    // online level: compile-time in the FT = 2 kernels; the FT = 1 (detect-only)
    // kernels take it from the arguments, so that their code matches the
    // online kernels' and the compiler schedules their loops alike
    const bool online = (FT == 2) || a.ft_level == 2;
    const bool correct = online && nr == 1 && ncl == 1;
    if (th.my_row >= 0 && th.my_row == fr) { s.bc[0] = Rr; s.bc[1] = rres; s.bc[2] = taur; }
    if (th.my_col >= 0 && th.my_col == fc) { s.bc[3] = cres; s.bc[4] = tauc; }
    // Coordinates of (fr, fc) in the accumulator layout; all but the lane
    // tests are uniform, so the block is picked by scalar branches and the
    // element by per-lane selects.
    const int fbi = correct ? (fr % TM) / 32 : -1;
    const int fjr = correct ? fc % TN : 0;
    const int fbj = fjr / 32, fjj = fjr % 32;
    const int freg = ((fjj >> 3) << 2) | (fjj & 3);
    const bool row_lane = correct && wm == fr / TM && l32 == (fr & 31);
    const bool own = row_lane && wn == fc / TN && hh == ((fjj >> 2) & 1);
    float oldv = 0.f;
    if (correct && wm == fr / TM) {
        // sum of row fr over this wave's columns, without element (fr, fc)
        float part = 0.f;
#pragma unroll
        for (int bi = 0; bi < MI; ++bi) {
            if (bi == fbi) {
#pragma unroll
                for (int bj = 0; bj < NI; ++bj)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float x = acc[bi][bj][r];
                        const bool hit = own && bj == fbj && r == freg;
                        part += hit ? 0.f : x;
                        oldv = hit ? x : oldv;
                    }
            }
        }
        part = row_lane ? part : 0.f;
        part = swap_add<5>(part, part);
        float* dst = (lane == (fr & 31)) ? &s.excl[wn] : &s.dummy[lane];
        *dst = part;
    }
    __syncthreads();
    // every thread has read the census: back to the cleared state for the
    // next check (whose writes come after at least one more barrier)
    if (lane == 0 && wave_flagged) {
        s.census[th.wave][0] = 0;
        s.census[th.wave][1] = -1;
        s.census[th.wave][2] = 0;
        s.census[th.wave][3] = -1;
    }
    if (th.tid == 0) s.nflagged = 0;
    if (correct) {
        // P_ij = R_i - sum_{j' != j} P_ij'
        float excl = 0.f;
#pragma unroll
        for (int w = 0; w < WN; ++w) excl += s.excl[w];
        const float newv = s.bc[0] - excl;
#pragma unroll
        for (int bi = 0; bi < MI; ++bi)
#pragma unroll
            for (int bj = 0; bj < NI; ++bj) {
                if (bi == fbi && bj == fbj) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[bi][bj][r] = (own && r == freg) ? newv : acc[bi][bj][r];
                }
            }
        if (own) {
            const unsigned e = atomicAdd(&a.counters[CNT_EVENTS], 1u);
            atomicAdd(&a.counters[CNT_DETECTED], 1u);
            atomicAdd(&a.counters[CNT_CORRECTED], 1u);
            if ((int)e < a.event_cap) {
                ftgemm_event_t E;
                E.problem = a.problem; E.tile_m = th.tm; E.tile_n = th.tn; E.kstep = t;
                E.row = fr; E.col = fc; E.kind = FTGEMM_EV_CORRECTED; E.n_rows = 1; E.n_cols = 1;
                E.pad_ = 0; E.value_before = oldv; E.value_after = newv;
                E.r_row = s.bc[1]; E.r_col = s.bc[3]; E.tau_row = s.bc[2]; E.tau_col = s.bc[4];
                a.events[e] = E;
            }
        }
    } else {
        int kind;
        if (!online) kind = FTGEMM_EV_DETECTED;
        else kind = (nr == 1 && ncl == 0) ? FTGEMM_EV_CHECKSUM_ROW
                  : (nr == 0 && ncl == 1) ? FTGEMM_EV_CHECKSUM_COL
                  : FTGEMM_EV_UNCORRECTABLE;
        if (online) {   // re-base the flagged checksums on the accumulator
            if (rf) Rr += rres;
            if (cf) Sc += cres;
        }
        if (th.tid == 0) {
            const unsigned e = atomicAdd(&a.counters[CNT_EVENTS], 1u);
            atomicAdd(&a.counters[CNT_DETECTED], 1u);
            if (kind == FTGEMM_EV_UNCORRECTABLE) atomicAdd(&a.counters[CNT_UNCORRECTABLE], 1u);
            if (kind == FTGEMM_EV_CHECKSUM_ROW || kind == FTGEMM_EV_CHECKSUM_COL)
                atomicAdd(&a.counters[CNT_CHECKSUM_ONLY], 1u);
            if ((int)e < a.event_cap) {
                ftgemm_event_t E;
                E.problem = a.problem; E.tile_m = th.tm; E.tile_n = th.tn; E.kstep = t;
                E.row = fr; E.col = fc; E.kind = kind; E.n_rows = nr; E.n_cols = ncl; E.pad_ = 0;
                E.value_before = E.value_after = 0.f;
                E.r_row = fr >= 0 ? s.bc[1] : 0.f; E.tau_row = fr >= 0 ? s.bc[2] : 0.f;
                E.r_col = fc >= 0 ? s.bc[3] : 0.f; E.tau_col = fc >= 0 ? s.bc[4] : 0.f;
                a.events[e] = E;
            }
        }
        if (th.tid == 0 && (kind == FTGEMM_EV_DETECTED || kind == FTGEMM_EV_UNCORRECTABLE)) s.tainted = 1;
    }
}

// ---------------------------------------------------------------------------
// wavefront-tile check (warp-level ABFT, section 4.2.2): every wavefront's
// TM x TN sub-tile is a check tile with its own encodings and reference
// checksums, so one fault per wavefront tile and check interval is corrected
// ---------------------------------------------------------------------------
// Decision, correction and event of wave (wm, wn)'s own check tile (some
// row or column flagged; census values in compute-tile coordinates).
template <class G, int FT>
__device__ __forceinline__ void own_tile_outcome(Acc<G>& acc, WaveCheckLds<G>& s, const LaunchArgs& a,
                                                 const Thread& th, int t, int nr, int ncl, int fr, int fc) {
    constexpr int MI = G::MI, NI = G::NI, TM = G::TM, TN = G::TN, WM = G::WM, WN = G::WN;
    const int lane = th.lane, l32 = th.l32, hh = th.hh, wm = th.wm, wn = th.wn;
    const bool online = (FT == 2) || a.ft_level == 2;
    const float* b = s.bw[wm + WM * wn];
    auto event = [&](int kind) {
        ftgemm_event_t E;
        E.problem = a.problem; E.tile_m = th.tm * WM + wm; E.tile_n = th.tn * WN + wn; E.kstep = t;
        E.row = fr >= 0 ? fr - wm * TM : -1; E.col = fc >= 0 ? fc - wn * TN : -1;
        E.kind = kind; E.n_rows = nr; E.n_cols = ncl; E.pad_ = 0;
        E.value_before = E.value_after = 0.f;
        E.r_row = fr >= 0 ? b[1] : 0.f; E.tau_row = fr >= 0 ? b[2] : 0.f;
        E.r_col = fc >= 0 ? b[3] : 0.f; E.tau_col = fc >= 0 ? b[4] : 0.f;
        return E;
    };
    if (online && nr == 1 && ncl == 1) {
        // P_ij = R_i - sum_{j' != j} P_ij' within the wave tile
        const int fbi = (fr % TM) / 32, fjr = fc % TN;
        const int fbj = fjr / 32, fjj = fjr % 32;
        const int freg = ((fjj >> 3) << 2) | (fjj & 3);
        const bool row_lane = l32 == (fr & 31);
        const bool own = row_lane && hh == ((fjj >> 2) & 1);
        float part = 0.f, oldv = 0.f;
#pragma unroll
        for (int bi = 0; bi < MI; ++bi) {
            if (bi == fbi) {
#pragma unroll
                for (int bj = 0; bj < NI; ++bj)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float x = acc[bi][bj][r];
                        const bool hit = own && bj == fbj && r == freg;
                        part += hit ? 0.f : x;
                        oldv = hit ? x : oldv;
                    }
            }
        }
        part = row_lane ? part : 0.f;
        part = swap_add<5>(part, part);
        const float newv = b[0] - part;
#pragma unroll
        for (int bi = 0; bi < MI; ++bi)
#pragma unroll
            for (int bj = 0; bj < NI; ++bj) {
                if (bi == fbi && bj == fbj) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[bi][bj][r] = (own && r == freg) ? newv : acc[bi][bj][r];
                }
            }
        if (own) {
            const unsigned e = atomicAdd(&a.counters[CNT_EVENTS], 1u);
            atomicAdd(&a.counters[CNT_DETECTED], 1u);
            atomicAdd(&a.counters[CNT_CORRECTED], 1u);
            if ((int)e < a.event_cap) {
                ftgemm_event_t E = event(FTGEMM_EV_CORRECTED);
                E.value_before = oldv; E.value_after = newv;
                a.events[e] = E;
            }
        }
    } else {
        const int kind = !online ? FTGEMM_EV_DETECTED
                       : (nr == 1 && ncl == 0) ? FTGEMM_EV_CHECKSUM_ROW
                       : (nr == 0 && ncl == 1) ? FTGEMM_EV_CHECKSUM_COL
                       : FTGEMM_EV_UNCORRECTABLE;
        if (lane == 0) {
            const unsigned e = atomicAdd(&a.counters[CNT_EVENTS], 1u);
            atomicAdd(&a.counters[CNT_DETECTED], 1u);
            if (kind == FTGEMM_EV_UNCORRECTABLE) atomicAdd(&a.counters[CNT_UNCORRECTABLE], 1u);
            if (kind == FTGEMM_EV_CHECKSUM_ROW || kind == FTGEMM_EV_CHECKSUM_COL)
                atomicAdd(&a.counters[CNT_CHECKSUM_ONLY], 1u);
            if ((int)e < a.event_cap) a.events[e] = event(kind);
            if (kind == FTGEMM_EV_DETECTED || kind == FTGEMM_EV_UNCORRECTABLE) s.tainted = 1;
        }
    }
}

// Owner geometry SPLIT: the row owner of tile row i keeps ref[q] = R_i of
// wave column q (q < WN), the column owner of tile column j keeps ref[q] =
// S_j of wave row q (q < WM); nrm2 is the owner's ||a_i||^2 or ||b_j||^2.
// Decisions, re-basing and events are per check tile, with the event's
// tile_m/tile_n counting check tiles of C and row/col relative to it.  Ends
// with a workgroup barrier.
template <class G, int FT, bool INJ, int NR>
__device__ void check_wave(Acc<G>& acc, WaveCheckLds<G>& s, const LaunchArgs& a, const Thread& th, int t, int kp,
                           float (&ref)[NR], float nrm2, int fnext, int& flogged) {
    constexpr int TM = G::TM, TN = G::TN, WM = G::WM, WN = G::WN, NW = G::NW;
    constexpr int RW = G::BM / 64;                  // waves 0 .. RW-1 own rows, the others columns
    constexpr int WPM = TM / 64, WPN = TN / 64;     // owner waves per wave row / wave column
    static_assert(G::SPLIT && TM % 64 == 0 && TN % 64 == 0 && NR == WaveCheckLds<G>::NR, "wavefront check geometry");
    const int lane = th.lane, wm = th.wm, wn = th.wn, wave = th.wave;
    const bool row_role = th.row_role;
    const int cnt = row_role ? WN : WM;             // check tiles the owner's line crosses

    // (1) sums over each wave tile, (2) per-wave norm sums
    tile_sums<G>(acc, s, th);
    const bool owner = th.my_row >= 0 || th.my_col >= 0;
    const float nv = owner ? sqrtf(nrm2) : 0.f;
    const float wnv = wave_sum(nv);
    if (lane == 0) s.nsum[0][wave] = wnv;
    __syncthreads();

    // (3) residual and threshold against crossed check tile q; recomputed
    // from LDS where needed again (the sums stay valid until the next check),
    // so only the flag bits stay in registers
    const float base = a.tol_c * 2.0f * kUnitRoundoff;
    const int mine = row_role ? th.my_row : th.my_col;
    const int line_tile = row_role ? mine / TM : mine / TN;   // own wave row / column index of the owner's line
    const bool in_range = row_role ? (th.my_row >= 0 && th.my_row < th.mI) : (th.my_col >= 0 && th.my_col < th.nJ);
    // Check tile (r, c) whose row or column norm sums are not finite (an Inf
    // or NaN operand in the k prefix): reported once, not decided on.
    auto finite_tile = [&](int r, int c) -> bool {
        float x = 0.f, y = 0.f;
#pragma unroll
        for (int w = 0; w < WPM; ++w) x += s.nsum[0][r * WPM + w];
#pragma unroll
        for (int w = 0; w < WPN; ++w) y += s.nsum[0][RW + c * WPN + w];
        return __builtin_isfinite(x) && __builtin_isfinite(y);
    };
    auto residual = [&](int q, float& res, float& tau) -> bool {
        const int ext = row_role ? th.nJ - q * TN : th.mI - q * TM;   // valid extent of the crossed tile
        if (!(q < cnt && in_range && ext > 0)) { res = tau = 0.f; return false; }
        if (!(row_role ? finite_tile(line_tile, q) : finite_tile(q, line_tile))) { res = tau = 0.f; return false; }
        float other_r = 0.f, other_c = 0.f;   // sums of the other side's norms over the crossed tile
#pragma unroll
        for (int w = 0; w < WPN; ++w) other_r += s.nsum[0][RW + q * WPN + w];
#pragma unroll
        for (int w = 0; w < WPM; ++w) other_c += s.nsum[0][q * WPM + w];
        const float other = row_role ? other_r : other_c;
        const float x = row_role ? s.rowpart[q][mine] : s.colpart[q][mine];
        res = x - ref[q];
        tau = base * (float)(kp + min(ext, row_role ? TN : TM) + 1) * nv * other;
        return !(fabsf(res) <= tau);
    };
    unsigned flags = 0;
    bool any = false;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        float res, tau;
        const bool f = residual(q, res, tau);
        flags |= f ? (1u << q) : 0u;
        // owners are in index order within a wave (one line per thread,
        // tid order): the first flagged line is the lowest flagged lane's
        const unsigned long long b = __ballot(f);
        const int first = b ? __builtin_amdgcn_readlane(mine, (int)__builtin_ctzll(b)) : -1;
        any = any || b != 0;
        if (lane == 0) { s.wcen[wave][q][0] = __popcll(b); s.wcen[wave][q][1] = first; }
    }
    if (lane == 0) s.wany[wave] = any ? 1 : 0;
    // the wave's own check tile (wm, wn), if it holds part of C: counted, and
    // reported once if its operands are not finite
    if (lane == 0 && wm * TM < th.mI && wn * TN < th.nJ) {
        atomicAdd(&s.nchecks, 1u);
        if (!finite_tile(wm, wn) && !(s.nonfinite & (1 << wave))) {
            atomicOr(&s.nonfinite, 1 << wave);
            log_nonfinite(a, th.tm * WM + wm, th.tn * WN + wn, t);
        }
    }
    if constexpr (INJ) {   // complete the fault log entries this check is the first to see
        for (int q = flogged; q < fnext; ++q) {
            const int slot = s.fslot[q];
            if (slot < 0 || slot >= a.fault_log_cap) continue;
            const int fr_ = s.fault[q].row, fc_ = s.fault[q].col;
            const bool mine_f = row_role ? th.my_row == fr_ : th.my_col == fc_;
            if (mine_f) {
                float rq = 0.f, tq = 0.f;
                (void)residual(row_role ? fc_ / TN : fr_ / TM, rq, tq);
                if (row_role) { a.fault_log[slot].r_row = rq; a.fault_log[slot].tau_row = tq; }
                else { a.fault_log[slot].r_col = rq; a.fault_log[slot].tau_col = tq; }
            }
            if (th.tid == 0) a.fault_log[slot].check_step = t;
        }
        flogged = fnext;
    }
    __syncthreads();

    int nany = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) nany += s.wany[w];
    if (nany == 0) return;

    // rare path (uniform branch): each wave takes the census of its own
    // check tile and publishes it
    int nr = 0, ncl = 0, fr = -1, fc = -1;
    for (int w = 0; w < WPM; ++w) {
        const int* e = s.wcen[wm * WPM + w][wn];
        nr += e[0];
        if (e[1] >= 0 && (fr < 0 || e[1] < fr)) fr = e[1];
    }
    for (int w = 0; w < WPN; ++w) {
        const int* e = s.wcen[RW + wn * WPN + w][wm];
        ncl += e[0];
        if (e[1] >= 0 && (fc < 0 || e[1] < fc)) fc = e[1];
    }
    if (lane == 0) { s.tdec[wave][0] = nr; s.tdec[wave][1] = ncl; s.tdec[wave][2] = fr; s.tdec[wave][3] = fc; }
    __syncthreads();
    // the owners of each check tile's first flagged row and column publish
    // their values; flagged checksums of tiles that are not corrected are
    // re-based on the accumulator (online level)
    const bool online = (FT == 2) || a.ft_level == 2;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        if (flags & (1u << q)) {
            float res, tau;
            (void)residual(q, res, tau);
            const int ct = row_role ? line_tile + WM * q : q + WM * line_tile;
            const int* d = s.tdec[ct];
            float* b = s.bw[ct];
            if (row_role && mine == d[2]) { b[0] = ref[q]; b[1] = res; b[2] = tau; }
            if (!row_role && mine == d[3]) { b[3] = res; b[4] = tau; }
            if (online && !(d[0] == 1 && d[1] == 1)) ref[q] += res;
        }
    }
    __syncthreads();
    if (nr + ncl > 0) own_tile_outcome<G, FT>(acc, s, a, th, t, nr, ncl, fr, fc);
    __syncthreads();   // s.tainted is read by every wave at the end of the tile
}

// ---------------------------------------------------------------------------
// recompute of tainted tiles
// ---------------------------------------------------------------------------
// Body of a retry launch: workgroup w recomputes queued tiles w, w + grid,
// ...; `tile_fn(tm, tn)` runs one tile.  The last workgroup to finish clears
// the queue for the next call, so the pair of launches needs no memset.
template <class TileFn>
__device__ __forceinline__ void retry_queue(const LaunchArgs& a, int ntm, TileFn&& tile_fn) {
    const unsigned count = a.retry[0];
    for (unsigned q = blockIdx.x; q < count; q += gridDim.x) {
        const int t = a.retry_tiles[q];
        tile_fn(t % ntm, t / ntm);
        __syncthreads();   // the next tile reuses the LDS
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&a.retry[1], 1u) == gridDim.x - 1) {
            atomicExch(&a.retry[0], 0u);
            atomicExch(&a.retry[1], 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// epilogue: C = alpha * scale * P + beta * C (beta == 0: C is not read)
// ---------------------------------------------------------------------------
template <class G>
__device__ __forceinline__ void epilogue(const Acc<G>& acc, const LaunchArgs& a, const Thread& th, float scale);

// End of a tile.  A tainted tile of a launch with recompute on is queued for
// the retry launch and leaves C untouched (so beta * C is still available);
// every other tile runs the epilogue.  In the retry launch every tile is
// written and counted, a tainted one also as failed.
template <class G, int FT>
__device__ __forceinline__ void finish_tile(const Acc<G>& acc, const CheckLds<G>& s, const LaunchArgs& a,
                                            const Thread& th, float scale) {
    const bool tainted = FT > 0 && s.tainted != 0;   // written before the last check's final barrier
    if (FT > 0 && th.tid == 0) atomicAdd(&a.counters[CNT_CHECKS], s.nchecks);   // ditto
    if (tainted && a.retry_tiles && !a.retry_pass) {
        if (th.tid == 0) {
            const int ntm = (a.M + G::BM - 1) / G::BM;
            const unsigned q = atomicAdd(&a.retry[0], 1u);
            a.retry_tiles[q] = th.tm + ntm * th.tn;
        }
        return;
    }
    if (a.retry_pass && th.tid == 0) {
        atomicAdd(&a.counters[CNT_RECOMPUTED], 1u);
        if (tainted) atomicAdd(&a.counters[CNT_RECOMPUTE_FAILED], 1u);
    }
    epilogue<G>(acc, a, th, scale);
}
template <class G>
__device__ __forceinline__ void epilogue(const Acc<G>& acc, const LaunchArgs& a, const Thread& th, float scale) {
    const float alpha = a.alpha * scale;
#pragma unroll
    for (int bi = 0; bi < G::MI; ++bi) {
        const int i = th.wm * G::TM + 32 * bi + th.l32;
#pragma unroll
        for (int bj = 0; bj < G::NI; ++bj)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = th.wn * G::TN + 32 * bj + 8 * (r >> 2) + 4 * th.hh + (r & 3);
                if (i < th.mI && j < th.nJ) {
                    float* pc = a.C + (size_t)(th.j0 + j) * a.ldc + (th.i0 + i);
                    float v = alpha * acc[bi][bj][r];
                    if (a.beta != 0.0f) v = fmaf(a.beta, *pc, v);
                    *pc = v;
                }
            }
    }
}

}  // namespace abft
}  // namespace ftgemm_impl
