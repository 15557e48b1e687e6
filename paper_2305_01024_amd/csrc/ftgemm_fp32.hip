// ftgemm_fp32.hip -- FP32 online ABFT GEMM kernels for gfx950 (MI355X).
//
// One workgroup (WM x WN wavefronts) computes one BM x BN output tile, which
// is also the check tile.  The k-loop runs in steps of BK with A/B panels
// double-buffered in LDS; the product runs on v_mfma_f32_32x32x2_f32.
//
// Fault tolerance (threadblock-level ABFT of section 4.2.3, in the online
// outer-product form of section 2.2, Eq. 4):
//   * encode (Eq. 1-2), fused with the global->LDS staging of each panel:
//       w[k] = sum_{i in tile} A[i,k]   (e^T A)
//       v[k] = sum_{j in tile} B[k,j]   (B e)
//     computed from the registers the panel was loaded into, reduced across
//     lanes, no extra global reads;
//   * reference checksums updated every k-step (Eq. 3 carried through Eq. 4):
//       R_i += sum_k A[i,k] v[k]   (row checksums, C e)
//       S_j += sum_k w[k] B[k,j]   (column checksums, e^T C)
//     plus ||a_i||^2 and ||b_j||^2 over the k prefix for the threshold;
//   * check every `check_interval` k-steps and after the last: row and column
//     sums of the accumulator (cross-lane butterflies inside a wave, LDS across
//     waves), residuals against R and S, NaN-safe compare with the threshold;
//   * one flagged row and one flagged column: the element at their
//     intersection is rebuilt from the row checksum,
//     P_ij = R_i - sum_{j' != j} P_ij'   (section 4.2.1, section 5.3);
//     other patterns are logged and the flagged checksums re-based.
//
// MFMA orientation: the instruction computes the transposed tile
// P^T = B^T A^T, so each lane owns one row i of C (lane % 32) and 16 columns
// per 32 x 32 block.  Stores to column-major C are then coalesced along i.
// The k index of the two lane halves is permuted (lane half h takes k = 8g +
// 4h + s in MFMA s of group g) so the B operand is one 16-byte LDS read per
// four MFMAs.
#include <type_traits>

#include "ftgemm_internal.h"

namespace ftgemm_impl {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr float kUnitRoundoff = 5.9604644775390625e-08f;  // 2^-24, binary32

template <int BM, int BN, int BK, int WM, int WN>
struct Smem {
    static constexpr int NW = WM * WN;
    float As[2][BK][BM];        // A panel, k-major (i contiguous)
    float Bs[2][BN][BK + 4];    // B panel, j-major (k contiguous), padded: conflict-free 16 B reads
    float wsum[2][BK];          // e^T A of the panel, per k
    float vsum[3][BK];          // B e of the panel, per k (accumulated across waves, 3 rotating slots)
    float dummy[256];           // sink for the stores/atomics of lanes that own no value
    float rowpart[WN][BM];      // check: row sums per wave column
    float colpart[WM][BN];      // check: column sums per wave row
    float nsum[2][NW];          // check: per-wave sums of ||a_i|| and of ||b_j||
    int census[NW][4];          // check: per-wave (#rows, first row, #cols, first col)
    float excl[WN];             // correction: row sum without the faulty element
    float bc[8];                // broadcast scratch
    ftgemm_fault_t fault[kMaxFaultsPerTile];
    int fslot[kMaxFaultsPerTile];
    int nf;
};

// ---------------------------------------------------------------------------
// cross-lane helpers (wave64)
// ---------------------------------------------------------------------------
// Partner value for the exchange level on lane bit BIT.  Levels 0-3 stay
// inside a 16-lane row and use DPP (no LDS round trip): quad_perm [1,0,3,2]
// (partner l^1), quad_perm [3,2,1,0] (l^3), row_half_mirror (l^7 within 8)
// and row_ror:8 (l^8); level 4 is an LDS swizzle (l^16), level 5 a
// permute (l^32).  Each pairs lane l with a lane whose bit BIT differs and
// whose higher bits agree, which is all a butterfly reduction needs: the
// sets of lanes summed into each value stay disjoint and end up complete.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}

template <int BIT>
__device__ __forceinline__ float partner(float x) {
    if constexpr (BIT == 0) return dpp_mov<0xB1>(x);        // quad_perm [1,0,3,2]
    else if constexpr (BIT == 1) return dpp_mov<0x1B>(x);   // quad_perm [3,2,1,0]
    else if constexpr (BIT == 2) return dpp_mov<0x141>(x);  // row_half_mirror
    else if constexpr (BIT == 3) return dpp_mov<0x128>(x);  // row_ror:8
    else if constexpr (BIT == 4)                            // swizzle: swap 16-lane halves of 32
        return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, x), 0x401F));
    else return __shfl_xor(x, 32);
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
            if constexpr (N > 1) {
                const bool up = ((lane >> BIT) & 1) != 0;
#pragma unroll
                for (int q = 0; q < N / 2; ++q) {
                    const float send = up ? x[q] : x[q + N / 2];
                    const float keep = up ? x[q + N / 2] : x[q];
                    x[q] = keep + partner<BIT>(send);
                }
                ReduceScatter<N / 2, BIT - 1, BLO>::run(x, lane);
            } else {
                x[0] += partner<BIT>(x[0]);
                ReduceScatter<1, BIT - 1, BLO>::run(x, lane);
            }
        }
    }
};

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// Sum over the 64 lanes of a wave, returned as a wave-uniform value.
__device__ __forceinline__ float wave_sum(float x) {
    float v[1] = {x};
    ReduceScatter<1, 4, 0>::run(v, 0);
    const int lo = __builtin_amdgcn_readlane(__builtin_bit_cast(int, v[0]), 0);
    const int hi = __builtin_amdgcn_readlane(__builtin_bit_cast(int, v[0]), 32);
    return __builtin_bit_cast(float, lo) + __builtin_bit_cast(float, hi);
}

__device__ __forceinline__ float bitflip(float v, int bit) {
    return __uint_as_float(__float_as_uint(v) ^ (1u << (bit & 31)));
}

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------
template <int BM, int BN, int BK, int WM, int WN, int FT, bool INJ>
__global__ __launch_bounds__(64 * WM * WN) void ftgemm_f32_kernel(LaunchArgs a) {
    constexpr int NT = 64 * WM * WN;           // threads
    constexpr int NW = WM * WN;                // wavefronts
    constexpr int TM = BM / WM, TN = BN / WN;  // wave tile
    constexpr int MI = TM / 32, NI = TN / 32;  // 32 x 32 MFMA blocks per wave
    constexpr int NA = BM * BK / (4 * NT);     // float4 slots of A per thread
    constexpr int NB = BN * BK / (4 * NT);     // float4 slots of B per thread
    constexpr int AG = (BM / 4 < 64) ? BM / 4 : 64;   // lanes sharing one k in the A load
    constexpr int BKQ = BK / 4;                       // lanes sharing one column in the B load
    // Checksum owners: thread t < BM owns tile row t; the column owners are the
    // next BN threads when there are enough threads, else thread t < BN.
    constexpr bool SPLIT = NT >= BM + BN;
    constexpr int COL0 = SPLIT ? BM : 0;
    static_assert(MI >= 1 && NI >= 1 && NA >= 1 && NB >= 1 && BK % 8 == 0, "tile shape");
    static_assert(NT % (BM / 4) == 0 || (BM / 4) % 64 == 0, "A slot mapping");
    static_assert(NT % BKQ == 0 && 64 % BKQ == 0 && BKQ <= 16, "B slot mapping");
    static_assert(NA <= AG, "encode reduce-scatter needs NA <= AG");

    __shared__ Smem<BM, BN, BK, WM, WN> sm;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int l32 = lane & 31, hh = lane >> 5;
    // with SPLIT the first BM/64 wavefronts own rows and the next BN/64 own
    // columns, so the role is wave-uniform (kept in scalar registers)
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);
    const bool row_role = !SPLIT || wave_u < BM / 64;
    const int my_row = (row_role && tid < BM) ? tid : -1;
    const int my_col = SPLIT ? ((!row_role && tid < COL0 + BN) ? tid - COL0 : -1) : (tid < BN ? tid : -1);

    const int ntm = (a.M + BM - 1) / BM;
    const int tm = blockIdx.x % ntm, tn = blockIdx.x / ntm;
    const int i0 = tm * BM, j0 = tn * BN;
    const int mI = min(BM, a.M - i0), nJ = min(BN, a.N - j0);
    const int nk = (a.K + BK - 1) / BK;

    const bool alignA = ((reinterpret_cast<uintptr_t>(a.A) & 15) == 0) && ((a.lda & 3) == 0);
    const bool alignB = ((reinterpret_cast<uintptr_t>(a.B) & 15) == 0) && ((a.ldb & 3) == 0);

    if constexpr (FT > 0) {
        for (int x = tid; x < 3 * BK; x += NT) (&sm.vsum[0][0])[x] = 0.f;
    }

    // ---- injection hook: gather this tile's fault sites ----
    int fnext = 0, flogged = 0;
    if constexpr (INJ) {
        if (tid == 0) sm.nf = 0;
        __syncthreads();
        for (int q = tid; q < a.n_faults; q += NT) {
            const ftgemm_fault_t f = a.faults[q];
            if (f.problem == a.problem && f.tile_m == tm && f.tile_n == tn) {
                const int s = atomicAdd(&sm.nf, 1);
                if (s < kMaxFaultsPerTile) { sm.fault[s] = f; sm.fslot[s] = -1; }
            }
        }
        __syncthreads();
        if (tid == 0) {   // order by (kstep, row, col): deterministic application
            const int n = min(sm.nf, kMaxFaultsPerTile);
            sm.nf = n;
            for (int x = 1; x < n; ++x) {
                const ftgemm_fault_t f = sm.fault[x];
                int y = x - 1;
                while (y >= 0 && (sm.fault[y].kstep > f.kstep ||
                                  (sm.fault[y].kstep == f.kstep && (sm.fault[y].row > f.row ||
                                   (sm.fault[y].row == f.row && sm.fault[y].col > f.col))))) {
                    sm.fault[y + 1] = sm.fault[y];
                    --y;
                }
                sm.fault[y + 1] = f;
            }
        }
    }
    __syncthreads();

    // ---- global -> register staging of one k-step's panels ----
    f32x4 ra[NA], rb[NB];
    const float* Abase = a.A + i0;
    const float* Bbase = a.B + (size_t)j0 * a.ldb;

    // Interior panels (whole tile inside C, full k-step, 16-byte aligned columns)
    // take the all-vector path; this test is uniform across the workgroup.
    // Edge panels load element by element from a clamped address and zero what
    // lies outside the matrix, without divergent branches.
    auto load_panels = [&](int t) {
        const int k0 = t * BK;
        const bool fullk = k0 + BK <= a.K;
        if (alignA && fullk && mI == BM) {
#pragma unroll
            for (int r = 0; r < NA; ++r) {
                const int f = tid + NT * r;
                const int i4 = f % (BM / 4), kk = f / (BM / 4);
                ra[r] = *reinterpret_cast<const f32x4*>(Abase + (size_t)(k0 + kk) * a.lda + 4 * i4);
            }
        } else {
#pragma unroll
            for (int r = 0; r < NA; ++r) {
                const int f = tid + NT * r;
                const int i4 = f % (BM / 4), kk = f / (BM / 4);
                const int gk = k0 + kk, gi = 4 * i4;
                const float* p = Abase + (size_t)gk * a.lda + gi;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool in = gk < a.K && gi + q < mI;
                    const float x = *(in ? p + q : a.A);
                    ra[r][q] = in ? x : 0.0f;
                }
            }
        }
        if (alignB && fullk && nJ == BN) {
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                const int f = tid + NT * r;
                const int kq = f % BKQ, jj = f / BKQ;
                rb[r] = *reinterpret_cast<const f32x4*>(Bbase + (size_t)jj * a.ldb + k0 + 4 * kq);
            }
        } else {
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                const int f = tid + NT * r;
                const int kq = f % BKQ, jj = f / BKQ;
                const int gk = k0 + 4 * kq;
                const float* p = Bbase + (size_t)jj * a.ldb + gk;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool in = jj < nJ && gk + q < a.K;
                    const float x = *(in ? p + q : a.B);
                    rb[r][q] = in ? x : 0.0f;
                }
            }
        }
    };

    // registers -> LDS, fused with the checksum encodings of the panel (Eq. 1-2).
    // No lane-divergent branch, so it can interleave with the MFMA stream:
    // lanes that own no result store into a private dummy slot instead.
    auto store_panels = [&](int buf, int vslot) {
        float ws[NA];
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            const int f = tid + NT * r;
            const int i4 = f % (BM / 4), kk = f / (BM / 4);
            *reinterpret_cast<f32x4*>(&sm.As[buf][kk][4 * i4]) = ra[r];
            ws[r] = (ra[r][0] + ra[r][1]) + (ra[r][2] + ra[r][3]);
        }
        f32x4 vp = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int f = tid + NT * r;
            const int kq = f % BKQ, jj = f / BKQ;
            *reinterpret_cast<f32x4*>(&sm.Bs[buf][jj][4 * kq]) = rb[r];
            vp += rb[r];
        }
        if constexpr (FT > 0) {
            // e^T A: slot r's column kk is held by AG consecutive lanes; one
            // reduce-scatter over those lanes leaves slot ((lane >> WSH) % NA)
            // in every lane, written by the lanes whose low WSH bits are zero.
            constexpr int WSH = ilog2(AG) - ilog2(NA);
            ReduceScatter<NA, ilog2(AG) - 1, 0>::run(ws, lane);
            {
                const int r = (lane >> WSH) & (NA - 1);
                const int kk = (tid - (lane & (AG - 1)) + NT * r) / (BM / 4);
                float* dst = ((lane & ((1 << WSH) - 1)) == 0) ? &sm.wsum[buf][kk] : &sm.dummy[lane];
                *dst = ws[0];
            }
            // B e: the 4 k of k-quad (lane % BKQ) are summed over the lanes of
            // that quad (bits log2(BKQ)..5); lane keeps k = 4 (lane % BKQ) +
            // ((lane >> 4) & 3); waves then add their partials in LDS.
            float vx[4] = {vp[0], vp[1], vp[2], vp[3]};
            ReduceScatter<4, 5, ilog2(BKQ)>::run(vx, lane);
            const int kv = 4 * (lane % BKQ) + ((lane >> 4) & 3);
            float* dst = ((lane & (16 - BKQ)) == 0) ? &sm.vsum[vslot][kv] : &sm.dummy[lane];
            atomicAdd(dst, vx[0]);
        }
    };

    f32x16 acc[MI][NI];
#pragma unroll
    for (int bi = 0; bi < MI; ++bi)
#pragma unroll
        for (int bj = 0; bj < NI; ++bj)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[bi][bj][r] = 0.0f;

    // Owned checksum vectors.  With SPLIT, thread t < BM owns row t (reference
    // row checksum R and ||a||^2) and the next BN threads own the columns
    // (S and ||b||^2), one vector per thread; otherwise every thread owns row
    // t (ck0, nq0) and column t (ck1, nq1), clamped in range and ignored when
    // out of range.  Addresses are selected per thread so the update is free
    // of branches and can be scheduled between MFMAs.
    float ck0 = 0.f, nq0 = 0.f, ck1 = 0.f, nq1 = 0.f;
    float& Rr = ck0;
    float& na2 = nq0;
    float& Sc = SPLIT ? ck0 : ck1;
    float& nb2 = SPLIT ? nq0 : nq1;
    const int x0_stride = row_role ? BM : 1;
    const int x0_off = row_role ? min(tid, BM - 1) : min(max(tid - COL0, 0), BN - 1) * (BK + 4);
    const int x0_buf = row_role ? BK * BM : BN * (BK + 4);
    const float* const x0_arr = row_role ? &sm.As[0][0][0] : &sm.Bs[0][0][0];
    const int x1_row = min(tid, BN - 1);

    // one group of 8 k: 4 MFMA k-substeps on every block of the wave tile
    auto mfma_group = [&](int cur, int g) {
        f32x4 bf[NI];
#pragma unroll
        for (int bj = 0; bj < NI; ++bj)
            bf[bj] = *reinterpret_cast<const f32x4*>(&sm.Bs[cur][wn * TN + 32 * bj + l32][8 * g + 4 * hh]);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            float af[MI];
#pragma unroll
            for (int bi = 0; bi < MI; ++bi) af[bi] = sm.As[cur][8 * g + 4 * hh + s][wm * TM + 32 * bi + l32];
#pragma unroll
            for (int bi = 0; bi < MI; ++bi)
#pragma unroll
                for (int bj = 0; bj < NI; ++bj)
                    acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x2f32(bf[bj][s], af[bi], acc[bi][bj], 0, 0, 0);
        }
    };

    // reference checksum update (Eq. 4) for the same 8 k:
    //   R_i += sum_k A[i,k] (B e)[k],  S_j += sum_k (e^T A)[k] B[k,j],  plus the norms
    auto ft_group = [&](int cur, int vcur, int g) {
        const float* px = x0_arr + cur * x0_buf + x0_off + 8 * g * x0_stride;
        const float* py = row_role ? &sm.vsum[vcur][8 * g] : &sm.wsum[cur][8 * g];
        const f32x4 ya = *reinterpret_cast<const f32x4*>(py);
        const f32x4 yb = *reinterpret_cast<const f32x4*>(py + 4);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float x = px[q * x0_stride];
            ck0 = fmaf(x, q < 4 ? ya[q] : yb[q - 4], ck0);
            nq0 = fmaf(x, x, nq0);
        }
        if constexpr (!SPLIT) {
            const f32x4 b0 = *reinterpret_cast<const f32x4*>(&sm.Bs[cur][x1_row][8 * g]);
            const f32x4 b1 = *reinterpret_cast<const f32x4*>(&sm.Bs[cur][x1_row][8 * g + 4]);
            const f32x4 w0 = *reinterpret_cast<const f32x4*>(&sm.wsum[cur][8 * g]);
            const f32x4 w1 = *reinterpret_cast<const f32x4*>(&sm.wsum[cur][8 * g + 4]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ck1 = fmaf(w0[q], b0[q], ck1);
                nq1 = fmaf(b0[q], b0[q], nq1);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ck1 = fmaf(w1[q], b1[q], ck1);
                nq1 = fmaf(b1[q], b1[q], nq1);
            }
        }
    };

    // One k-step.  The next panel's global loads are issued first; the LDS
    // store and encode of that panel follow the last MFMA group (its loads
    // have landed by then) and, like the checksum update, carry no branch,
    // so the compiler can interleave them with the MFMAs in flight.
    auto step = [&](int t, auto has_next) {
        constexpr bool NEXT = decltype(has_next)::value;
        const int cur = t & 1;
        if constexpr (NEXT) load_panels(t + 1);
        if constexpr (FT > 0 && NEXT)   // slot for step t+2: its last reader finished before this step
            (&sm.vsum[(t + 2) % 3][0])[tid < BK ? tid : BK - 1] = 0.f;
#pragma unroll
        for (int g = 0; g < BK / 8; ++g) {
            mfma_group(cur, g);
            if constexpr (FT > 0) ft_group(cur, t % 3, g);
            if constexpr (NEXT) {
                if (g == (BK / 8 >= 2 ? BK / 8 - 2 : 0)) store_panels(cur ^ 1, (t + 1) % 3);
            }
        }
    };

    // ---- injection hook: faults of k-step t hit the accumulator ----
    auto inject = [&](int t) {
        if constexpr (INJ) {
            while (fnext < sm.nf && sm.fault[fnext].kstep == t) {   // uniform loop
                const ftgemm_fault_t f = sm.fault[fnext];
                const int ir = f.row % TM, jr = f.col % TN;
                const int fbi = ir / 32, fbj = jr / 32, jj = jr % 32;
                const int freg = ((jj >> 3) << 2) | (jj & 3);
                const bool own = f.row / TM == wm && f.col / TN == wn && lane == ((jj >> 2) & 1) * 32 + (ir % 32);
                float oldv = 0.f, newv = 0.f;
#pragma unroll
                for (int bi = 0; bi < MI; ++bi)
#pragma unroll
                    for (int bj = 0; bj < NI; ++bj) {
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
                    sm.fslot[fnext] = slot;
                    if (slot < a.fault_log_cap) {
                        ftgemm_fault_log_t L;
                        L.problem = a.problem; L.tile_m = tm; L.tile_n = tn; L.kstep = t;
                        L.row = f.row; L.col = f.col; L.kind = f.kind; L.check_step = -1;
                        L.old_v = oldv; L.new_v = newv;
                        L.r_row = L.r_col = L.tau_row = L.tau_col = 0.f;
                        L.pad0_ = L.pad1_ = 0.f;
                        a.fault_log[slot] = L;
                    }
                }
                ++fnext;
            }
        }
    };

    auto check = [&](int t) -> bool {
        // ---- online check ----
        bool do_check = false;
        if constexpr (FT == 2) do_check = ((t + 1) % a.check_interval == 0) || (t == nk - 1);
        if constexpr (FT == 1) do_check = (t == nk - 1);
        if (do_check) {
            // (1) one pass over the accumulator, one 32-column block at a time:
            // per-lane partial row sums (over the lane's columns) and the block's
            // column sums over this wave's rows; the 16 column sums of a lane are
            // reduce-scattered over the 32 lanes of its half, leaving lane pair
            // (2x, 2x+1) with entry x.  The scheduling fence keeps the
            // accumulator reads of one block from being hoisted into the next.
            float rpart[MI];
#pragma unroll
            for (int bi = 0; bi < MI; ++bi) rpart[bi] = 0.f;
#pragma unroll
            for (int bj = 0; bj < NI; ++bj) {
                float cs[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) cs[r] = 0.f;
#pragma unroll
                for (int bi = 0; bi < MI; ++bi) {
                    float rs = 0.f;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float x = acc[bi][bj][r];
                        cs[r] += x;
                        rs += x;
                    }
                    rpart[bi] += rs;
                }
                ReduceScatter<16, 4, 0>::run(cs, lane);
                if ((l32 & 1) == 0) {
                    const int r = l32 >> 1;
                    sm.colpart[wm][wn * TN + 32 * bj + 8 * (r >> 2) + 4 * hh + (r & 3)] = cs[0];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int bi = 0; bi < MI; ++bi) {
                const float rs = rpart[bi] + __shfl_xor(rpart[bi], 32);
                if (hh == 0) sm.rowpart[wn][wm * TM + 32 * bi + l32] = rs;
            }
            // (2) per-wave sums of the row and column norms for the threshold
            const float na = (my_row >= 0) ? sqrtf(na2) : 0.f;
            const float nb = (my_col >= 0) ? sqrtf(nb2) : 0.f;
            const float wna = wave_sum(na), wnb = wave_sum(nb);
            if (lane == 0) { sm.nsum[0][wave] = wna; sm.nsum[1][wave] = wnb; }
            __syncthreads();

            // (3) residuals, thresholds, flags
            float sa = 0.f, sb = 0.f;
#pragma unroll
            for (int w = 0; w < NW; ++w) { sa += sm.nsum[0][w]; sb += sm.nsum[1][w]; }
            const int kp = min((t + 1) * BK, a.K);
            const float base = a.tol_c * 2.0f * kUnitRoundoff;
            float rres = 0.f, cres = 0.f, taur = 0.f, tauc = 0.f;
            bool rf = false, cf = false;
            if (my_row >= 0 && my_row < mI) {
                float s = 0.f;
#pragma unroll
                for (int w = 0; w < WN; ++w) s += sm.rowpart[w][my_row];
                rres = s - Rr;
                taur = base * (float)(kp + nJ + 1) * na * sb;
                rf = !(fabsf(rres) <= taur);
            }
            if (my_col >= 0 && my_col < nJ) {
                float s = 0.f;
#pragma unroll
                for (int w = 0; w < WM; ++w) s += sm.colpart[w][my_col];
                cres = s - Sc;
                tauc = base * (float)(kp + mI + 1) * nb * sa;
                cf = !(fabsf(cres) <= tauc);
            }
            const unsigned long long rb_ = __ballot(rf), cb_ = __ballot(cf);
            if (lane == 0) {
                sm.census[wave][0] = __popcll(rb_);
                sm.census[wave][1] = rb_ ? wave * 64 + __ffsll((long long)rb_) - 1 : -1;
                sm.census[wave][2] = __popcll(cb_);
                sm.census[wave][3] = cb_ ? wave * 64 + __ffsll((long long)cb_) - 1 - COL0 : -1;
            }
            // complete the fault log entries this check is the first to see
            if constexpr (INJ) {
                for (int q = flogged; q < fnext; ++q) {
                    const int slot = sm.fslot[q];
                    if (slot < 0 || slot >= a.fault_log_cap) continue;
                    if (my_row == sm.fault[q].row) { a.fault_log[slot].r_row = rres; a.fault_log[slot].tau_row = taur; }
                    if (my_col == sm.fault[q].col) { a.fault_log[slot].r_col = cres; a.fault_log[slot].tau_col = tauc; }
                    if (tid == 0) a.fault_log[slot].check_step = t;
                }
                flogged = fnext;
            }
            __syncthreads();

            int nr = 0, ncl = 0, fr = -1, fc = -1;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                nr += sm.census[w][0];
                ncl += sm.census[w][2];
                if (fr < 0) fr = sm.census[w][1];
                if (fc < 0) fc = sm.census[w][3];
            }

            if (nr + ncl > 0) {   // rare path: something was flagged (uniform branch)
                const bool correct = (FT == 2) && nr == 1 && ncl == 1;
                if (my_row >= 0 && my_row == fr) { sm.bc[0] = Rr; sm.bc[1] = rres; sm.bc[2] = taur; }
                if (my_col >= 0 && my_col == fc) { sm.bc[3] = cres; sm.bc[4] = tauc; }
                // Coordinates of (fr, fc) in the accumulator layout; all but the
                // lane tests are uniform, so the block is picked by scalar
                // branches and the element by per-lane selects (compact code).
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
                    part += __shfl_xor(part, 32);
                    float* dst = (lane == (fr & 31)) ? &sm.excl[wn] : &sm.dummy[lane];
                    *dst = part;
                }
                __syncthreads();
                if (correct) {
                    float excl = 0.f;
#pragma unroll
                    for (int w = 0; w < WN; ++w) excl += sm.excl[w];
                    const float newv = sm.bc[0] - excl;
#pragma unroll
                    for (int bi = 0; bi < MI; ++bi)
#pragma unroll
                        for (int bj = 0; bj < NI; ++bj) {
                            if (bi == fbi && bj == fbj) {
#pragma unroll
                                for (int r = 0; r < 16; ++r)
                                    acc[bi][bj][r] = (own && r == freg) ? newv : acc[bi][bj][r];
                            }
                        }
                    if (own) {
                        const unsigned e = atomicAdd(&a.counters[CNT_EVENTS], 1u);
                        atomicAdd(&a.counters[CNT_DETECTED], 1u);
                        atomicAdd(&a.counters[CNT_CORRECTED], 1u);
                        if ((int)e < a.event_cap) {
                            ftgemm_event_t E;
                            E.problem = a.problem; E.tile_m = tm; E.tile_n = tn; E.kstep = t;
                            E.row = fr; E.col = fc; E.kind = FTGEMM_EV_CORRECTED; E.n_rows = 1; E.n_cols = 1;
                            E.pad_ = 0; E.value_before = oldv; E.value_after = newv;
                            E.r_row = sm.bc[1]; E.r_col = sm.bc[3]; E.tau_row = sm.bc[2]; E.tau_col = sm.bc[4];
                            a.events[e] = E;
                        }
                    }
                } else {
                    int kind;
                    if constexpr (FT == 1) kind = FTGEMM_EV_DETECTED;
                    else kind = (nr == 1 && ncl == 0) ? FTGEMM_EV_CHECKSUM_ROW
                              : (nr == 0 && ncl == 1) ? FTGEMM_EV_CHECKSUM_COL
                              : FTGEMM_EV_UNCORRECTABLE;
                    if constexpr (FT == 2) {   // re-base the flagged checksums on the accumulator
                        if (rf) Rr += rres;
                        if (cf) Sc += cres;
                    }
                    if (tid == 0) {
                        const unsigned e = atomicAdd(&a.counters[CNT_EVENTS], 1u);
                        atomicAdd(&a.counters[CNT_DETECTED], 1u);
                        if (kind == FTGEMM_EV_UNCORRECTABLE) atomicAdd(&a.counters[CNT_UNCORRECTABLE], 1u);
                        if (kind == FTGEMM_EV_CHECKSUM_ROW || kind == FTGEMM_EV_CHECKSUM_COL)
                            atomicAdd(&a.counters[CNT_CHECKSUM_ONLY], 1u);
                        if ((int)e < a.event_cap) {
                            ftgemm_event_t E;
                            E.problem = a.problem; E.tile_m = tm; E.tile_n = tn; E.kstep = t;
                            E.row = fr; E.col = fc; E.kind = kind; E.n_rows = nr; E.n_cols = ncl; E.pad_ = 0;
                            E.value_before = E.value_after = 0.f;
                            E.r_row = fr >= 0 ? sm.bc[1] : 0.f; E.tau_row = fr >= 0 ? sm.bc[2] : 0.f;
                            E.r_col = fc >= 0 ? sm.bc[3] : 0.f; E.tau_col = fc >= 0 ? sm.bc[4] : 0.f;
                            a.events[e] = E;
                        }
                    }
                }
            }
        }
        return do_check;
    };

    load_panels(0);
    store_panels(0, 0);
    __syncthreads();
    for (int t = 0; t + 1 < nk; ++t) {
        step(t, std::true_type{});
        inject(t);
        // a check ends with a workgroup barrier after its census, which also
        // orders this step's LDS panel writes before the next step's reads
        if (!check(t)) __syncthreads();
    }
    step(nk - 1, std::false_type{});
    inject(nk - 1);
    check(nk - 1);

    // ---- epilogue: C = alpha * P + beta * C ----
#pragma unroll
    for (int bi = 0; bi < MI; ++bi) {
        const int i = wm * TM + 32 * bi + l32;
#pragma unroll
        for (int bj = 0; bj < NI; ++bj)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = wn * TN + 32 * bj + 8 * (r >> 2) + 4 * hh + (r & 3);
                if (i < mI && j < nJ) {
                    float* pc = a.C + (size_t)(j0 + j) * a.ldc + (i0 + i);
                    float v = a.alpha * acc[bi][bj][r];
                    if (a.beta != 0.0f) v = fmaf(a.beta, *pc, v);
                    *pc = v;
                }
            }
    }
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

hipError_t launch_scale(float* C, int64_t ldc, int32_t M, int32_t N, float beta, hipStream_t s) {
    const int64_t total = (int64_t)M * N;
    const int blocks = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
    hipLaunchKernelGGL(scale_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, C, ldc, M, N, beta);
    return hipGetLastError();
}

}  // namespace ftgemm_impl
