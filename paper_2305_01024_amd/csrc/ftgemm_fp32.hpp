// ftgemm_fp32.hpp -- FP32 online ABFT GEMM kernels for gfx950 (MI355X).
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
// Both panels sit in LDS k-contiguous ([row][k], padded to BK + 4 floats):
// B (column-major) is k-contiguous in memory already; A (column-major, i
// contiguous) is loaded as 4 x 4 blocks (four 16-byte loads along i at four
// consecutive k) and transposed in registers on the way to LDS.  The k index
// of the two lane halves is permuted (lane half h takes k = 8g + 4h + s in
// MFMA s of group g), so each operand is one 16-byte LDS read per four MFMAs
// and a checksum owner reads its row or column 16 bytes at a time.
#pragma once

#include "ftgemm_abft.hpp"

namespace ftgemm_impl {
namespace f32 {

using namespace abft;

// The 16-byte chunk c of A panel row i is stored at chunk c ^ aswz(i).  With
// the BK + 4 pitch, the 16 rows 4 iq + q (iq = 0..15) that one transposing
// store instruction writes then fall into 16 distinct bank groups, while 16
// consecutive rows read at one chunk (MFMA fragments, checksum owners) stay
// conflict-free.
__device__ __forceinline__ constexpr int aswz(int i) { return (i >> 4) & 3; }

// EA / EB: encodings per panel (1 for compute-tile checks; WM / WN for
// wavefront-tile checks, one per wave row / wave column of the tile).
template <int BM, int BN, int BK, int EA = 1, int EB = 1>
struct alignas(16) Operands {   // 16-byte aligned: the panel reads are 16-byte LDS loads
    static constexpr int KP = BK + 4;   // row pitch: conflict-free 16-byte reads by 16 lanes on 16 rows
    float As[2][BM][KP];        // A panel, i-major (k contiguous)
    float Bs[2][BN][KP];        // B panel, j-major (k contiguous)
    float wsum[2][EA][BK];      // e^T A of the panel (per wave row group), per k
    float vsum[3][EB][BK];      // B e of the panel (per wave column group), per k (accumulated across waves, 3 rotating slots)
    float dummy[256];           // sink for the stores/atomics of lanes that own no value
};

template <int BM, int BN, int BK, int WM, int WN, bool WAVE = false>
struct Smem {
    using G = Geometry<BM, BN, WM, WN>;
    Operands<BM, BN, BK, WAVE ? WM : 1, WAVE ? WN : 1> op;
    std::conditional_t<WAVE, WaveCheckLds<G>, CheckLds<G>> ck;
};

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------
// One BM x BN output tile (tm, tn) of the problem in `a`, computed by one
// workgroup of 64 * WM * WN threads with `sm` as its LDS.  WAVE: each
// wavefront's TM x TN sub-tile is a check tile (warp-level ABFT, section
// 4.2.2) instead of the whole tile (section 4.2.3).
template <int BM, int BN, int BK, int WM, int WN, int FT, bool INJ, bool WAVE = false>
__device__ __forceinline__ void tile(const LaunchArgs& a, int tm, int tn, Smem<BM, BN, BK, WM, WN, WAVE>& sm) {
    using G = Geometry<BM, BN, WM, WN>;
    constexpr int NT = G::NT, TM = G::TM, TN = G::TN, MI = G::MI, NI = G::NI;
    constexpr int KP = Operands<BM, BN, BK>::KP;
    constexpr int EA = WAVE ? WM : 1, EB = WAVE ? WN : 1;
    constexpr int AIQ = BM / 4;                // i-quads of the A panel
    constexpr int NA = BM * BK / (16 * NT);    // 4 x 4 blocks of A per thread
    constexpr int NB = BN * BK / (4 * NT);     // float4 slots of B per thread
    constexpr int AG = AIQ < 64 ? AIQ : 64;    // lanes sharing one k-quad in the A load
    constexpr int LAG = ilog2(AG), LNA = ilog2(4 * NA);
    constexpr int BKQ = BK / 4;                // lanes sharing one column in the B load
    constexpr bool SPLIT = G::SPLIT;
    static_assert(NA >= 1 && NB >= 1 && BK % 8 == 0, "tile shape");
    static_assert(BM * BK == 16 * NA * NT && (AIQ % 64 == 0 || 64 % AIQ == 0), "A block mapping");
    static_assert(LNA <= LAG, "encode reduce-scatter needs 4 NA <= AG");
    static_assert(NT % BKQ == 0 && 64 % BKQ == 0 && BKQ <= 16, "B slot mapping");
    static_assert(!WAVE || (G::SPLIT && TN % (NT / BKQ) == 0 && TM / 4 <= AG && NT >= EB * BK),
                  "wavefront checks: one owner per line, each B slot inside one wave column");

    auto& op = sm.op;

    const Thread th = make_thread<G, (FT > 0)>(a, tm, tn);
    const int tid = th.tid, lane = th.lane, wm = th.wm, wn = th.wn, l32 = th.l32, hh = th.hh;
    const int mI = th.mI, nJ = th.nJ;
    const int nk = (a.K + BK - 1) / BK;

    const bool alignA = ((reinterpret_cast<uintptr_t>(a.A) & 15) == 0) && ((a.lda & 3) == 0);
    const bool alignB = ((reinterpret_cast<uintptr_t>(a.B) & 15) == 0) && ((a.ldb & 3) == 0);

    if constexpr (FT > 0) {
        for (int x = tid; x < 3 * EB * BK; x += NT) (&op.vsum[0][0][0])[x] = 0.f;
        clear_check(sm.ck, tid);
    }
    int fnext = 0, flogged = 0;
    if constexpr (INJ) gather_faults<G, WAVE>(sm.ck, a, th);
    __syncthreads();

    // ---- global -> register staging of one k-step's panels ----
    f32x4 ra[NA][4], rb[NB];     // ra[r][e]: rows 4 iq .. 4 iq + 3 of k = 4 kq + e
    const float* Abase = a.A + th.i0;
    const float* Bbase = a.B + (size_t)th.j0 * a.ldb;

    // Interior panels (whole tile inside C, full k-step, 16-byte aligned columns)
    // take the all-vector path; this test is uniform across the workgroup.
    // Edge panels load element by element from a clamped address and zero what
    // lies outside the matrix, without divergent branches.
    // Interior panels are read with buffer loads: the per-lane byte offset of
    // each slot is fixed for the whole k-loop, the per-step panel origin goes
    // into the (scalar) resource base and the k-column stride into the scalar
    // offset, so the loop spends no vector instructions on addresses.  Used
    // while every offset of a panel fits in 31 bits.
    const bool bufA = alignA && (int64_t)BK * a.lda * 4 < (int64_t(1) << 31);
    const bool bufB = alignB && (int64_t)BN * a.ldb * 4 < (int64_t(1) << 31);
    int voffA[NA], voffB[NB];
#pragma unroll
    for (int r = 0; r < NA; ++r) {
        const int f = tid + NT * r;
        voffA[r] = ((f / AIQ) * 4 * (int)a.lda + 4 * (f % AIQ)) * 4;
    }
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        const int f = tid + NT * r;
        voffB[r] = ((f / BKQ) * (int)a.ldb + 4 * (f % BKQ)) * 4;
    }
    constexpr int kRsrcWord3 = 0x00020000;   // raw 32-bit data format

    auto load_A = [&](int t) {
        const int k0 = t * BK;
        const bool fullk = k0 + BK <= a.K;
        int k0e = k0;   // edge-path k origin, opaque to the loop optimiser (no per-step pointer updates)
        asm volatile("" : "+s"(k0e));
        if (bufA && fullk && mI == BM) {
            const auto rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<float*>(Abase + (size_t)k0 * a.lda), (short)0, 0x7fffffff, kRsrcWord3);
#pragma unroll
            for (int r = 0; r < NA; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    ra[r][e] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(
                                                             rs, voffA[r], e * (int)a.lda * 4, 0));
        } else {
#pragma unroll
            for (int r = 0; r < NA; ++r) {
                const int f = tid + NT * r;
                const int iq = f % AIQ, kq = f / AIQ;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int gk = k0e + 4 * kq + e, gi = 4 * iq;
                    const float* p = Abase + (size_t)gk * a.lda + gi;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const bool in = gk < a.K && gi + q < mI;
                        const float x = *(in ? p + q : a.A);
                        ra[r][e][q] = in ? x : 0.0f;
                    }
                }
            }
        }
    };
    auto load_B = [&](int t) {
        const int k0 = t * BK;
        const bool fullk = k0 + BK <= a.K;
        int k0e = k0;   // edge-path k origin, opaque to the loop optimiser (no per-step pointer updates)
        asm volatile("" : "+s"(k0e));
        if (bufB && fullk && nJ == BN) {
            const auto rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(Bbase + k0), (short)0, 0x7fffffff,
                                                              kRsrcWord3);
#pragma unroll
            for (int r = 0; r < NB; ++r)
                rb[r] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voffB[r], 0, 0));
        } else {
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                const int f = tid + NT * r;
                const int kq = f % BKQ, jj = f / BKQ;
                const int gk = k0e + 4 * kq;
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
    auto store_A = [&](int buf) {
        float ws[4 * NA];
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            const int f = tid + NT * r;
            const int iq = f % AIQ, kq = f / AIQ;
#pragma unroll
            for (int q = 0; q < 4; ++q) {   // row 4 iq + q gets its 4 k (element stores: no register shuffles)
                const int i = 4 * iq + q;
                float* dst = &op.As[buf][i][4 * (kq ^ aswz(i))];
#pragma unroll
                for (int e = 0; e < 4; ++e) dst[e] = ra[r][e][q];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) ws[4 * r + e] = (ra[r][e][0] + ra[r][e][1]) + (ra[r][e][2] + ra[r][e][3]);
        }
        if constexpr (FT > 0 && !WAVE) {
            // e^T A: the AG lanes of one k-quad group (lane bits 0 .. LAG-1)
            // hold all BM rows of their k-quads; one reduce-scatter over those
            // bits leaves entry v = (lane >> (LAG - LNA)) of the 4 NA sums in
            // every lane, stored by the lanes whose lower bits are zero.
            ReduceScatter<4 * NA, LAG - 1, 0>::run(ws, lane);
            const int v = (lane >> (LAG - LNA)) & (4 * NA - 1);
            const int f = tid - (lane & (AG - 1)) + NT * (v >> 2);
            const int kk = 4 * (f / AIQ) + (v & 3);
            float* dst = ((lane & ((1 << (LAG - LNA)) - 1)) == 0) ? &op.wsum[buf][0][kk] : &op.dummy[lane];
            *dst = ws[0];
        } else if constexpr (FT > 0) {
            // e^T A_w per wave row group: the same reduce-scatter over the AW
            // lanes that hold one group's TM rows of a k-quad (lane bits
            // 0 .. LAW-1)
            constexpr int AW = TM / 4, LAW = ilog2(AW);
            static_assert(LNA <= LAW, "encode reduce-scatter needs 4 NA <= AW");
            ReduceScatter<4 * NA, LAW - 1, 0>::run(ws, lane);
            const int v = (lane >> (LAW - LNA)) & (4 * NA - 1);
            const int f = tid - (lane & (AW - 1)) + NT * (v >> 2);
            const int kk = 4 * (f / AIQ) + (v & 3);
            const int grp = 4 * (f % AIQ) / TM;
            float* dst = ((lane & ((1 << (LAW - LNA)) - 1)) == 0) ? &op.wsum[buf][grp][kk] : &op.dummy[lane];
            *dst = ws[0];
        }
    };
    auto store_B = [&](int buf, int vslot) {
        f32x4 vp = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int f = tid + NT * r;
            const int kq = f % BKQ, jj = f / BKQ;
            *reinterpret_cast<f32x4*>(&op.Bs[buf][jj][4 * kq]) = rb[r];
            if constexpr (!WAVE) vp += rb[r];
        }
        // B e: the 4 k of k-quad (lane % BKQ) are summed over the lanes of
        // that quad (bits log2(BKQ)..5); lane keeps k = 4 (lane % BKQ) +
        // ((lane >> 4) & 3); waves then add their partials in LDS.
        if constexpr (FT > 0 && !WAVE) {
            float vx[4] = {vp[0], vp[1], vp[2], vp[3]};
            ReduceScatter<4, 5, ilog2(BKQ)>::run(vx, lane);
            const int kv = 4 * (lane % BKQ) + ((lane >> 4) & 3);
            float* dst = ((lane & (16 - BKQ)) == 0) ? &op.vsum[vslot][0][kv] : &op.dummy[lane];
            atomicAdd(dst, vx[0]);
        } else if constexpr (FT > 0) {
            // B_w e per wave column group q (slot r lies in group (NT r / BKQ) / TN)
#pragma unroll
            for (int q = 0; q < EB; ++q) {
                f32x4 vq = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int r = 0; r < NB; ++r)
                    if ((NT * r / BKQ) / TN == q) vq += rb[r];
                float vx[4] = {vq[0], vq[1], vq[2], vq[3]};
                ReduceScatter<4, 5, ilog2(BKQ)>::run(vx, lane);
                const int kv = 4 * (lane % BKQ) + ((lane >> 4) & 3);
                float* dst = ((lane & (16 - BKQ)) == 0) ? &op.vsum[vslot][q][kv] : &op.dummy[lane];
                atomicAdd(dst, vx[0]);
            }
        }
    };

    Acc<G> acc;
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
    const bool row_role = th.row_role;
    const int x0_row = row_role ? min(tid, BM - 1) : min(max(tid - G::COL0, 0), BN - 1);
    const float* const x0_arr = row_role ? &op.As[0][0][0] : &op.Bs[0][0][0];
    const int x0_swz = row_role ? aswz(x0_row) : 0;
    constexpr int XB_A = BM * KP, XB_B = BN * KP;
    const int x0_buf = row_role ? XB_A : XB_B;
    const int x1_row = min(tid, BN - 1);
    // one group of 8 k: 4 MFMA k-substeps on every block of the wave tile
    // Operand fragments of group g+1 are read while group g's MFMAs run.  The
    // FT kernels double-buffer only the B fragments and read the A fragments
    // at the start of their group: the registers go to the checksum update.
    constexpr bool PFA = (FT == 0);
    f32x4 bfr[2][NI], afr[PFA ? 2 : 1][MI];
    auto load_b = [&](int cur, int g) {
#pragma unroll
        for (int bj = 0; bj < NI; ++bj)
            bfr[g & 1][bj] = *reinterpret_cast<const f32x4*>(&op.Bs[cur][wn * TN + 32 * bj + l32][8 * g + 4 * hh]);
    };
    auto load_a = [&](int cur, int g) {
#pragma unroll
        for (int bi = 0; bi < MI; ++bi) {
            const int i = wm * TM + 32 * bi + l32;
            afr[PFA ? (g & 1) : 0][bi] = *reinterpret_cast<const f32x4*>(&op.As[cur][i][4 * ((2 * g + hh) ^ aswz(i))]);
        }
    };
    auto mfma_group = [&](int cur, int g) {
        if (g == 0) {
            load_b(cur, 0);
            if constexpr (PFA) load_a(cur, 0);
        }
        if (g + 1 < BK / 8) {
            load_b(cur, g + 1);
            if constexpr (PFA) load_a(cur, g + 1);
        }
        if constexpr (!PFA) load_a(cur, g);
        const int ab = PFA ? (g & 1) : 0;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int bi = 0; bi < MI; ++bi)
#pragma unroll
                for (int bj = 0; bj < NI; ++bj)
                    acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x2f32(bfr[g & 1][bj][s], afr[ab][bi][s], acc[bi][bj], 0, 0, 0);
    };

    // reference checksum update (Eq. 4) for the same 8 k:
    //   R_i += sum_k A[i,k] (B e)[k],  S_j += sum_k (e^T A)[k] B[k,j],  plus the norms
    // The operands of a group's update are read before the group's MFMAs (with
    // the next group's fragments) and applied after them, so their LDS
    // latency hides behind the MFMAs instead of stalling the wave.
    // Wavefront-tile checks: the row owner keeps R against each wave
    // column's encoding vsum[.][q] (q < WN), the column owner S against each
    // wave row's wsum[.][q] (q < WM); wref[q] for q beyond the owner's count
    // is computed and ignored.
    constexpr int NR = WAVE ? (WM > WN ? WM : WN) : 1;
    float wref[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) wref[q] = 0.f;
    // The wavefront-check update runs after the k-step's MFMAs, 4 k at a
    // time, where the fragment and staging registers are free (the other
    // wavefront on the SIMD keeps the matrix cores busy meanwhile).
    struct FtHalf {
        f32x4 x, y[NR];
    };
    auto ft_load_half = [&](int cur, int vcur, int g, int h) {
        FtHalf o;
        const float* px = x0_arr + cur * x0_buf + x0_row * KP;
        o.x = *reinterpret_cast<const f32x4*>(px + 4 * ((2 * g + h) ^ x0_swz));
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const float* py = row_role ? &op.vsum[vcur][q < EB ? q : EB - 1][8 * g + 4 * h]
                                       : &op.wsum[cur][q < EA ? q : EA - 1][8 * g + 4 * h];
            o.y[q] = *reinterpret_cast<const f32x4*>(py);
        }
        return o;
    };
    auto ft_apply_half = [&](const FtHalf& o) {
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) wref[q] = fmaf(o.x[e], o.y[q][e], wref[q]);
#pragma unroll
        for (int e = 0; e < 4; ++e) nq0 = fmaf(o.x[e], o.x[e], nq0);
    };
    struct FtOps {
        f32x4 xa, xb, ya, yb, b0, b1, w0, w1;
    };
    auto ft_load = [&](int cur, int vcur, int g) {
        FtOps o;
        const float* px = x0_arr + cur * x0_buf + x0_row * KP;
        o.xa = *reinterpret_cast<const f32x4*>(px + 4 * ((2 * g) ^ x0_swz));
        o.xb = *reinterpret_cast<const f32x4*>(px + 4 * ((2 * g + 1) ^ x0_swz));
        const float* py = row_role ? &op.vsum[vcur][0][8 * g] : &op.wsum[cur][0][8 * g];
        o.ya = *reinterpret_cast<const f32x4*>(py);
        o.yb = *reinterpret_cast<const f32x4*>(py + 4);
        if constexpr (!SPLIT) {
            o.b0 = *reinterpret_cast<const f32x4*>(&op.Bs[cur][x1_row][8 * g]);
            o.b1 = *reinterpret_cast<const f32x4*>(&op.Bs[cur][x1_row][8 * g + 4]);
            o.w0 = *reinterpret_cast<const f32x4*>(&op.wsum[cur][0][8 * g]);
            o.w1 = *reinterpret_cast<const f32x4*>(&op.wsum[cur][0][8 * g + 4]);
        }
        return o;
    };
    auto ft_apply = [&](const FtOps& o) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ck0 = fmaf(o.xa[q], o.ya[q], ck0);
            nq0 = fmaf(o.xa[q], o.xa[q], nq0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ck0 = fmaf(o.xb[q], o.yb[q], ck0);
            nq0 = fmaf(o.xb[q], o.xb[q], nq0);
        }
        if constexpr (!SPLIT) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ck1 = fmaf(o.w0[q], o.b0[q], ck1);
                nq1 = fmaf(o.b0[q], o.b0[q], nq1);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ck1 = fmaf(o.w1[q], o.b1[q], ck1);
                nq1 = fmaf(o.b1[q], o.b1[q], nq1);
            }
        }
    };

    // One k-step.  FT kernels load the next A panel from global memory at the
    // start and store it to LDS (with its encode) after group GA, then load the
    // next B panel and store it (with its encode) after the last group, so only
    // one panel's staging registers are live at a time.  The plain kernel,
    // with registers to spare, loads both at the start and stores both after
    // group NG - 2.  The stores carry no branch, so the compiler can
    // interleave them with the MFMAs in flight.
    constexpr int NG = BK / 8;
    constexpr int GA = FT > 0 ? (NG >= 2 ? NG / 2 - 1 : 0) : (NG >= 2 ? NG - 2 : 0);
    constexpr int GB = FT > 0 ? NG - 1 : GA;
    auto step = [&](int t, auto has_next) {
        constexpr bool NEXT = decltype(has_next)::value;
        const int cur = t & 1;
        if constexpr (NEXT) {
            load_A(t + 1);
            if constexpr (FT == 0) load_B(t + 1);
        }
        if constexpr (FT > 0 && NEXT)   // slot for step t+2: its last reader finished before this step
            (&op.vsum[(t + 2) % 3][0][0])[tid < EB * BK ? tid : EB * BK - 1] = 0.f;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            FtOps o;
            if constexpr (FT > 0 && !WAVE) o = ft_load(cur, t % 3, g);
            mfma_group(cur, g);
            if constexpr (FT > 0 && !WAVE) ft_apply(o);
            if constexpr (NEXT) {
                if (g == GA) {
                    store_A(cur ^ 1);
                    if constexpr (FT > 0) load_B(t + 1);
                }
                if (g == GB) store_B(cur ^ 1, (t + 1) % 3);
            }
        }
        if constexpr (FT > 0 && WAVE) {
#pragma unroll
            for (int g = 0; g < NG; ++g)
#pragma unroll
                for (int hf = 0; hf < 2; ++hf) ft_apply_half(ft_load_half(cur, t % 3, g, hf));
        }
    };

    // injection hook and online check after k-step t.  The detect-only level
    // has the same loop: the host sets its check interval beyond the last
    // k-step, so it checks once, after the last step.
    auto post = [&](int t) -> bool {
        if constexpr (INJ) inject<G, WAVE>(acc, sm.ck, a, th, t, fnext);
        bool do_check = false;
        if constexpr (FT > 0) do_check = ((t + 1) % a.check_interval == 0) || (t == nk - 1);
        if (do_check) {
            if constexpr (WAVE) check_wave<G, FT, INJ>(acc, sm.ck, a, th, t, min((t + 1) * BK, a.K), wref, nq0, fnext, flogged);
            else check<G, FT, INJ>(acc, sm.ck, a, th, t, min((t + 1) * BK, a.K), Rr, na2, Sc, nb2, fnext, flogged);
        }
        return do_check;
    };

    load_A(0);
    load_B(0);
    store_A(0);
    store_B(0, 0);
    __syncthreads();
    for (int t = 0; t + 1 < nk; ++t) {
        step(t, std::true_type{});
        // a check ends with a workgroup barrier after its census, which also
        // orders this step's LDS panel writes before the next step's reads
        if (!post(t)) __syncthreads();
    }
    step(nk - 1, std::false_type{});
    post(nk - 1);
    finish_tile<G, FT>(acc, sm.ck, a, th, 1.0f);
}

}  // namespace f32
}  // namespace ftgemm_impl
