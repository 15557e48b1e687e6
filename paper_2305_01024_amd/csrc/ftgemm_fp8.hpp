// ftgemm_fp8.hpp -- FP8 (OCP E4M3) input online ABFT GEMM kernels for gfx950.
//
// C = alpha * (scale_a * A) (scale_b * B) + beta * C with A, B as E4M3 codes
// and FP32 accumulation on v_mfma_scale_f32_32x32x64_f8f6f4 (unit scales).  The fault tolerance
// is the threadblock-level online ABFT of the FP32 kernels (section 2.2
// Eq. 1-4, section 4.2.3): every E4M3 value converts exactly to FP32
// (v_cvt_pk_f32_fp8), so the encodings e^T A and B e, the reference
// checksums, the norms and the check run in FP32 on the decoded operands with
// the FP32 roundoff threshold.  The per-tensor scales are applied in the
// epilogue, outside the checked region.
//
// Layout: both operands sit in LDS k-contiguous ([row][k], 16-byte padded
// rows): lane l of a 32x32x64 MFMA supplies 32 consecutive k (32 bytes) of
// one row.  B (column-major K x N) is k-contiguous already; A (column-major
// M x K) is i-contiguous, so each thread loads an 8-row x 4-k byte block
// (four 8-byte loads) and transposes it in registers on the way to LDS.  As
// in the other kernels the MFMA computes P^T = B^T A^T, so lane l % 32 owns
// one row of C.
#pragma once

#include "ftgemm_abft.hpp"

namespace ftgemm_impl {
namespace fp8 {

using namespace abft;

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

template <int BM, int BN, int BK>
struct alignas(16) OperandsFP8 {   // 16-byte aligned: the panel reads are 16-byte LDS loads
    static constexpr int KP = BK + 16;         // row pitch in bytes (16 B of padding)
    unsigned char As[2][BM][KP];               // A panel, i-major, k contiguous
    unsigned char Bs[2][BN][KP];               // B panel, j-major, k contiguous
    float wsum[3][BK];                         // e^T A per k (accumulated across waves, 3 rotating slots)
    float vsum[3][BK];                         // B e per k (accumulated across waves, 3 rotating slots)
};

template <int BM, int BN, int BK, int WM, int WN>
struct SmemFP8 {
    OperandsFP8<BM, BN, BK> op;
    CheckLds<Geometry<BM, BN, WM, WN>> ck;
};

// the four E4M3 values of a dword, exactly as FP32 (byte q -> element q)
__device__ __forceinline__ void decode4(unsigned x, float* f) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)x, false);
    const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)x, true);
    f[0] = lo[0];
    f[1] = lo[1];
    f[2] = hi[0];
    f[3] = hi[1];
}

// One BM x BN output tile (tm, tn) of the problem in `a`, computed by one
// workgroup of 64 * WM * WN threads with `sm` as its LDS.
template <int BM, int BN, int BK, int WM, int WN, int FT, bool INJ>
__device__ __forceinline__ void tile(const LaunchArgs& a, int tm, int tn, SmemFP8<BM, BN, BK, WM, WN>& sm) {
    using G = Geometry<BM, BN, WM, WN>;
    constexpr int NT = G::NT, TM = G::TM, TN = G::TN, MI = G::MI, NI = G::NI;
    constexpr int KP = OperandsFP8<BM, BN, BK>::KP;
    // A: an 8-row x 4-k block per thread (rows 8 ac.., k 4 akq..), the 16
    // k-quads of the panel on consecutive lanes.  The transposed stores of a
    // block go to 8 rows 8 ac + r; rows 8 apart are 640 bytes apart, the same
    // LDS bank, so lanes with different ac but the same k-quad would all
    // write one bank.  With the k-quad on the low lane bits the 16 lanes of a
    // store group write 16 consecutive dwords of one row (no conflict).  A
    // global load of a wave then reads 32 contiguous bytes of each of 16
    // columns.  B: 16-byte k-chunks (16 k of one column).
    constexpr int ARB = BM / 8;                 // row blocks of the A panel
    constexpr int AKQ = BK / 4;                 // k-quads per panel
    constexpr int BKC = BK / 16;                // k-chunks per column
    constexpr int NB = BN * BKC / NT;           // B chunks per thread
    static_assert(G::SPLIT, "the fp8 kernel assumes one owned row or column per thread");
    static_assert(ARB * AKQ == NT && AKQ == 16, "one A block per thread, the 16 k-quads on lane bits 0-3");
    static_assert(NB >= 1 && NT % BKC == 0 && BK % 16 == 0 && BKC == 4, "B chunk mapping");
    static_assert(BM == BN, "owner addressing assumes square tiles");

    OperandsFP8<BM, BN, BK>& op = sm.op;

    const Thread th = make_thread<G, (FT > 0)>(a, tm, tn);
    const int tid = th.tid, lane = th.lane, wm = th.wm, wn = th.wn, l32 = th.l32, hh = th.hh;
    const int mI = th.mI, nJ = th.nJ;
    const int nk = (a.K + BK - 1) / BK;
    const unsigned char* A = static_cast<const unsigned char*>(static_cast<const void*>(a.A));
    const unsigned char* B = static_cast<const unsigned char*>(static_cast<const void*>(a.B));

    const bool alignA = ((reinterpret_cast<uintptr_t>(A) & 7) == 0) && ((a.lda & 7) == 0);
    const bool alignB = ((reinterpret_cast<uintptr_t>(B) & 15) == 0) && ((a.ldb & 15) == 0);

    if constexpr (FT > 0) {
        for (int x = tid; x < 3 * BK; x += NT) {
            (&op.wsum[0][0])[x] = 0.f;
            (&op.vsum[0][0])[x] = 0.f;
        }
        clear_check(sm.ck, tid);
    }
    int fnext = 0, flogged = 0;
    if constexpr (INJ) gather_faults<G>(sm.ck, a, th);
    __syncthreads();

    // ---- global -> register staging ----
    // The plain kernel keeps two staging sets and loads two k-steps ahead: a
    // 64-k FP8 step is too short to cover the global load latency with one.
    // The FT kernels have no registers for a second set.
    constexpr int NS = FT == 0 ? 2 : 1;
    const int akq = tid % AKQ, ac = tid / AKQ;     // A block: rows 8 ac.., k 4 akq..
    u32x2 ras[NS][4];                               // 4 k-columns x 8 rows (bytes)
    u32x4 rbs[NS][NB];                              // 16 k of one column each
    const unsigned char* Abase = A + th.i0;
    const unsigned char* Bbase = B + (size_t)th.j0 * a.ldb;

    // Interior panels: buffer loads with per-lane byte offsets fixed for the
    // whole k-loop and the per-step origin in the scalar resource base (no
    // vector address arithmetic in the loop), while the offsets fit in 31 bits.
    const bool bufA = alignA && (int64_t)BK * a.lda < (int64_t(1) << 31);
    const bool bufB = alignB && (int64_t)BN * a.ldb < (int64_t(1) << 31);
    const int voffA = 4 * akq * (int)a.lda + 8 * ac;
    int voffB[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        const int f = tid + NT * r;
        voffB[r] = (f / BKC) * (int)a.ldb + 16 * (f % BKC);
    }
    constexpr int kRsrcWord3 = 0x00020000;   // raw 32-bit data format

    // The plain 256 x 256 kernel keeps the per-lane staging indices above for
    // the whole k-loop.  The FT kernels and the 128 x 128 tile (which the
    // batched kernel compiles beside its other tile variants) re-derive them
    // from opaque_tid() inside every step, which frees their registers for the
    // encodings (online 8192^3 2.03 -> 1.86 ms); re-deriving them cost the
    // plain kernel 5%.
    constexpr bool OPQ = BM == 128 || FT > 0;

    auto load_panels = [&](int t, auto set) {
        u32x2* ra = ras[decltype(set)::value];
        u32x4* rb = rbs[decltype(set)::value];
        const int tid_s = OPQ ? opaque_tid() : tid;
        const int akq_s = OPQ ? tid_s % AKQ : akq, ac_s = OPQ ? tid_s / AKQ : ac;
        const int voffA_s = OPQ ? 4 * akq_s * (int)a.lda + 8 * ac_s : voffA;
        const int k0 = t * BK;
        const bool fullk = k0 + BK <= a.K;
        // the edge paths take their k origin through an empty asm so that the
        // loop optimiser cannot turn their per-element pointers into
        // induction variables advanced on every step of the interior path
        int k0e = k0;
        asm volatile("" : "+s"(k0e));
        if (bufA && fullk && mI == BM) {
            const auto rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<unsigned char*>(Abase + (size_t)k0 * a.lda), (short)0, 0x7fffffff, kRsrcWord3);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                ra[e] = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, voffA_s, e * (int)a.lda, 0));
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gk = k0e + 4 * akq_s + e, gi = 8 * ac_s;
                const unsigned char* p = Abase + (size_t)gk * a.lda + gi;
                unsigned v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const bool in = gk < a.K && gi + q < mI;
                    const unsigned x = *(in ? p + q : A);
                    v[q] = in ? x : 0u;
                }
                ra[e][0] = v[0] | (v[1] << 8) | (v[2] << 16) | (v[3] << 24);
                ra[e][1] = v[4] | (v[5] << 8) | (v[6] << 16) | (v[7] << 24);
            }
        }
        if (bufB && fullk && nJ == BN) {
            const auto rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char*>(Bbase + k0), (short)0,
                                                              0x7fffffff, kRsrcWord3);
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                const int f = tid_s + NT * r;
                const int voffB_s = OPQ ? (f / BKC) * (int)a.ldb + 16 * (f % BKC) : voffB[r];
                rb[r] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voffB_s, 0, 0));
            }
        } else {
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                const int f = tid_s + NT * r;
                const int kc = f % BKC, jj = f / BKC;
                const int gk = k0e + 16 * kc;
                const unsigned char* p = Bbase + (size_t)jj * a.ldb + gk;
                unsigned v[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const bool in = jj < nJ && gk + q < a.K;
                    const unsigned x = *(in ? p + q : B);
                    v[q] = in ? x : 0u;
                }
#pragma unroll
                for (int d = 0; d < 4; ++d)
                    rb[r][d] = v[4 * d] | (v[4 * d + 1] << 8) | (v[4 * d + 2] << 16) | (v[4 * d + 3] << 24);
            }
        }
    };

    // registers -> LDS (A transposed to k-contiguous rows)
    auto store_panels = [&](int buf, auto set) {
        const u32x2* ra = ras[decltype(set)::value];
        const u32x4* rb = rbs[decltype(set)::value];
        const int tid_s = OPQ ? opaque_tid() : tid;
        const int akq_s = OPQ ? tid_s % AKQ : akq, ac_s = OPQ ? tid_s / AKQ : ac;
        // column e of the block holds rows 8 ac .. 8 ac + 7 as bytes; row r
        // gathers byte r of the 4 columns into one dword (k 4 akq .. +3).
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int d = r >> 2, sh = 8 * (r & 3);
            const unsigned w = ((ra[0][d] >> sh) & 0xffu) | (((ra[1][d] >> sh) & 0xffu) << 8) |
                               (((ra[2][d] >> sh) & 0xffu) << 16) | (((ra[3][d] >> sh) & 0xffu) << 24);
            *reinterpret_cast<unsigned*>(&op.As[buf][8 * ac_s + r][4 * akq_s]) = w;
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int f = tid_s + NT * r;
            const int kc = f % BKC, jj = f / BKC;
            *reinterpret_cast<u32x4*>(&op.Bs[buf][jj][16 * kc]) = rb[r];
        }
    };
    // the encodings e^T A and B e of the staged panels in FP32 (section 2.2,
    // Eq. 1-2), from the staging registers: in the 256 x 256 kernels one
    // sub-step after the LDS stores (after the step's last MFMAs, 5% faster
    // online at 8192^3), in the 128 x 128 tile, which the batched kernel also
    // holds, right after them
    auto encode_panels = [&](int slot, auto set) {
        const u32x2* ra = ras[decltype(set)::value];
        const u32x4* rb = rbs[decltype(set)::value];
        if constexpr (FT > 0) {
            const int tid_s = OPQ ? opaque_tid() : tid;
            const int lane_s = OPQ ? tid_s & 63 : lane, akq_s = OPQ ? tid_s % AKQ : akq;
            // e^T A for the thread's 4 k over its 8 rows, then over the 4
            // lanes of the same k-quad in the wave (bits 4, 5): the
            // reduce-scatter leaves k = 4 akq + ((lane >> 4) & 3); waves add
            // in LDS.
            float ws[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float f0[4], f1[4];
                decode4(ra[e][0], f0);
                decode4(ra[e][1], f1);
                ws[e] = ((f0[0] + f0[1]) + (f0[2] + f0[3])) + ((f1[0] + f1[1]) + (f1[2] + f1[3]));
            }
            ReduceScatter<4, 5, 4>::run(ws, lane_s);
            atomicAdd(&op.wsum[slot][4 * akq_s + ((lane_s >> 4) & 3)], ws[0]);
            // B e for the thread's 16 k over its NB columns, then over the
            // lanes of the same k-chunk (bits 2..5): lane keeps
            // k = 16 kc + ((lane >> 2) & 15); waves add in LDS.
            float vs[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) vs[q] = 0.f;
#pragma unroll
            for (int r = 0; r < NB; ++r)
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    float f[4];
                    decode4(rb[r][d], f);
#pragma unroll
                    for (int q = 0; q < 4; ++q) vs[4 * d + q] += f[q];
                }
            ReduceScatter<16, 5, 2>::run(vs, lane_s);
            atomicAdd(&op.vsum[slot][16 * (tid_s % BKC) + ((lane_s >> 2) & 15)], vs[0]);
        }
    };

    Acc<G> acc;
#pragma unroll
    for (int bi = 0; bi < MI; ++bi)
#pragma unroll
        for (int bj = 0; bj < NI; ++bj)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[bi][bj][r] = 0.0f;

    // owned checksum vector: a row of A (with B e) or a column of B (with
    // e^T A); both are k-contiguous rows of the LDS panels
    float ck0 = 0.f, nq0 = 0.f;
    float& Rr = ck0;
    float& na2 = nq0;
    float& Sc = ck0;
    float& nb2 = nq0;
    const bool row_role = th.row_role;
    const int own = row_role ? min(tid, BM - 1) : min(max(tid - G::COL0, 0), BN - 1);
    const unsigned char* const x_arr = row_role ? &op.As[0][0][0] : &op.Bs[0][0][0];
    constexpr int XBUF = BM * KP;   // == BN * KP

    // The whole 64-k step is one v_mfma_scale_f32_32x32x64_f8f6f4 per block
    // (E4M3 operands, unit block scales): lane l supplies 32 consecutive k
    // (32 bytes, two 16-byte LDS reads) of one row, the lane halves taking
    // k 0..31 and 32..63.  Both operands are read with the same lane -> k
    // assignment, so every product pairs a_ik with b_kj.  The step has four
    // sub-steps of 16 k for the checksum update; sub-step s issues the MFMAs
    // of row block s (none when the wavefront has fewer than s + 1 row
    // blocks); the column-block fragments are read at s = 0 and kept for the
    // step.
    static_assert(MI <= BK / 16 && BK == 64, "at most one row block per sub-step, one MFMA per block per step");
    typedef int i32x8 __attribute__((ext_vector_type(8)));
    constexpr int kScaleOne = 127;   // E8M0 block scale 2^0
    i32x8 bxk[NI];
    auto frag = [&](const unsigned char* p) {
        const u32x4 lo = *reinterpret_cast<const u32x4*>(p);
        const u32x4 hi = *reinterpret_cast<const u32x4*>(p + 16);
        return i32x8{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
    };
    auto mfma_sub = [&](int cur, int s) {
        if (s == 0) {
#pragma unroll
            for (int bj = 0; bj < NI; ++bj) bxk[bj] = frag(&op.Bs[cur][wn * TN + 32 * bj + l32][32 * hh]);
        }
        const i32x8 ay = frag(&op.As[cur][wm * TM + 32 * s + l32][32 * hh]);
#pragma unroll
        for (int bj = 0; bj < NI; ++bj)
            acc[s][bj] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(bxk[bj], ay, acc[s][bj], 0, 0, 0, kScaleOne,
                                                                        0, kScaleOne);
    };

    // reference checksum update (Eq. 4) for the same 16 k
    auto ft_sub = [&](int cur, int slot, int s) {
        const unsigned char* px = x_arr + cur * XBUF + own * KP + 16 * s;
        const float* py = row_role ? &op.vsum[slot][16 * s] : &op.wsum[slot][16 * s];
        const u32x4 xv = *reinterpret_cast<const u32x4*>(px);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const f32x4 y = *reinterpret_cast<const f32x4*>(py + 4 * d);
            float x[4];
            decode4(xv[d], x);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ck0 = fmaf(x[q], y[q], ck0);
                nq0 = fmaf(x[q], x[q], nq0);
            }
        }
    };

    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, NS - 1>;
    // One k-step.  NEXT: store the staged panels of step t + 1 (set `held`).
    // FT kernels load step t + 1 into their one set first; the plain kernel
    // loads step t + 2 (if any) into the other set.
    auto step = [&](int t, auto has_next, auto held) {
        constexpr bool NEXT = decltype(has_next)::value;
        constexpr int H = decltype(held)::value;
        const int cur = t & 1;
        if constexpr (NS == 1) {
            if constexpr (NEXT) load_panels(t + 1, S0{});
        } else {
            if (t + 2 < nk) load_panels(t + 2, std::integral_constant<int, 1 - H>{});
        }
        if constexpr (FT > 0 && NEXT) {   // slot for step t+2: its last reader finished before this step
            const int tz = OPQ ? opaque_tid() : tid, x = tz < BK ? tz : BK - 1;
            op.wsum[(t + 2) % 3][x] = 0.f;
            op.vsum[(t + 2) % 3][x] = 0.f;
        }
#pragma unroll
        for (int s = 0; s < BK / 16; ++s) {
            if (s < MI) mfma_sub(cur, s);
            if constexpr (FT > 0) ft_sub(cur, t % 3, s);
            if constexpr (NEXT) {
                if (s == BK / 16 - 2) store_panels(cur ^ 1, held);
                if (s == (BM == 256 ? BK / 16 - 1 : BK / 16 - 2)) encode_panels((t + 1) % 3, held);
            }
        }
    };

    // injection hook and online check after k-step t.  The detect-only level
    // has the same loop: the host sets its check interval beyond the last
    // k-step, so it checks once, after the last step.
    auto post = [&](int t) -> bool {
        if constexpr (INJ) inject<G>(acc, sm.ck, a, th, t, fnext);
        bool do_check = false;
        if constexpr (FT > 0) do_check = ((t + 1) % a.check_interval == 0) || (t == nk - 1);
        if (do_check) check<G, FT, INJ>(acc, sm.ck, a, th, t, min((t + 1) * BK, a.K), Rr, na2, Sc, nb2, fnext, flogged);
        return do_check;
    };

    load_panels(0, S0{});
    store_panels(0, S0{});
    encode_panels(0, S0{});
    if constexpr (NS == 2) {
        if (nk > 1) load_panels(1, S1{});
    }
    __syncthreads();
    int t = 0;
    if constexpr (NS == 1) {
        for (; t + 1 < nk; ++t) {
            step(t, std::true_type{}, S0{});
            if (!post(t)) __syncthreads();
        }
    } else {
        // steps in pairs, so that each step's staging set is a compile-time index
        for (; t + 2 < nk; t += 2) {
            step(t, std::true_type{}, S1{});
            if (!post(t)) __syncthreads();
            step(t + 1, std::true_type{}, S0{});
            if (!post(t + 1)) __syncthreads();
        }
        if (t + 1 < nk) {
            step(t, std::true_type{}, S1{});
            if (!post(t)) __syncthreads();
            ++t;
        }
    }
    step(nk - 1, std::false_type{}, S0{});
    post(nk - 1);
    finish_tile<G, FT>(acc, sm.ck, a, th, a.scale);
}

}  // namespace fp8
}  // namespace ftgemm_impl
