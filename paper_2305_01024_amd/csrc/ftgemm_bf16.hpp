// ftgemm_bf16.hpp -- BF16-input online ABFT GEMM kernels for gfx950 (MI355X).
//
// C = alpha * (scale_a * A) (scale_b * B) + beta * C with A, B in bfloat16 and
// FP32 accumulation on v_mfma_f32_32x32x16_bf16.  The fault tolerance is the
// same threadblock-level online ABFT as the FP32 kernels (section 2.2 Eq. 1-4,
// section 4.2.3): every bf16 value decodes exactly to FP32, so the encodings
// e^T A and B e, the reference checksums, the norms and the check all run in
// FP32 on the decoded operands, with the FP32 roundoff threshold.  The
// per-tensor scales are powers of two applied in the epilogue, outside the
// checked region.
//
// Layout: both operands sit in LDS k-contiguous ([row][k], 16-byte padded
// rows), which is what a 32x32x16 MFMA operand wants: lane l supplies 8
// consecutive k of one row.  B (column-major K x N) is k-contiguous already;
// A (column-major M x K) is i-contiguous, so each thread loads an 8-row x
// 4-k block and transposes it in registers (v_perm_b32) on the way to LDS.
// As in the FP32 kernels the MFMA computes P^T = B^T A^T, so lane l % 32 owns
// one row of C.
#pragma once

#include "ftgemm_abft.hpp"

namespace ftgemm_impl {
namespace bf16 {

using namespace abft;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

template <int BM, int BN, int BK>
struct alignas(16) OperandsBF16 {   // 16-byte aligned: the panel reads are 16-byte LDS loads
    static constexpr int KP = BK + 8;          // row pitch in bf16 (16 B of padding)
    unsigned short As[2][BM][KP];              // A panel, i-major, k contiguous
    unsigned short Bs[2][BN][KP];              // B panel, j-major, k contiguous
    float wsum[3][BK];                         // e^T A per k (accumulated across waves, 3 rotating slots)
    float vsum[3][BK];                         // B e per k (same)
    float dummy[64];
};

template <int BM, int BN, int BK, int WM, int WN>
struct SmemBF16 {
    OperandsBF16<BM, BN, BK> op;
    CheckLds<Geometry<BM, BN, WM, WN>> ck;
};

// bf16 halves of a packed dword, exactly as FP32
__device__ __forceinline__ float bf_lo(unsigned x) { return __uint_as_float(x << 16); }
__device__ __forceinline__ float bf_hi(unsigned x) { return __uint_as_float(x & 0xffff0000u); }

// x.lo * y.lo + x.hi * y.hi + acc with exact bf16 products (v_dot2_f32_bf16)
__device__ __forceinline__ float dot2(unsigned x, unsigned y, float acc) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, x), __builtin_bit_cast(bf16x2, y), acc, false);
}
// bf16 pairs (1, 1), (1, 0) and (0, 1) as dot2 selectors.  They reach the
// instruction through scalar registers: the compiler would otherwise fold
// (1, 0) into the inline constant 1.0, which the packed-bf16 operand does not
// read as (1, 0).
constexpr unsigned kBfOnes = 0x3f803f80u;
constexpr unsigned kBfLo = 0x00003f80u;     // the low half alone
constexpr unsigned kBfHi = 0x3f800000u;     // the high half alone
__device__ __forceinline__ unsigned opaque_sgpr(unsigned x) {
    asm volatile("" : "+s"(x));
    return x;
}

// One BM x BN output tile (tm, tn) of the problem in `a`, computed by one
// workgroup of 64 * WM * WN threads with `sm` as its LDS.
template <int BM, int BN, int BK, int WM, int WN, int FT, bool INJ>
__device__ __forceinline__ void tile(const LaunchArgs& a, int tm, int tn, SmemBF16<BM, BN, BK, WM, WN>& sm) {
    using G = Geometry<BM, BN, WM, WN>;
    constexpr int NT = G::NT, TM = G::TM, TN = G::TN, MI = G::MI, NI = G::NI;
    constexpr int KP = OperandsBF16<BM, BN, BK>::KP;
    // A: an 8-row x 4-k block per thread; B: 16-byte k-chunks (8 k of a column)
    constexpr int AKQ = BK / 4;                 // k-quads per panel
    constexpr int BKC = BK / 8;                 // k-chunks per column
    constexpr int NB = BN * BKC / NT;           // B chunks per thread
    static_assert(G::SPLIT, "the bf16 kernel assumes one owned row or column per thread");
    static_assert(BM / 8 * AKQ == NT, "one A block per thread");
    static_assert(NB >= 1 && NT % BKC == 0 && BK % 16 == 0, "B chunk mapping");
    static_assert(AKQ == 16 && BKC == 8, "encode lane mapping assumes BK = 64");

    OperandsBF16<BM, BN, BK>& op = sm.op;

    const Thread th = make_thread<G, (FT > 0)>(a, tm, tn);
    const int tid = th.tid, lane = th.lane, wm = th.wm, wn = th.wn, l32 = th.l32, hh = th.hh;
    const int mI = th.mI, nJ = th.nJ;
    const int nk = (a.K + BK - 1) / BK;
    const unsigned short* A = static_cast<const unsigned short*>(static_cast<const void*>(a.A));
    const unsigned short* B = static_cast<const unsigned short*>(static_cast<const void*>(a.B));

    const bool alignA = ((reinterpret_cast<uintptr_t>(A) & 15) == 0) && ((a.lda & 7) == 0);
    const bool alignB = ((reinterpret_cast<uintptr_t>(B) & 15) == 0) && ((a.ldb & 7) == 0);

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
    const int akq = tid % AKQ, ac = tid / AKQ;     // A block: rows 8ac.., k 4akq..
    u32x4 ra[4];                                    // 4 k-columns x 8 rows (bf16 pairs)
    u32x4 rb[NB];                                   // 8 k of one column each
    const unsigned short* Abase = A + th.i0;
    const unsigned short* Bbase = B + (size_t)th.j0 * a.ldb;

    // Interior panels: buffer loads with per-lane byte offsets fixed for the
    // whole k-loop and the per-step origin in the scalar resource base (no
    // vector address arithmetic in the loop), while the offsets fit in 31 bits.
    const bool bufA = alignA && (int64_t)BK * a.lda * 2 < (int64_t(1) << 31);
    const bool bufB = alignB && (int64_t)BN * a.ldb * 2 < (int64_t(1) << 31);
    const int voffA = (4 * akq * (int)a.lda + 8 * ac) * 2;
    int voffB[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        const int f = tid + NT * r;
        voffB[r] = ((f / BKC) * (int)a.ldb + 8 * (f % BKC)) * 2;
    }
    constexpr int kRsrcWord3 = 0x00020000;   // raw 32-bit data format

    // The per-lane staging indices above are kept for the whole k-loop by the
    // 256 x 256 kernels.  The 128 x 128 tile, which the batched kernel
    // compiles beside its other tile variants, re-derives them from
    // opaque_tid() inside every step: kept, they were spilled there and
    // reloaded at every step (re-deriving them in the 256 x 256 kernels cost
    // the plain kernel 13% at 8192^3).
    constexpr bool OPQ = BM == 128;
    auto load_panels = [&](int t) {
        const int tid_s = OPQ ? opaque_tid() : tid;
        const int akq_s = OPQ ? tid_s % AKQ : akq, ac_s = OPQ ? tid_s / AKQ : ac;
        const int voffA_s = OPQ ? (4 * akq_s * (int)a.lda + 8 * ac_s) * 2 : voffA;
        const int k0 = t * BK;
        const bool fullk = k0 + BK <= a.K;
        // the edge paths take their k origin through an empty asm so that the
        // loop optimiser cannot turn their per-element pointers into
        // induction variables advanced on every step of the interior path
        int k0e = k0;
        asm volatile("" : "+s"(k0e));
        if (bufA && fullk && mI == BM) {
            const auto rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<unsigned short*>(Abase + (size_t)k0 * a.lda), (short)0, 0x7fffffff, kRsrcWord3);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                ra[e] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voffA_s, e * (int)a.lda * 2, 0));
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gk = k0e + 4 * akq_s + e, gi = 8 * ac_s;
                const unsigned short* p = Abase + (size_t)gk * a.lda + gi;
                unsigned v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const bool in = gk < a.K && gi + q < mI;
                    const unsigned x = *(in ? p + q : A);
                    v[q] = in ? x : 0u;
                }
#pragma unroll
                for (int d = 0; d < 4; ++d) ra[e][d] = v[2 * d] | (v[2 * d + 1] << 16);
            }
        }
        if (bufB && fullk && nJ == BN) {
            const auto rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned short*>(Bbase + k0), (short)0,
                                                              0x7fffffff, kRsrcWord3);
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                const int f = tid_s + NT * r;
                const int voffB_s = OPQ ? ((f / BKC) * (int)a.ldb + 8 * (f % BKC)) * 2 : voffB[r];
                rb[r] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voffB_s, 0, 0));
            }
        } else {
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                const int f = tid_s + NT * r;
                const int kc = f % BKC, jj = f / BKC;
                const int gk = k0e + 8 * kc;
                const unsigned short* p = Bbase + (size_t)jj * a.ldb + gk;
                unsigned v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const bool in = jj < nJ && gk + q < a.K;
                    const unsigned x = *(in ? p + q : B);
                    v[q] = in ? x : 0u;
                }
#pragma unroll
                for (int d = 0; d < 4; ++d) rb[r][d] = v[2 * d] | (v[2 * d + 1] << 16);
            }
        }
    };

    // registers -> LDS (A transposed to k-contiguous rows)
    auto store_panels = [&](int buf) {
        const int tid_s = OPQ ? opaque_tid() : tid;
        const int akq_s = OPQ ? tid_s % AKQ : akq, ac_s = OPQ ? tid_s / AKQ : ac;
        // A: column e of the thread's block holds rows 8ac..8ac+7 as bf16
        // pairs; row r gathers element r of columns 0..3 into 8 bytes.
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int d = r >> 1;
            const unsigned sel = (r & 1) ? 0x07060302u : 0x05040100u;   // high or low halves
            u32x2 w;
            w[0] = __builtin_amdgcn_perm(ra[1][d], ra[0][d], sel);
            w[1] = __builtin_amdgcn_perm(ra[3][d], ra[2][d], sel);
            *reinterpret_cast<u32x2*>(&op.As[buf][8 * ac_s + r][4 * akq_s]) = w;
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int f = tid_s + NT * r;
            const int kc = f % BKC, jj = f / BKC;
            *reinterpret_cast<u32x4*>(&op.Bs[buf][jj][8 * kc]) = rb[r];
        }
    };
    // the encodings e^T A and B e of the staged panels in FP32 (section 2.2,
    // Eq. 1-2), from the staging registers.  The 256 x 256 FT kernels run
    // them one sub-step after the LDS stores, after the step's last MFMAs (5%
    // faster online at 8192^3 than right after the stores); the 128 x 128
    // tile, which the batched kernel also holds, right after the stores (the
    // later placement doubles the batched kernel's spills).
    auto encode_panels = [&](int slot) {
        if constexpr (FT > 0) {
            const int tid_s = OPQ ? opaque_tid() : tid;
            const int lane_s = OPQ ? tid_s & 63 : lane, akq_s = OPQ ? tid_s % AKQ : akq;
            // one v_dot2 per packed pair (an FP32 add of an exact product)
            const unsigned sel_ones = opaque_sgpr(kBfOnes), sel_lo = opaque_sgpr(kBfLo), sel_hi = opaque_sgpr(kBfHi);
            // e^T A for the thread's 4 k over its 8 rows, then over the 32
            // threads of the same k-quad: lane bits 4, 5 in-wave (reduce-
            // scatter leaves k = 4 akq + ((lane >> 4) & 3)), waves in LDS.
            float ws[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float x = 0.f;
#pragma unroll
                for (int d = 0; d < 4; ++d) x = dot2(ra[e][d], sel_ones, x);
                ws[e] = x;
            }
            ReduceScatter<4, 5, 4>::run(ws, lane_s);
            atomicAdd(&op.wsum[slot][4 * akq_s + ((lane_s >> 4) & 3)], ws[0]);
            // B e for the thread's 8 k over its NB columns, then over the
            // lanes of the same k-chunk (bits 3..5): lane keeps
            // k = 8 kc + ((lane >> 3) & 7); waves add in LDS.
            float vs[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) vs[q] = 0.f;
#pragma unroll
            for (int r = 0; r < NB; ++r)
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    vs[2 * d] = dot2(rb[r][d], sel_lo, vs[2 * d]);
                    vs[2 * d + 1] = dot2(rb[r][d], sel_hi, vs[2 * d + 1]);
                }
            ReduceScatter<8, 5, 3>::run(vs, lane_s);
            atomicAdd(&op.vsum[slot][8 * (tid_s % BKC) + ((lane_s >> 3) & 7)], vs[0]);
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
    const unsigned short* const x_arr = row_role ? &op.As[0][0][0] : &op.Bs[0][0][0];
    constexpr int XBUF = BM * KP;   // == BN * KP (square tiles)
    static_assert(BM == BN, "owner addressing assumes square tiles");

    // operand fragments of sub-step s (16 k) of buffer `cur`
    auto load_frags = [&](int cur, int s, bf16x8* bx, bf16x8* ay) {
#pragma unroll
        for (int bj = 0; bj < NI; ++bj)
            bx[bj] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(
                                                    &op.Bs[cur][wn * TN + 32 * bj + l32][16 * s + 8 * hh]));
#pragma unroll
        for (int bi = 0; bi < MI; ++bi)
            ay[bi] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(
                                                    &op.As[cur][wm * TM + 32 * bi + l32][16 * s + 8 * hh]));
    };
    // The plain kernel reads the fragments of sub-step s + 1 before issuing
    // the MFMAs of sub-step s (within a k-step); the FT kernels have no
    // registers to spare for the second set.
    bf16x8 bxq[2][NI], ayq[2][MI];

    // one k16 sub-step: an MFMA on every block of the wave tile
    auto mfma_sub = [&](int cur, int s) {
        bf16x8 bxl[NI], ayl[MI];
        bf16x8* bx = bxl;
        bf16x8* ay = ayl;
        if constexpr (FT == 0) {
            if (s == 0) load_frags(cur, 0, bxq[0], ayq[0]);
            if (s + 1 < BK / 16) load_frags(cur, s + 1, bxq[(s + 1) & 1], ayq[(s + 1) & 1]);
            bx = bxq[s & 1];
            ay = ayq[s & 1];
        } else {
            load_frags(cur, s, bxl, ayl);
        }
#pragma unroll
        for (int bi = 0; bi < MI; ++bi)
#pragma unroll
            for (int bj = 0; bj < NI; ++bj)
                acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bx[bj], ay[bi], acc[bi][bj], 0, 0, 0);
    };

    // reference checksum update (Eq. 4) for the same 16 k
    auto ft_sub = [&](int cur, int slot, int s) {
        const unsigned short* px = x_arr + cur * XBUF + own * KP + 16 * s;
        const float* py = row_role ? &op.vsum[slot][16 * s] : &op.wsum[slot][16 * s];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const u32x4 xv = *reinterpret_cast<const u32x4*>(px + 8 * h);
            const f32x4 y0 = *reinterpret_cast<const f32x4*>(py + 8 * h);
            const f32x4 y1 = *reinterpret_cast<const f32x4*>(py + 8 * h + 4);
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const float lo = bf_lo(xv[d]), hi = bf_hi(xv[d]);
                const float ylo = d < 2 ? y0[2 * d] : y1[2 * d - 4];
                const float yhi = d < 2 ? y0[2 * d + 1] : y1[2 * d - 3];
                ck0 = fmaf(lo, ylo, ck0);
                ck0 = fmaf(hi, yhi, ck0);
                // both squares of the packed pair in one v_dot2 (bf16 products are exact)
                nq0 = dot2(xv[d], xv[d], nq0);
            }
        }
    };

    auto step = [&](int t, auto has_next) {
        constexpr bool NEXT = decltype(has_next)::value;
        const int cur = t & 1;
        if constexpr (NEXT) load_panels(t + 1);
        if constexpr (FT > 0 && NEXT) {   // slot for step t+2: its last reader finished before this step
            const int tz = OPQ ? opaque_tid() : tid, x = tz < BK ? tz : BK - 1;
            op.wsum[(t + 2) % 3][x] = 0.f;
            op.vsum[(t + 2) % 3][x] = 0.f;
        }
#pragma unroll
        for (int s = 0; s < BK / 16; ++s) {
            mfma_sub(cur, s);
            if constexpr (FT > 0) ft_sub(cur, t % 3, s);
            if constexpr (NEXT) {
                if (s == BK / 16 - 2) store_panels(cur ^ 1);
                if (s == (BM == 256 ? BK / 16 - 1 : BK / 16 - 2)) encode_panels((t + 1) % 3);
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

    load_panels(0);
    store_panels(0);
    encode_panels(0);
    __syncthreads();
    for (int t = 0; t + 1 < nk; ++t) {
        step(t, std::true_type{});
        if (!post(t)) __syncthreads();
    }
    step(nk - 1, std::false_type{});
    post(nk - 1);
    finish_tile<G, FT>(acc, sm.ck, a, th, a.scale);
}

}  // namespace bf16
}  // namespace ftgemm_impl
