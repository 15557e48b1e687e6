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
#include "ftgemm_abft.hpp"

namespace ftgemm_impl {
namespace {

using namespace abft;

template <int BM, int BN, int BK>
struct Operands {
    float As[2][BK][BM];        // A panel, k-major (i contiguous)
    float Bs[2][BN][BK + 4];    // B panel, j-major (k contiguous), padded: conflict-free 16 B reads
    float wsum[2][BK];          // e^T A of the panel, per k
    float vsum[3][BK];          // B e of the panel, per k (accumulated across waves, 3 rotating slots)
    float dummy[256];           // sink for the stores/atomics of lanes that own no value
};

template <int BM, int BN, int BK, int WM, int WN>
struct Smem {
    Operands<BM, BN, BK> op;
    CheckLds<Geometry<BM, BN, WM, WN>> ck;
};

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------
template <int BM, int BN, int BK, int WM, int WN, int FT, bool INJ>
__global__ __launch_bounds__(64 * WM * WN) void ftgemm_f32_kernel(LaunchArgs a) {
    using G = Geometry<BM, BN, WM, WN>;
    constexpr int NT = G::NT, TM = G::TM, TN = G::TN, MI = G::MI, NI = G::NI;
    constexpr int NA = BM * BK / (4 * NT);     // float4 slots of A per thread
    constexpr int NB = BN * BK / (4 * NT);     // float4 slots of B per thread
    constexpr int AG = (BM / 4 < 64) ? BM / 4 : 64;   // lanes sharing one k in the A load
    constexpr int BKQ = BK / 4;                       // lanes sharing one column in the B load
    constexpr bool SPLIT = G::SPLIT;
    constexpr int COL0 = G::COL0;
    static_assert(NA >= 1 && NB >= 1 && BK % 8 == 0, "tile shape");
    static_assert(NT % (BM / 4) == 0 || (BM / 4) % 64 == 0, "A slot mapping");
    static_assert(NT % BKQ == 0 && 64 % BKQ == 0 && BKQ <= 16, "B slot mapping");
    static_assert(NA <= AG, "encode reduce-scatter needs NA <= AG");

    __shared__ Smem<BM, BN, BK, WM, WN> sm;
    Operands<BM, BN, BK>& op = sm.op;

    const int ntm = (a.M + BM - 1) / BM;
    const Thread th = make_thread<G>(a, blockIdx.x % ntm, blockIdx.x / ntm);
    const int tid = th.tid, lane = th.lane, wm = th.wm, wn = th.wn, l32 = th.l32, hh = th.hh;
    const int mI = th.mI, nJ = th.nJ;
    const int nk = (a.K + BK - 1) / BK;

    const bool alignA = ((reinterpret_cast<uintptr_t>(a.A) & 15) == 0) && ((a.lda & 3) == 0);
    const bool alignB = ((reinterpret_cast<uintptr_t>(a.B) & 15) == 0) && ((a.ldb & 3) == 0);

    if constexpr (FT > 0) {
        for (int x = tid; x < 3 * BK; x += NT) (&op.vsum[0][0])[x] = 0.f;
    }
    int fnext = 0, flogged = 0;
    if constexpr (INJ) gather_faults<G>(sm.ck, a, th);
    __syncthreads();

    // ---- global -> register staging of one k-step's panels ----
    f32x4 ra[NA], rb[NB];
    const float* Abase = a.A + th.i0;
    const float* Bbase = a.B + (size_t)th.j0 * a.ldb;

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
            *reinterpret_cast<f32x4*>(&op.As[buf][kk][4 * i4]) = ra[r];
            ws[r] = (ra[r][0] + ra[r][1]) + (ra[r][2] + ra[r][3]);
        }
        f32x4 vp = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int f = tid + NT * r;
            const int kq = f % BKQ, jj = f / BKQ;
            *reinterpret_cast<f32x4*>(&op.Bs[buf][jj][4 * kq]) = rb[r];
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
                float* dst = ((lane & ((1 << WSH) - 1)) == 0) ? &op.wsum[buf][kk] : &op.dummy[lane];
                *dst = ws[0];
            }
            // B e: the 4 k of k-quad (lane % BKQ) are summed over the lanes of
            // that quad (bits log2(BKQ)..5); lane keeps k = 4 (lane % BKQ) +
            // ((lane >> 4) & 3); waves then add their partials in LDS.
            float vx[4] = {vp[0], vp[1], vp[2], vp[3]};
            ReduceScatter<4, 5, ilog2(BKQ)>::run(vx, lane);
            const int kv = 4 * (lane % BKQ) + ((lane >> 4) & 3);
            float* dst = ((lane & (16 - BKQ)) == 0) ? &op.vsum[vslot][kv] : &op.dummy[lane];
            atomicAdd(dst, vx[0]);
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
    const int x0_stride = row_role ? BM : 1;
    const int x0_off = row_role ? min(tid, BM - 1) : min(max(tid - COL0, 0), BN - 1) * (BK + 4);
    const int x0_buf = row_role ? BK * BM : BN * (BK + 4);
    const float* const x0_arr = row_role ? &op.As[0][0][0] : &op.Bs[0][0][0];
    const int x1_row = min(tid, BN - 1);
    // one group of 8 k: 4 MFMA k-substeps on every block of the wave tile
    auto mfma_group = [&](int cur, int g) {
        f32x4 bf[NI];
#pragma unroll
        for (int bj = 0; bj < NI; ++bj)
            bf[bj] = *reinterpret_cast<const f32x4*>(&op.Bs[cur][wn * TN + 32 * bj + l32][8 * g + 4 * hh]);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            float af[MI];
#pragma unroll
            for (int bi = 0; bi < MI; ++bi) af[bi] = op.As[cur][8 * g + 4 * hh + s][wm * TM + 32 * bi + l32];
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
        const float* py = row_role ? &op.vsum[vcur][8 * g] : &op.wsum[cur][8 * g];
        const f32x4 ya = *reinterpret_cast<const f32x4*>(py);
        const f32x4 yb = *reinterpret_cast<const f32x4*>(py + 4);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float x = px[q * x0_stride];
            ck0 = fmaf(x, q < 4 ? ya[q] : yb[q - 4], ck0);
            nq0 = fmaf(x, x, nq0);
        }
        if constexpr (!SPLIT) {
            const f32x4 b0 = *reinterpret_cast<const f32x4*>(&op.Bs[cur][x1_row][8 * g]);
            const f32x4 b1 = *reinterpret_cast<const f32x4*>(&op.Bs[cur][x1_row][8 * g + 4]);
            const f32x4 w0 = *reinterpret_cast<const f32x4*>(&op.wsum[cur][8 * g]);
            const f32x4 w1 = *reinterpret_cast<const f32x4*>(&op.wsum[cur][8 * g + 4]);
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
            (&op.vsum[(t + 2) % 3][0])[tid < BK ? tid : BK - 1] = 0.f;
#pragma unroll
        for (int g = 0; g < BK / 8; ++g) {
            mfma_group(cur, g);
            if constexpr (FT > 0) ft_group(cur, t % 3, g);
            if constexpr (NEXT) {
                if (g == (BK / 8 >= 2 ? BK / 8 - 2 : 0)) store_panels(cur ^ 1, (t + 1) % 3);
            }
        }
    };

    auto post = [&](int t) -> bool {   // injection hook and check after k-step t
        if constexpr (INJ) inject<G>(acc, sm.ck, a, th, t, fnext);
        bool do_check = false;
        if constexpr (FT == 2) do_check = ((t + 1) % a.check_interval == 0) || (t == nk - 1);
        if constexpr (FT == 1) do_check = (t == nk - 1);
        if (do_check) check<G, FT, INJ>(acc, sm.ck, a, th, t, min((t + 1) * BK, a.K), Rr, na2, Sc, nb2, fnext, flogged);
        return do_check;
    };

    load_panels(0);
    store_panels(0, 0);
    __syncthreads();
    for (int t = 0; t + 1 < nk; ++t) {
        step(t, std::true_type{});
        // a check ends with a workgroup barrier after its census, which also
        // orders this step's LDS panel writes before the next step's reads
        if (!post(t)) __syncthreads();
    }
    step(nk - 1, std::false_type{});
    post(nk - 1);
    epilogue<G>(acc, a, th, 1.0f);
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
