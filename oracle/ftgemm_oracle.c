/*
 * ftgemm_oracle.c -- plain FP64 CPU oracle for online ABFT GEMM.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library
 * and its Python binding) may load, call or link this file.  It is used by
 * the test suite, by the smoke check and by the CPU-baseline leg of the
 * benchmark, and it shares no code, header, table or helper with the GPU
 * library.
 *
 * What it computes follows Wu et al., "Anatomy of High-Performance GEMM with
 * Online Fault Tolerance on GPUs" (ICS'23, arXiv:2305.01024):
 *   - the plain product C = alpha*A*B + beta*C0 (section 3.1, the device-level
 *     C += A*B, here with the BLAS alpha/beta epilogue);
 *   - the Huang-Abraham checksum encodings e^T A and B e (section 2.2,
 *     Eq. 1-2) and the checksum relation of the encoded product (Eq. 3);
 *   - the outer-product online form in which the relation holds after every
 *     rank-k_s update, so a check after each step can correct one error per
 *     step (section 2.2, Eq. 4);
 *   - location of a single error at the intersection of the offending row
 *     and column and its correction from the checksum (section 4.2.1 and
 *     section 5.3).
 * The paper leaves the detection threshold unstated (section 2.2 fixes it in
 * advance without a value).  The oracle uses the analytic roundoff bound
 *   beta_row_i = 2u (K' + n_J + 1) ||a_i[0:K']||_2 * sum_{j in J} ||b_j[0:K']||_2
 *   beta_col_j = 2u (K' + m_I + 1) ||b_j[0:K']||_2 * sum_{i in I} ||a_i[0:K']||_2
 * with tau = c * beta, u the unit roundoff of the modelled GPU arithmetic and
 * K' the number of k indices accumulated so far (a standard gamma_n bound
 * for any-order summation, turned into norms by Cauchy-Schwarz).
 *
 * The paper's checks assume finite operands (its fault model, section 4.1,
 * covers errors in the computation, not in the data).  A tile whose operands
 * hold Inf or NaN has non-finite norms, references and bounds, so no check
 * can separate rounding from a fault there: the replay reports such a tile
 * once (kind ORACLE_EV_NONFINITE, at the first check that sees the value),
 * locates and corrects nothing in it, and leaves its part of C to IEEE
 * arithmetic.
 *
 * All arithmetic is FP64.  Matrices are column-major with leading
 * dimensions, as in BLAS.  Parallelism is OpenMP over independent output
 * columns (plain GEMM) or output tiles (replay); every per-element sum runs
 * in ascending k order.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define AT(M, ld, r, c) ((M)[(size_t)(r) + (size_t)(c) * (size_t)(ld)])

/* ------------------------------------------------------------------------ */
/* Plain GEMM (section 3.1): C = alpha * A * B + beta * C0, column-major.    */
/* beta == 0 means C0 is not read (BLAS convention); k == 0 or alpha == 0     */
/* gives C = beta * C0.  Returns 0, or minus the 1-based position of the      */
/* first invalid argument.                                                    */
/* ------------------------------------------------------------------------ */
int oracle_gemm(int64_t m, int64_t n, int64_t k, double alpha,
                const double* A, int64_t lda, const double* B, int64_t ldb,
                double beta, double* C, int64_t ldc)
{
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (k < 0) return -3;
    if (lda < (m > 1 ? m : 1)) return -6;
    if (ldb < (k > 1 ? k : 1)) return -8;
    if (ldc < (m > 1 ? m : 1)) return -11;
    if (m == 0 || n == 0) return 0;

    #pragma omp parallel
    {
        double* col = (double*)malloc((size_t)m * sizeof(double));
        #pragma omp for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            for (int64_t i = 0; i < m; ++i) col[i] = 0.0;
            if (alpha != 0.0) {
                /* col[i] = sum_{p=0}^{k-1} A[i,p] * B[p,j], p ascending */
                for (int64_t p = 0; p < k; ++p) {
                    const double b = AT(B, ldb, p, j);
                    for (int64_t i = 0; i < m; ++i) col[i] += AT(A, lda, i, p) * b;
                }
            }
            for (int64_t i = 0; i < m; ++i) {
                const double c0 = (beta == 0.0) ? 0.0 : beta * AT(C, ldc, i, j);
                AT(C, ldc, i, j) = alpha * col[i] + c0;
            }
        }
        free(col);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Checksum encodings (section 2.2, Eq. 1 and Eq. 2).                         */
/*   column checksum of A:  w[p] = sum_{i < rows} A[i, p]   (row of e^T A)   */
/*   row checksum of B:     v[p] = sum_{j < cols} B[p, j]   (column of B e)  */
/* ------------------------------------------------------------------------ */
void oracle_encode_col(int64_t rows, int64_t kcount, const double* A, int64_t lda, double* w)
{
    for (int64_t p = 0; p < kcount; ++p) {
        double s = 0.0;
        for (int64_t i = 0; i < rows; ++i) s += AT(A, lda, i, p);
        w[p] = s;
    }
}

void oracle_encode_row(int64_t kcount, int64_t cols, const double* B, int64_t ldb, double* v)
{
    for (int64_t p = 0; p < kcount; ++p) {
        double s = 0.0;
        for (int64_t j = 0; j < cols; ++j) s += AT(B, ldb, p, j);
        v[p] = s;
    }
}

/* Detection bound (see the header comment).  kprime = k indices accumulated,
 * count = number of terms in the checked row (n_J) or column (m_I),
 * own_norm = ||a_i|| (or ||b_j||), other_norm_sum = sum of the other side's
 * norms over the tile. */
double oracle_beta(double u, int64_t kprime, int64_t count, double own_norm, double other_norm_sum)
{
    return 2.0 * u * (double)(kprime + count + 1) * own_norm * other_norm_sum;
}

/* ------------------------------------------------------------------------ */
/* Online ABFT replay.                                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t m, n, k;
    int64_t mc, nc;        /* check tile */
    int64_t ku;            /* k-step of the outer-product update (k_s in Eq. 4) */
    int64_t g;             /* check every g k-steps, and after the last one */
    double alpha, beta;
    double u;              /* unit roundoff of the modelled GPU arithmetic */
    double c;              /* tau = c * beta_bound */
    int32_t ft_level;      /* 0 off, 1 detect only (final check), 2 detect + correct */
    int32_t pad_;
} oracle_cfg_t;

typedef struct {
    int64_t tile_m, tile_n, kstep, row, col;   /* row/col are tile-relative */
    double old_v, new_v;                       /* accumulator value before/after the fault */
    int32_t force;    /* -1: own decision; else bit0 = row flagged, bit1 = col flagged */
    int32_t comp;     /* complex replay: the faulty component, 0 real, 1 imaginary (else 0) */
} oracle_inj_t;

enum {
    ORACLE_EV_CORRECTED = 1,
    ORACLE_EV_CHECKSUM_ROW = 2,   /* one row flagged, no column */
    ORACLE_EV_CHECKSUM_COL = 3,   /* one column flagged, no row */
    ORACLE_EV_UNCORRECTABLE = 4,  /* any other non-empty pattern */
    ORACLE_EV_DETECTED = 5,       /* detect-only level: any non-empty pattern */
    ORACLE_EV_NONFINITE = 6       /* the tile's operands hold Inf or NaN: no decision possible */
};

typedef struct {
    int64_t tile_m, tile_n, kstep, row, col;
    int32_t kind, n_rows, n_cols;
    int32_t comp;     /* complex replay: component the decision is about, 0 real, 1 imaginary (else 0) */
    double value_before, value_after, r_row, r_col, tau_row, tau_col;
} oracle_event_t;

typedef struct {
    int32_t cls;          /* 0 benign, 1 grey, 2 must-detect, -1 not evaluated */
    int32_t pad_;
    int64_t check_step;   /* first check step at or after the injection */
    double delta, tau_row, tau_col, beta_row, beta_col;
} oracle_injclass_t;

typedef struct {
    oracle_event_t* ev;
    int64_t n, cap;
} evbuf_t;

static void ev_push(evbuf_t* b, const oracle_event_t* e)
{
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 8;
        b->ev = (oracle_event_t*)realloc(b->ev, (size_t)b->cap * sizeof(oracle_event_t));
    }
    b->ev[b->n++] = *e;
}

static int is_check_step(const oracle_cfg_t* cfg, int64_t t, int64_t nk)
{
    if (cfg->ft_level == 1) return t == nk - 1;
    return (t % cfg->g) == cfg->g - 1 || t == nk - 1;
}

/* One check tile (I, J) = rows [i0, i0+mI) x cols [j0, j0+nJ). */
static void replay_tile(const oracle_cfg_t* cfg, int64_t tm, int64_t tn,
                        const double* A, int64_t lda, const double* B, int64_t ldb,
                        const double* C0, int64_t ldc0, double* C, int64_t ldc,
                        const oracle_inj_t* inj, const int64_t* inj_idx, int64_t n_inj_tile,
                        oracle_injclass_t* cls, evbuf_t* evs)
{
    const int64_t i0 = tm * cfg->mc, j0 = tn * cfg->nc;
    const int64_t mI = (cfg->m - i0 < cfg->mc) ? cfg->m - i0 : cfg->mc;
    const int64_t nJ = (cfg->n - j0 < cfg->nc) ? cfg->n - j0 : cfg->nc;
    const int64_t K = cfg->k, ku = cfg->ku;
    const int64_t nk = (K + ku - 1) / ku;

    double* P = (double*)calloc((size_t)(mI * nJ), sizeof(double));   /* P[i + j*mI] */
    double* R = (double*)calloc((size_t)mI, sizeof(double));          /* reference row checksums  C e   */
    double* S = (double*)calloc((size_t)nJ, sizeof(double));          /* reference col checksums  e^T C */
    double* na2 = (double*)calloc((size_t)mI, sizeof(double));        /* ||a_i[0:K']||^2 */
    double* nb2 = (double*)calloc((size_t)nJ, sizeof(double));        /* ||b_j[0:K']||^2 */
    double* w = (double*)malloc((size_t)(ku > 0 ? ku : 1) * sizeof(double));
    double* v = (double*)malloc((size_t)(ku > 0 ? ku : 1) * sizeof(double));
    double* rres = (double*)malloc((size_t)mI * sizeof(double));
    double* cres = (double*)malloc((size_t)nJ * sizeof(double));
    double* rtau = (double*)malloc((size_t)mI * sizeof(double));
    double* ctau = (double*)malloc((size_t)nJ * sizeof(double));
    double* rbet = (double*)malloc((size_t)mI * sizeof(double));
    double* cbet = (double*)malloc((size_t)nJ * sizeof(double));
    unsigned char* rflag = (unsigned char*)malloc((size_t)mI);
    unsigned char* cflag = (unsigned char*)malloc((size_t)nJ);

    int64_t next_inj = 0;        /* injections of this tile, sorted by kstep */
    int64_t first_open = 0;      /* first injection not yet evaluated by a check */
    int nonfinite = 0;           /* a non-finite operand has been reported for this tile */

    for (int64_t t = 0; t < nk; ++t) {
        const int64_t k0 = t * ku;
        const int64_t k1 = (k0 + ku < K) ? k0 + ku : K;
        const int64_t kc = k1 - k0;
        const double* Ak = &AT(A, lda, i0, k0);   /* A[I, kt] */
        const double* Bk = &AT(B, ldb, k0, j0);   /* B[kt, J] */

        /* Encode this step's panels (Eq. 1-2). */
        if (cfg->ft_level > 0) {
            oracle_encode_col(mI, kc, Ak, lda, w);
            oracle_encode_row(kc, nJ, Bk, ldb, v);
        }

        /* Rank-kc update of the tile, C_s = A(:, s) B(s, :) (Eq. 4). */
        for (int64_t j = 0; j < nJ; ++j)
            for (int64_t p = 0; p < kc; ++p) {
                const double b = AT(Bk, ldb, p, j);
                for (int64_t i = 0; i < mI; ++i) P[i + j * mI] += AT(Ak, lda, i, p) * b;
            }

        if (cfg->ft_level > 0) {
            /* Reference checksums carried through the update (Eq. 4):
             * C_s e = A(:, s) (B(s, :) e),  e^T C_s = (e^T A(:, s)) B(s, :). */
            for (int64_t i = 0; i < mI; ++i) {
                double s = 0.0, q = 0.0;
                for (int64_t p = 0; p < kc; ++p) {
                    const double a = AT(Ak, lda, i, p);
                    s += a * v[p];
                    q += a * a;
                }
                R[i] += s;
                na2[i] += q;
            }
            for (int64_t j = 0; j < nJ; ++j) {
                double s = 0.0, q = 0.0;
                for (int64_t p = 0; p < kc; ++p) {
                    const double b = AT(Bk, ldb, p, j);
                    s += w[p] * b;
                    q += b * b;
                }
                S[j] += s;
                nb2[j] += q;
            }
        }

        /* Faults logged for this step: applied to the accumulator after the update. */
        while (next_inj < n_inj_tile && inj[inj_idx[next_inj]].kstep == t) {
            const oracle_inj_t* f = &inj[inj_idx[next_inj]];
            double* x = &P[f->row + f->col * mI];
            if (isfinite(f->old_v) && isfinite(f->new_v)) *x += f->new_v - f->old_v;
            else *x = f->new_v;
            ++next_inj;
        }

        if (cfg->ft_level == 0 || !is_check_step(cfg, t, nk)) continue;

        /* ---- check (section 2.2: compare sums with the checksums against a threshold) ---- */
        double sum_na = 0.0, sum_nb = 0.0;
        for (int64_t i = 0; i < mI; ++i) sum_na += sqrt(na2[i]);
        for (int64_t j = 0; j < nJ; ++j) sum_nb += sqrt(nb2[j]);

        /* An Inf or NaN among the operands read so far makes the norms, the
         * reference checksums and the bound non-finite: the check can no longer
         * tell rounding from a fault.  The tile is reported once, at the first
         * check that sees it, with no location, nothing is corrected or
         * re-based, and its part of C is whatever IEEE arithmetic gives.  The
         * faults such a check would have seen are left unclassified. */
        if (!isfinite(sum_na) || !isfinite(sum_nb)) {
            for (int64_t q = first_open; q < next_inj; ++q)
                if (cls) cls[inj_idx[q]].check_step = t;
            first_open = next_inj;
            if (!nonfinite) {
                oracle_event_t e;
                memset(&e, 0, sizeof e);
                e.tile_m = tm; e.tile_n = tn; e.kstep = t; e.row = -1; e.col = -1;
                e.kind = ORACLE_EV_NONFINITE;
                ev_push(evs, &e);
                nonfinite = 1;
            }
            continue;
        }
        int64_t nr = 0, ncf = 0, fr = -1, fc = -1;
        for (int64_t i = 0; i < mI; ++i) {
            double s = 0.0;
            for (int64_t j = 0; j < nJ; ++j) s += P[i + j * mI];
            rres[i] = s - R[i];
            rbet[i] = oracle_beta(cfg->u, k1, nJ, sqrt(na2[i]), sum_nb);
            rtau[i] = cfg->c * rbet[i];
            rflag[i] = !(fabs(rres[i]) <= rtau[i]);
        }
        for (int64_t j = 0; j < nJ; ++j) {
            double s = 0.0;
            for (int64_t i = 0; i < mI; ++i) s += P[i + j * mI];
            cres[j] = s - S[j];
            cbet[j] = oracle_beta(cfg->u, k1, mI, sqrt(nb2[j]), sum_na);
            ctau[j] = cfg->c * cbet[j];
            cflag[j] = !(fabs(cres[j]) <= ctau[j]);
        }

        /* Classify the injections this check is the first to see, and apply the
         * GPU's decision for those the caller forces (grey-zone sites). */
        for (int64_t q = first_open; q < next_inj; ++q) {
            const int64_t id = inj_idx[q];
            const oracle_inj_t* f = &inj[id];
            if (cls) {
                oracle_injclass_t* o = &cls[id];
                const double d = (isfinite(f->old_v) && isfinite(f->new_v)) ? f->new_v - f->old_v : INFINITY;
                o->check_step = t;
                o->delta = d;
                o->tau_row = rtau[f->row]; o->tau_col = ctau[f->col];
                o->beta_row = rbet[f->row]; o->beta_col = cbet[f->col];
                /* relative slack for the GPU's own FP32 evaluation of tau */
                const double sl = 1e-3;
                const double ad = fabs(d);
                const int must = !isfinite(f->new_v) ||
                    (ad > (rtau[f->row] + rbet[f->row]) * (1 + sl) && ad > (ctau[f->col] + cbet[f->col]) * (1 + sl));
                const int benign = isfinite(f->new_v) &&
                    ad < (rtau[f->row] - rbet[f->row]) * (1 - sl) && ad < (ctau[f->col] - cbet[f->col]) * (1 - sl);
                o->cls = must ? 2 : (benign ? 0 : 1);
            }
            if (f->force >= 0) {
                rflag[f->row] = (unsigned char)((f->force & 1) != 0);
                cflag[f->col] = (unsigned char)((f->force & 2) != 0);
            }
        }
        first_open = next_inj;

        for (int64_t i = 0; i < mI; ++i) if (rflag[i]) { if (fr < 0) fr = i; ++nr; }
        for (int64_t j = 0; j < nJ; ++j) if (cflag[j]) { if (fc < 0) fc = j; ++ncf; }
        if (nr == 0 && ncf == 0) continue;

        oracle_event_t e;
        memset(&e, 0, sizeof e);
        e.tile_m = tm; e.tile_n = tn; e.kstep = t; e.row = fr; e.col = fc;
        e.n_rows = (int32_t)nr; e.n_cols = (int32_t)ncf;
        e.r_row = fr >= 0 ? rres[fr] : 0.0; e.tau_row = fr >= 0 ? rtau[fr] : 0.0;
        e.r_col = fc >= 0 ? cres[fc] : 0.0; e.tau_col = fc >= 0 ? ctau[fc] : 0.0;
        if (fr >= 0 && fc >= 0) e.value_before = e.value_after = P[fr + fc * mI];

        if (cfg->ft_level == 1) {
            e.kind = ORACLE_EV_DETECTED;
        } else if (nr == 1 && ncf == 1) {
            /* Locate at the row/column intersection and rebuild the element from
             * the row checksum: P_ij = R_i - sum_{j' != j} P_ij'. */
            double s = 0.0;
            for (int64_t j = 0; j < nJ; ++j) if (j != fc) s += P[fr + j * mI];
            P[fr + fc * mI] = R[fr] - s;
            e.value_after = P[fr + fc * mI];
            e.kind = ORACLE_EV_CORRECTED;
        } else {
            e.kind = (nr == 1 && ncf == 0) ? ORACLE_EV_CHECKSUM_ROW
                   : (nr == 0 && ncf == 1) ? ORACLE_EV_CHECKSUM_COL
                   : ORACLE_EV_UNCORRECTABLE;
            /* Re-base every flagged checksum on the accumulator so later checks
             * only see new faults. */
            for (int64_t i = 0; i < mI; ++i) if (rflag[i]) R[i] += rres[i];
            for (int64_t j = 0; j < nJ; ++j) if (cflag[j]) S[j] += cres[j];
        }
        ev_push(evs, &e);
    }

    for (int64_t j = 0; j < nJ; ++j)
        for (int64_t i = 0; i < mI; ++i) {
            const double c0 = (cfg->beta == 0.0) ? 0.0 : cfg->beta * AT(C0, ldc0, i0 + i, j0 + j);
            AT(C, ldc, i0 + i, j0 + j) = cfg->alpha * P[i + j * mI] + c0;
        }

    free(P); free(R); free(S); free(na2); free(nb2); free(w); free(v);
    free(rres); free(cres); free(rtau); free(ctau); free(rbet); free(cbet);
    free(rflag); free(cflag);
}

static const oracle_inj_t* g_sort_inj;
static int cmp_inj(const void* a, const void* b)
{
    const oracle_inj_t* x = &g_sort_inj[*(const int64_t*)a];
    const oracle_inj_t* y = &g_sort_inj[*(const int64_t*)b];
    if (x->tile_m != y->tile_m) return x->tile_m < y->tile_m ? -1 : 1;
    if (x->tile_n != y->tile_n) return x->tile_n < y->tile_n ? -1 : 1;
    if (x->kstep != y->kstep) return x->kstep < y->kstep ? -1 : 1;
    const int64_t ia = *(const int64_t*)a, ib = *(const int64_t*)b;
    return ia < ib ? -1 : (ia > ib);
}

/*
 * Replay of the online FT-GEMM over the tile decomposition (cfg->mc, cfg->nc)
 * and k-steps of cfg->ku, with the logged faults applied where the GPU applied
 * them.  With tiles_sel == NULL every tile is replayed; otherwise only the
 * n_sel tiles listed as (tile_m, tile_n) pairs, and only their part of C is
 * written.  Events are returned in (tile_m, tile_n, kstep) order.
 * Returns the number of events (which may exceed ev_cap; only ev_cap are
 * stored), or a negative value on invalid arguments.
 */
int64_t oracle_ftgemm_replay(const oracle_cfg_t* cfg,
                             const double* A, int64_t lda, const double* B, int64_t ldb,
                             const double* C0, int64_t ldc0, double* C, int64_t ldc,
                             const oracle_inj_t* inj, int64_t n_inj,
                             const int64_t* tiles_sel, int64_t n_sel,
                             oracle_injclass_t* cls,
                             oracle_event_t* ev, int64_t ev_cap)
{
    if (!cfg || cfg->m < 0 || cfg->n < 0 || cfg->k < 0) return -1;
    if (cfg->mc <= 0 || cfg->nc <= 0 || cfg->ku <= 0 || cfg->g <= 0) return -2;
    if (cfg->m == 0 || cfg->n == 0) return 0;
    const int64_t ntm = (cfg->m + cfg->mc - 1) / cfg->mc;
    const int64_t ntn = (cfg->n + cfg->nc - 1) / cfg->nc;
    const int64_t ntiles = tiles_sel ? n_sel : ntm * ntn;

    /* bucket the injections by tile, sorted by kstep */
    int64_t* order = (int64_t*)malloc((size_t)(n_inj > 0 ? n_inj : 1) * sizeof(int64_t));
    for (int64_t q = 0; q < n_inj; ++q) {
        order[q] = q;
        if (inj[q].tile_m < 0 || inj[q].tile_m >= ntm || inj[q].tile_n < 0 || inj[q].tile_n >= ntn) { free(order); return -3; }
        if (cls) { cls[q].cls = -1; cls[q].check_step = -1; }
    }
    g_sort_inj = inj;
    qsort(order, (size_t)n_inj, sizeof(int64_t), cmp_inj);

    evbuf_t* bufs = (evbuf_t*)calloc((size_t)(ntiles > 0 ? ntiles : 1), sizeof(evbuf_t));

    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < ntiles; ++s) {
        const int64_t tm = tiles_sel ? tiles_sel[2 * s] : s / ntn;
        const int64_t tn = tiles_sel ? tiles_sel[2 * s + 1] : s % ntn;
        if (tm < 0 || tm >= ntm || tn < 0 || tn >= ntn) continue;
        int64_t lo = 0, hi = n_inj;   /* range of injections of tile (tm, tn) */
        while (lo < n_inj && (inj[order[lo]].tile_m < tm || (inj[order[lo]].tile_m == tm && inj[order[lo]].tile_n < tn))) ++lo;
        hi = lo;
        while (hi < n_inj && inj[order[hi]].tile_m == tm && inj[order[hi]].tile_n == tn) ++hi;
        replay_tile(cfg, tm, tn, A, lda, B, ldb, C0, ldc0, C, ldc, inj, order + lo, hi - lo, cls, &bufs[s]);
    }

    int64_t total = 0;
    for (int64_t s = 0; s < ntiles; ++s) {
        for (int64_t e = 0; e < bufs[s].n; ++e) {
            if (total < ev_cap && ev) ev[total] = bufs[s].ev[e];
            ++total;
        }
        free(bufs[s].ev);
    }
    free(bufs);
    free(order);
    return total;
}

/* ======================================================================== */
/* Complex binary64: the double-complex GEMM that the conclusion (section 6)  */
/* names as future work, with the same online ABFT.                           */
/*                                                                            */
/* Matrices are column-major arrays of (re, im) double pairs; leading         */
/* dimensions count complex elements.  The encodings e^T A and B e, the       */
/* reference checksums and the accumulator are complex, and every product is  */
/* a complex multiply.  The checksum relation (Eq. 3, Eq. 4) is linear, so it */
/* holds for the real and the imaginary part separately; a complex            */
/* accumulator element is two real values, and the single-event-upset model   */
/* of section 4.1 is read per real value: each component is checked, located  */
/* and corrected on its own, with events labelled by component.  The bound of */
/* a component: each component of a complex sum of K' products is a real sum  */
/* of 2K' products (re = ar br - ai bi, im = ar bi + ai br), and              */
/* |ar br| + |ai bi| <= |a| |b|, so the real bound holds with K' -> 2K' and   */
/* complex 2-norms:                                                           */
/*   beta_row_i = 2u (2K' + n_J + 1) ||a_i[0:K']|| sum_{j in J} ||b_j[0:K']|| */
/* (and the column bound likewise), for |Re r_i| and |Im r_i| alike.          */
/* ======================================================================== */
typedef double _Complex zdouble;

static inline zdouble zget(const double* M, int64_t ld, int64_t r, int64_t c)
{
    const size_t x = 2 * ((size_t)r + (size_t)c * (size_t)ld);
    return CMPLX(M[x], M[x + 1]);
}

static inline void zput(double* M, int64_t ld, int64_t r, int64_t c, zdouble v)
{
    const size_t x = 2 * ((size_t)r + (size_t)c * (size_t)ld);
    M[x] = creal(v);
    M[x + 1] = cimag(v);
}

static inline double zcomp(zdouble v, int c) { return c ? cimag(v) : creal(v); }
static inline zdouble zwith(zdouble v, int c, double x) { return c ? CMPLX(creal(v), x) : CMPLX(x, cimag(v)); }

/* Plain complex GEMM: C = alpha * A * B + beta * C0 (beta == 0: C0 not read). */
int oracle_zgemm(int64_t m, int64_t n, int64_t k, double alpha_re, double alpha_im,
                 const double* A, int64_t lda, const double* B, int64_t ldb,
                 double beta_re, double beta_im, double* C, int64_t ldc)
{
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (k < 0) return -3;
    if (lda < (m > 1 ? m : 1)) return -6;
    if (ldb < (k > 1 ? k : 1)) return -8;
    if (ldc < (m > 1 ? m : 1)) return -11;
    if (m == 0 || n == 0) return 0;
    const zdouble alpha = CMPLX(alpha_re, alpha_im), beta = CMPLX(beta_re, beta_im);

    #pragma omp parallel
    {
        zdouble* col = (zdouble*)malloc((size_t)m * sizeof(zdouble));
        #pragma omp for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            for (int64_t i = 0; i < m; ++i) col[i] = 0.0;
            if (alpha != 0.0) {
                for (int64_t p = 0; p < k; ++p) {
                    const zdouble b = zget(B, ldb, p, j);
                    for (int64_t i = 0; i < m; ++i) col[i] += zget(A, lda, i, p) * b;
                }
            }
            for (int64_t i = 0; i < m; ++i) {
                const zdouble c0 = (beta == 0.0) ? 0.0 : beta * zget(C, ldc, i, j);
                zput(C, ldc, i, j, alpha * col[i] + c0);
            }
        }
        free(col);
    }
    return 0;
}

/* Complex encodings (Eq. 1-2): w = e^T A over `rows` rows, v = B e over `cols`
 * columns, kcount complex values each (2 kcount doubles). */
void oracle_zencode_col(int64_t rows, int64_t kcount, const double* A, int64_t lda, double* w)
{
    for (int64_t p = 0; p < kcount; ++p) {
        zdouble s = 0.0;
        for (int64_t i = 0; i < rows; ++i) s += zget(A, lda, i, p);
        w[2 * p] = creal(s);
        w[2 * p + 1] = cimag(s);
    }
}

void oracle_zencode_row(int64_t kcount, int64_t cols, const double* B, int64_t ldb, double* v)
{
    for (int64_t p = 0; p < kcount; ++p) {
        zdouble s = 0.0;
        for (int64_t j = 0; j < cols; ++j) s += zget(B, ldb, p, j);
        v[2 * p] = creal(s);
        v[2 * p + 1] = cimag(s);
    }
}

static void zreplay_tile(const oracle_cfg_t* cfg, zdouble alpha, zdouble beta, int64_t tm, int64_t tn,
                         const double* A, int64_t lda, const double* B, int64_t ldb,
                         const double* C0, int64_t ldc0, double* C, int64_t ldc,
                         const oracle_inj_t* inj, const int64_t* inj_idx, int64_t n_inj_tile,
                         oracle_injclass_t* cls, evbuf_t* evs)
{
    const int64_t i0 = cfg->mc * tm, j0 = cfg->nc * tn;
    const int64_t mI = (cfg->m - i0 < cfg->mc) ? cfg->m - i0 : cfg->mc;
    const int64_t nJ = (cfg->n - j0 < cfg->nc) ? cfg->n - j0 : cfg->nc;
    const int64_t K = cfg->k, ku = cfg->ku;
    const int64_t nk = (K + ku - 1) / ku;

    zdouble* P = (zdouble*)calloc((size_t)(mI * nJ), sizeof(zdouble));
    zdouble* R = (zdouble*)calloc((size_t)mI, sizeof(zdouble));
    zdouble* S = (zdouble*)calloc((size_t)nJ, sizeof(zdouble));
    double* na2 = (double*)calloc((size_t)mI, sizeof(double));
    double* nb2 = (double*)calloc((size_t)nJ, sizeof(double));
    double* w = (double*)malloc((size_t)(2 * (ku > 0 ? ku : 1)) * sizeof(double));
    double* v = (double*)malloc((size_t)(2 * (ku > 0 ? ku : 1)) * sizeof(double));
    double* rres = (double*)malloc((size_t)mI * sizeof(double));
    double* cres = (double*)malloc((size_t)nJ * sizeof(double));
    double* rtau = (double*)malloc((size_t)mI * sizeof(double));
    double* ctau = (double*)malloc((size_t)nJ * sizeof(double));
    double* rbet = (double*)malloc((size_t)mI * sizeof(double));
    double* cbet = (double*)malloc((size_t)nJ * sizeof(double));
    unsigned char* rflag = (unsigned char*)malloc((size_t)mI);
    unsigned char* cflag = (unsigned char*)malloc((size_t)nJ);

    int64_t next_inj = 0, first_open = 0;
    int nonfinite = 0;

    for (int64_t t = 0; t < nk; ++t) {
        const int64_t k0 = t * ku;
        const int64_t k1 = (k0 + ku < K) ? k0 + ku : K;
        const int64_t kc = k1 - k0;

        if (cfg->ft_level > 0) {
            oracle_zencode_col(mI, kc, A + 2 * ((size_t)i0 + (size_t)k0 * (size_t)lda), lda, w);
            oracle_zencode_row(kc, nJ, B + 2 * ((size_t)k0 + (size_t)j0 * (size_t)ldb), ldb, v);
        }
        /* rank-kc update of the tile with complex products (Eq. 4) */
        for (int64_t j = 0; j < nJ; ++j)
            for (int64_t p = 0; p < kc; ++p) {
                const zdouble b = zget(B, ldb, k0 + p, j0 + j);
                for (int64_t i = 0; i < mI; ++i) P[i + j * mI] += zget(A, lda, i0 + i, k0 + p) * b;
            }
        if (cfg->ft_level > 0) {
            for (int64_t i = 0; i < mI; ++i) {
                zdouble s = 0.0;
                double q = 0.0;
                for (int64_t p = 0; p < kc; ++p) {
                    const zdouble a = zget(A, lda, i0 + i, k0 + p);
                    s += a * CMPLX(v[2 * p], v[2 * p + 1]);
                    q += creal(a) * creal(a) + cimag(a) * cimag(a);
                }
                R[i] += s;
                na2[i] += q;
            }
            for (int64_t j = 0; j < nJ; ++j) {
                zdouble s = 0.0;
                double q = 0.0;
                for (int64_t p = 0; p < kc; ++p) {
                    const zdouble b = zget(B, ldb, k0 + p, j0 + j);
                    s += CMPLX(w[2 * p], w[2 * p + 1]) * b;
                    q += creal(b) * creal(b) + cimag(b) * cimag(b);
                }
                S[j] += s;
                nb2[j] += q;
            }
        }
        /* faults of this step hit one component of the accumulator */
        while (next_inj < n_inj_tile && inj[inj_idx[next_inj]].kstep == t) {
            const oracle_inj_t* f = &inj[inj_idx[next_inj]];
            zdouble* x = &P[f->row + f->col * mI];
            const double cur = zcomp(*x, f->comp);
            const double nv = (isfinite(f->old_v) && isfinite(f->new_v)) ? cur + (f->new_v - f->old_v) : f->new_v;
            *x = zwith(*x, f->comp, nv);
            ++next_inj;
        }
        if (cfg->ft_level == 0 || !is_check_step(cfg, t, nk)) continue;

        double sum_na = 0.0, sum_nb = 0.0;
        for (int64_t i = 0; i < mI; ++i) sum_na += sqrt(na2[i]);
        for (int64_t j = 0; j < nJ; ++j) sum_nb += sqrt(nb2[j]);
        if (!(isfinite(sum_na) && isfinite(sum_nb))) {   /* non-finite operands: as in the real replay */
            for (int64_t q = first_open; q < next_inj; ++q)
                if (cls) cls[inj_idx[q]].check_step = t;
            first_open = next_inj;
            if (nonfinite == 0) {
                oracle_event_t e;
                memset(&e, 0, sizeof e);
                e.tile_m = tm; e.tile_n = tn; e.kstep = t; e.row = -1; e.col = -1;
                e.kind = ORACLE_EV_NONFINITE;
                ev_push(evs, &e);
                nonfinite = 1;
            }
            continue;
        }
        for (int c = 0; c < 2; ++c) {
            int64_t nrc = 0, ncc = 0, fr = -1, fc = -1;
            for (int64_t i = 0; i < mI; ++i) {
                zdouble s = 0.0;
                for (int64_t j = 0; j < nJ; ++j) s += P[i + j * mI];
                rres[i] = zcomp(s, c) - zcomp(R[i], c);
                rbet[i] = oracle_beta(cfg->u, 2 * k1, nJ, sqrt(na2[i]), sum_nb);
                rtau[i] = cfg->c * rbet[i];
                rflag[i] = (unsigned char)!(fabs(rres[i]) <= rtau[i]);
            }
            for (int64_t j = 0; j < nJ; ++j) {
                zdouble s = 0.0;
                for (int64_t i = 0; i < mI; ++i) s += P[i + j * mI];
                cres[j] = zcomp(s, c) - zcomp(S[j], c);
                cbet[j] = oracle_beta(cfg->u, 2 * k1, mI, sqrt(nb2[j]), sum_na);
                ctau[j] = cfg->c * cbet[j];
                cflag[j] = (unsigned char)!(fabs(cres[j]) <= ctau[j]);
            }
            for (int64_t q = first_open; q < next_inj; ++q) {
                const int64_t id = inj_idx[q];
                const oracle_inj_t* f = &inj[id];
                if (f->comp != c) continue;
                if (cls) {
                    oracle_injclass_t* o = &cls[id];
                    const double d = (isfinite(f->old_v) && isfinite(f->new_v)) ? f->new_v - f->old_v : INFINITY;
                    o->check_step = t;
                    o->delta = d;
                    o->tau_row = rtau[f->row]; o->tau_col = ctau[f->col];
                    o->beta_row = rbet[f->row]; o->beta_col = cbet[f->col];
                    const double sl = 1e-3, ad = fabs(d);
                    const int must = !isfinite(f->new_v) ||
                        (ad > (rtau[f->row] + rbet[f->row]) * (1 + sl) && ad > (ctau[f->col] + cbet[f->col]) * (1 + sl));
                    const int benign = isfinite(f->new_v) &&
                        ad < (rtau[f->row] - rbet[f->row]) * (1 - sl) && ad < (ctau[f->col] - cbet[f->col]) * (1 - sl);
                    o->cls = must ? 2 : (benign ? 0 : 1);
                }
                if (f->force >= 0) {
                    rflag[f->row] = (unsigned char)((f->force & 1) != 0);
                    cflag[f->col] = (unsigned char)((f->force & 2) != 0);
                }
            }
            for (int64_t i = 0; i < mI; ++i) if (rflag[i]) { if (fr < 0) fr = i; ++nrc; }
            for (int64_t j = 0; j < nJ; ++j) if (cflag[j]) { if (fc < 0) fc = j; ++ncc; }
            if (nrc == 0 && ncc == 0) continue;

            oracle_event_t e;
            memset(&e, 0, sizeof e);
            e.tile_m = tm; e.tile_n = tn; e.kstep = t; e.row = fr; e.col = fc; e.comp = c;
            e.n_rows = (int32_t)nrc; e.n_cols = (int32_t)ncc;
            e.r_row = fr >= 0 ? rres[fr] : 0.0; e.tau_row = fr >= 0 ? rtau[fr] : 0.0;
            e.r_col = fc >= 0 ? cres[fc] : 0.0; e.tau_col = fc >= 0 ? ctau[fc] : 0.0;
            if (fr >= 0 && fc >= 0) e.value_before = e.value_after = zcomp(P[fr + fc * mI], c);
            if (cfg->ft_level == 1) {
                e.kind = ORACLE_EV_DETECTED;
            } else if (nrc == 1 && ncc == 1) {
                /* component c of the element rebuilt from the row checksum */
                double s = 0.0;
                for (int64_t j = 0; j < nJ; ++j) if (j != fc) s += zcomp(P[fr + j * mI], c);
                P[fr + fc * mI] = zwith(P[fr + fc * mI], c, zcomp(R[fr], c) - s);
                e.value_after = zcomp(P[fr + fc * mI], c);
                e.kind = ORACLE_EV_CORRECTED;
            } else {
                e.kind = (nrc == 1 && ncc == 0) ? ORACLE_EV_CHECKSUM_ROW
                       : (nrc == 0 && ncc == 1) ? ORACLE_EV_CHECKSUM_COL
                       : ORACLE_EV_UNCORRECTABLE;
                for (int64_t i = 0; i < mI; ++i) if (rflag[i]) R[i] = zwith(R[i], c, zcomp(R[i], c) + rres[i]);
                for (int64_t j = 0; j < nJ; ++j) if (cflag[j]) S[j] = zwith(S[j], c, zcomp(S[j], c) + cres[j]);
            }
            ev_push(evs, &e);
        }
        first_open = next_inj;
    }

    for (int64_t j = 0; j < nJ; ++j)
        for (int64_t i = 0; i < mI; ++i) {
            const zdouble c0 = (beta == 0.0) ? 0.0 : beta * zget(C0, ldc0, i0 + i, j0 + j);
            zput(C, ldc, i0 + i, j0 + j, alpha * P[i + j * mI] + c0);
        }

    free(P); free(R); free(S); free(na2); free(nb2); free(w); free(v);
    free(rres); free(cres); free(rtau); free(ctau); free(rbet); free(cbet);
    free(rflag); free(cflag);
}

/*
 * Replay of the online complex FT-GEMM, as oracle_ftgemm_replay (cfg->alpha
 * and cfg->beta are the real parts of alpha and beta, alpha_im and beta_im the
 * imaginary parts).  Injections name the faulty component (comp), and events
 * the component they decide on.
 */
int64_t oracle_zftgemm_replay(const oracle_cfg_t* cfg, double alpha_im, double beta_im,
                              const double* A, int64_t lda, const double* B, int64_t ldb,
                              const double* C0, int64_t ldc0, double* C, int64_t ldc,
                              const oracle_inj_t* inj, int64_t n_inj,
                              const int64_t* tiles_sel, int64_t n_sel,
                              oracle_injclass_t* cls,
                              oracle_event_t* ev, int64_t ev_cap)
{
    if (!cfg || cfg->m < 0 || cfg->n < 0 || cfg->k < 0) return -1;
    if (cfg->mc <= 0 || cfg->nc <= 0 || cfg->ku <= 0 || cfg->g <= 0) return -2;
    if (cfg->m == 0 || cfg->n == 0) return 0;
    const int64_t ntm = (cfg->m + cfg->mc - 1) / cfg->mc;
    const int64_t ntn = (cfg->n + cfg->nc - 1) / cfg->nc;
    const int64_t ntiles = tiles_sel ? n_sel : ntm * ntn;
    const zdouble alpha = CMPLX(cfg->alpha, alpha_im), beta = CMPLX(cfg->beta, beta_im);

    int64_t* order = (int64_t*)malloc((size_t)(n_inj > 0 ? n_inj : 1) * sizeof(int64_t));
    for (int64_t q = 0; q < n_inj; ++q) {
        order[q] = q;
        if (inj[q].tile_m < 0 || inj[q].tile_m >= ntm || inj[q].tile_n < 0 || inj[q].tile_n >= ntn ||
            inj[q].comp < 0 || inj[q].comp > 1) { free(order); return -3; }
        if (cls) { cls[q].cls = -1; cls[q].check_step = -1; }
    }
    g_sort_inj = inj;
    qsort(order, (size_t)n_inj, sizeof(int64_t), cmp_inj);

    evbuf_t* bufs = (evbuf_t*)calloc((size_t)(ntiles > 0 ? ntiles : 1), sizeof(evbuf_t));

    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < ntiles; ++s) {
        const int64_t tm = tiles_sel ? tiles_sel[2 * s] : s / ntn;
        const int64_t tn = tiles_sel ? tiles_sel[2 * s + 1] : s % ntn;
        if (tm < 0 || tm >= ntm || tn < 0 || tn >= ntn) continue;
        int64_t lo = 0, hi;
        while (lo < n_inj && (inj[order[lo]].tile_m < tm || (inj[order[lo]].tile_m == tm && inj[order[lo]].tile_n < tn))) ++lo;
        hi = lo;
        while (hi < n_inj && inj[order[hi]].tile_m == tm && inj[order[hi]].tile_n == tn) ++hi;
        zreplay_tile(cfg, alpha, beta, tm, tn, A, lda, B, ldb, C0, ldc0, C, ldc, inj, order + lo, hi - lo, cls,
                     &bufs[s]);
    }

    int64_t total = 0;
    for (int64_t s = 0; s < ntiles; ++s) {
        for (int64_t e = 0; e < bufs[s].n; ++e) {
            if (total < ev_cap && ev) ev[total] = bufs[s].ev[e];
            ++total;
        }
        free(bufs[s].ev);
    }
    free(bufs);
    free(order);
    return total;
}

/* Number of OpenMP threads the oracle runs with (for reporting). */
int oracle_threads(void) { return omp_get_max_threads(); }

/* Threads for later calls (the benchmark times one thread and all of them). */
void oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }

/* ABI self-description used by the Python loader to check struct layouts. */
int64_t oracle_sizeof(int which)
{
    switch (which) {
        case 0: return (int64_t)sizeof(oracle_cfg_t);
        case 1: return (int64_t)sizeof(oracle_inj_t);
        case 2: return (int64_t)sizeof(oracle_event_t);
        case 3: return (int64_t)sizeof(oracle_injclass_t);
        default: return -1;
    }
}
