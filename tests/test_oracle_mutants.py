"""Planted mistakes in the oracle must be caught by its pins.

Each mutant is a one-line textual edit of oracle/ftgemm_oracle.c (a dropped
term, a wrong sign, a transposed index, a weakened bound, ...).  The edited
source is built into a temporary library and the pin suite is run against it
in a subprocess; the suite must fail.  All mutants keep every memory access
in bounds.  CPU only.
"""
import os
import subprocess
import sys

import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "gemm drops the last k term": (
        "for (int64_t p = 0; p < k; ++p) {\n                    const double b = AT(B, ldb, p, j);",
        "for (int64_t p = 0; p < k - 1; ++p) {\n                    const double b = AT(B, ldb, p, j);"),
    "encode_col transposed operand": (
        "for (int64_t i = 0; i < rows; ++i) s += AT(A, lda, i, p);",
        "for (int64_t i = 0; i < rows; ++i) s += AT(A, lda, p < rows ? p : 0, i < kcount ? i : 0);"),
    "row residual sign": ("rres[i] = s - R[i];", "rres[i] = s + R[i];"),
    "correction sign": ("P[fr + fc * mI] = R[fr] - s;", "P[fr + fc * mI] = R[fr] + s;"),
    "threshold 100x too small": ("return 2.0 * u *", "return 0.02 * u *"),
    "column checksum uses B e": ("s += w[p] * b;", "s += v[p] * b;"),
    "tile row offset uses nc": ("const int64_t i0 = tm * cfg->mc, j0 = tn * cfg->nc;",
                                "const int64_t i0 = tm * cfg->nc, j0 = tn * cfg->nc;"),
    "check step off by one": ("return (t % cfg->g) == cfg->g - 1 || t == nk - 1;",
                              "return (t % cfg->g) == 0 || t == nk - 1;"),
    "NaN-unsafe flag": ("rflag[i] = !(fabs(rres[i]) <= rtau[i]);", "rflag[i] = fabs(rres[i]) > rtau[i];"),
    "row/col event labels swapped": ("e.kind = (nr == 1 && ncf == 0) ? ORACLE_EV_CHECKSUM_ROW",
                                     "e.kind = (nr == 1 && ncf == 0) ? ORACLE_EV_CHECKSUM_COL"),
    "beta epilogue sign": ("AT(C, ldc, i0 + i, j0 + j) = cfg->alpha * P[i + j * mI] + c0;",
                           "AT(C, ldc, i0 + i, j0 + j) = cfg->alpha * P[i + j * mI] - c0;"),
    "row-norm accumulates |a| not a^2": ("q += a * a;", "q += fabs(a);"),
    "row threshold ignores u (binary32 roundoff fixed)": (
        "rbet[i] = oracle_beta(cfg->u, k1, nJ, sqrt(na2[i]), sum_nb);",
        "rbet[i] = oracle_beta(5.9604644775390625e-08, k1, nJ, sqrt(na2[i]), sum_nb);"),
    "non-finite operands go through the decision table": (
        "if (!isfinite(sum_na) || !isfinite(sum_nb)) {", "if (0) {"),
    "non-finite tile reported at every check": ("            if (!nonfinite) {\n", "            if (1) {\n"),
    # complex binary64 replay
    "complex product conjugates B": ("P[i + j * mI] += zget(A, lda, i0 + i, k0 + p) * b;",
                                     "P[i + j * mI] += zget(A, lda, i0 + i, k0 + p) * conj(b);"),
    "complex row reference uses conj(B e)": ("s += a * CMPLX(v[2 * p], v[2 * p + 1]);",
                                             "s += a * CMPLX(v[2 * p], -v[2 * p + 1]);"),
    "complex bound counts K' products per component, not 2K'": (
        "rbet[i] = oracle_beta(cfg->u, 2 * k1, nJ, sqrt(na2[i]), sum_nb);",
        "rbet[i] = oracle_beta(cfg->u, k1, nJ, sqrt(na2[i]), sum_nb);"),
    "complex norm drops the imaginary part": ("q += creal(a) * creal(a) + cimag(a) * cimag(a);",
                                              "q += creal(a) * creal(a);"),
    "complex correction from the other component's checksum": ("zcomp(R[fr], c) - s", "zcomp(R[fr], 1 - c) - s"),
    "complex event labelled with the wrong component": ("e.comp = c;", "e.comp = 0;"),
    "complex fault applied to the real part": ("*x = zwith(*x, f->comp, nv);", "*x = zwith(*x, 0, nv);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(O.SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found once: {name}"
    msrc = tmp_path / "ftgemm_oracle.c"
    msrc.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    str(msrc), "-o", str(lib), "-lm"], check=True)
    env = dict(os.environ, FTGEMM_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_complex.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant '{name}' survived the pins:\n{r.stdout[-2000:]}"
