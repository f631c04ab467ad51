"""The pins must catch plausible mistakes: each case builds a copy of oracle.c with one planted
error (on the CPU, in a temporary directory) and runs the pin checks against it; at least one
check has to fail.  The shipped oracle is never modified."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import synth

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "oracle.c")

MUTATIONS = {
    # eq. diagScal2 taken literally: scale by 1/psi instead of psi^-1/2
    "scale_1_over_psi": ("g[m - 1] = dinv[m - 1];", "g[m - 1] = dinv[m - 1] * dinv[m - 1];"),
    # gradient from row i only (drops the sum over the pattern)
    "grad_row_i_only": ("for (int32_t t = 0; t < m; ++t) {\n            int32_t r = P[t];",
                        "for (int32_t t = m - 1; t < m; ++t) {\n            int32_t r = P[t];"),
    # tie rule resolved towards the largest column
    "tie_largest": ("(best < 0 || j < w->elig[best])", "(best < 0 || j > w->elig[best])"),
    # exit test with the inequality reversed
    "exit_reversed": ("if (psi <= eps * psi0) {", "if (psi >= eps * psi0) {"),
    # back substitution sign
    "solve_sign": ("g[t] = -(acc * dinv[t]);", "g[t] = (acc * dinv[t]);"),
    # pivot reciprocal taken from the wrong column
    "pivot_index": ("L[r * m + c] = acc * dinv[c];", "L[r * m + c] = acc * dinv[r];"),
    # new positions inserted after i instead of before it
    "append_after_i": ("P[m - 1] = S[q];\n            P[m] = i;", "P[m] = S[q];"),
    # Cholesky update sign
    "chol_sign": ("acc = acc - L[r * m + t] * L[c * m + t];", "acc = acc + L[r * m + t] * L[c * m + t];"),
    # gather with a transposed / wrong index
    "gather_index": ("csr_entry(rp, ci, av, P[p], P[q])", "csr_entry(rp, ci, av, P[q], P[q])"),
    # candidates allowed beyond the diagonal (upper part)
    "upper_candidates": ("if (j >= i) continue;", "if (j == i) continue;"),
    # smallest instead of largest gradient
    "select_smallest": ("if (fabs(w->v[j]) >= band && (best < 0", "if (fabs(w->v[j]) <= band && (best < 0"),
    # PCG beta inverted
    "pcg_beta": ("double beta = rho1 / rho;", "double beta = rho / rho1;"),
    # PCG residual update sign
    "pcg_residual": ("r[i] = r[i] - alpha * q[i];", "r[i] = r[i] + alpha * q[i];"),
    # application: forgets the transpose (applies G twice)
    "apply_no_transpose": ("oracle_spmv_t(n, grp, gci, gv, t, z);", "oracle_spmv(n, grp, gci, gv, t, z);"),
}


def _pins_pass() -> bool:
    """A compact subset of the pins (closed forms, LAPACK, SciPy, invariants)."""
    import math

    import scipy.sparse.linalg as spla

    try:
        # 3x3 closed form (k_max = 2 reaches column 0 through row 1)
        A3 = synth.CSR.from_dense(np.array([[4.0, 1, 0], [1, 4, 1], [0, 1, 4]]))
        G = oracle.setup(A3, 2, 1, 0.0).to_scipy().toarray()
        if not np.allclose(G, np.linalg.inv(np.linalg.cholesky(A3.to_scipy().toarray())), rtol=1e-13, atol=1e-15):
            return False
        # full pattern = chol^-1 on dense SPD
        a = synth.random_spd_dense(7, 3)
        G = oracle.setup(synth.CSR.from_dense(a), 6, 1, 0.0).to_scipy().toarray()
        if not np.allclose(G, np.linalg.inv(np.linalg.cholesky(a)), rtol=1e-10, atol=1e-12):
            return False
        # 7-point: tie rule, exact counts, unit diagonal of G A G^T
        A = synth.lap7(6)
        G1 = oracle.setup(A, 1, 1, 0.0)
        i = 3 + 6 * 3 + 36 * 3
        if list(G1.col[G1.row_ptr[i]:G1.row_ptr[i + 1]]) != [i - 36, i]:
            return False
        c = math.sqrt(35.0 / 6.0)
        if abs(G1.val[G1.row_ptr[i + 1] - 1] - 1 / c) > 1e-14:
            return False
        P = synth.poisson7(10)
        G = oracle.setup(P.A, 5, 1, 1e-2)
        if not np.array_equal(G.rows.m, np.minimum(6, np.arange(P.n) + 1)):
            return False
        Gs = G.to_scipy()
        if not np.allclose((Gs @ P.A.to_scipy() @ Gs.T).diagonal(), 1.0, rtol=1e-12):
            return False
        if np.any(G.col > np.repeat(np.arange(P.n), np.diff(G.row_ptr))):
            return False
        Ge = oracle.setup(A, 4, 1, 0.98)
        if not np.all(Ge.rows.m[Ge.rows.steps > 0] == 2):
            return False
        # application against SciPy, PCG against a direct solve
        r = synth.uniform(1, 5, P.n)
        if not np.allclose(oracle.apply(G, r), Gs.T @ (Gs @ r), rtol=1e-12, atol=1e-14):
            return False
        res = oracle.pcg(P.A, G, P.b, 1e-8, maxit=500)
        xs = spla.spsolve(P.A.to_scipy().tocsc(), P.b)
        if res.status != oracle.OK or np.linalg.norm(res.x - xs) > 1e-6 * np.linalg.norm(xs):
            return False
        return True
    except oracle.OracleError:
        return False


def test_unmodified_oracle_passes_the_subset():
    assert _pins_pass()


def _run_child(so_path: str) -> int:
    """Runs the pin subset against a variant library in a child process (a planted mistake
    may also crash the variant, which then counts as caught)."""
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r); sys.path.insert(0, %r); import oracle; "
            "import test_oracle_mutations as t; oracle._lib = oracle.load_variant(%r); "
            "sys.exit(0 if t._pins_pass() else 1)") % (root, os.path.join(root, "tests"), so_path)
    env = dict(os.environ, OMP_NUM_THREADS="2")
    return subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, timeout=300).returncode


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name):
    with tempfile.TemporaryDirectory() as tmp:
        src = open(SRC).read()
        old, new = MUTATIONS[name]
        assert src.count(old) == 1, name
        path_c = os.path.join(tmp, f"{name}.c")
        path_so = os.path.join(tmp, f"lib{name}.so")
        open(path_c, "w").write(src.replace(old, new))
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o",
                        path_so, path_c, "-lm"], check=True)
        rc = _run_child(path_so)
        assert rc != 0, f"planted mistake {name!r} was not caught"
