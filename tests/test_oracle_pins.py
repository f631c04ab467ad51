"""Pins of the FP64 oracle against facts the mathematics of Sec. 2 fixes independently of
the oracle's own code: closed forms, LAPACK/SciPy routines, invariants and brute force.

Each test names the plausible mistake it is there to catch.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import oracle
import synth


def dense(A):
    return A.to_scipy().toarray()


def _elast_small():
    return synth.elast27(5, 1.0, 7)


def _aniso_small():
    return synth.lap7(7, 6, 5, (1.0, 1.0, 300.0))


# --------------------------------------------------------------------------------------
# P9: hand-checkable 3x3 case (closed forms derived from eqs. DensSys / diagScal / grapsi)
# --------------------------------------------------------------------------------------
def test_tridiag3_closed_form():
    """A = tridiag(1,4,1).  k_max=1: rows 1 and 2 take their single lower neighbour and
    g = (-1/(2 sqrt15), 2/sqrt15).  k_max=2: the gradient of row 2 through row 1 reaches
    column 0 (v_0 = a_01 g_1 = -1/(2 sqrt15)) and G becomes chol(A)^-1 exactly.
    Catches: a gradient that only scans row i, a wrong scaling, a wrong back substitution."""
    A = synth.CSR.from_dense(np.array([[4.0, 1, 0], [1, 4, 1], [0, 1, 4]]))
    r15 = math.sqrt(15.0)
    G1 = oracle.setup(A, 1, 1, 0.0).to_scipy().toarray()
    expect1 = np.array([[0.5, 0, 0], [-1 / (2 * r15), 2 / r15, 0], [0, -1 / (2 * r15), 2 / r15]])
    np.testing.assert_allclose(G1, expect1, rtol=1e-15, atol=1e-16)
    G2 = oracle.setup(A, 2, 1, 0.0)
    # row 2 of chol(A)^-1 in closed form: L = chol(A) has L22 = sqrt(4 - 1/(15/4)) = sqrt(56/15)
    l22 = math.sqrt(56.0 / 15.0)
    # solve L^T x = e_3 by hand: x2 = 1/L22, x1 = -(L21 x2)/L11, x0 = -(L10 x1)/L00
    L00, L10, L11, L21 = 2.0, 0.5, r15 / 2, 1.0 / (r15 / 2)
    x2 = 1 / l22
    x1 = -(L21 * x2) / L11
    x0 = -(L10 * x1) / L00
    row2 = np.array([x0, x1, x2])
    np.testing.assert_allclose(G2.to_scipy().toarray()[2], row2, rtol=1e-14)
    np.testing.assert_allclose(row2, [0.0345033, -0.1380131, 0.5175492], atol=5e-8)
    assert list(G2.rows.m) == [1, 2, 3]


def test_tridiag3_golden_file():
    """Values stored in tests/golden/tridiag3.txt (hand-derived; see the file header)."""
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "tridiag3.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    A = synth.CSR.from_dense(np.array([[4.0, 1, 0], [1, 4, 1], [0, 1, 4]]))
    for kmax, i, j, val in ((int(r[0]), int(r[1]), int(r[2]), float(r[3])) for r in rows):
        G = oracle.setup(A, kmax, 1, 0.0).to_scipy().toarray()
        assert abs(G[i, j] - val) <= 1e-15 * max(1.0, abs(val)), (kmax, i, j)


# --------------------------------------------------------------------------------------
# P1: full lower pattern reproduces the exact inverse Cholesky factor
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("n,seed", [(2, 1), (5, 2), (8, 3), (10, 4)])
def test_full_pattern_is_inverse_cholesky(n, seed):
    """With k_max*s >= n-1 and eps = 0 every row fills its whole lower part (dense SPD A has
    generically nonzero gradients), so G = chol(A)^-1 (the Frobenius minimiser of eq. Froben_1
    over all lower-triangular matrices is L^-1 up to the diagonal scaling of eq. diagScal).
    Catches: wrong Cholesky indexing, transposed solve, wrong diagonal scaling."""
    a = synth.random_spd_dense(n, seed)
    A = synth.CSR.from_dense(a)
    G = oracle.setup(A, n - 1, 1, 0.0).to_scipy().toarray()
    Linv = np.linalg.inv(np.linalg.cholesky(a))
    np.testing.assert_allclose(G, Linv, rtol=1e-11, atol=1e-13 * np.abs(Linv).max())
    np.testing.assert_allclose(G @ a @ G.T, np.eye(n), atol=1e-12)
    G3 = oracle.setup(A, 1, n - 1, 0.0).to_scipy().toarray()  # all positions in one step
    np.testing.assert_allclose(G3, Linv, rtol=1e-11, atol=1e-13 * np.abs(Linv).max())


# --------------------------------------------------------------------------------------
# P2/P3: per-row normalisation and the defining equations
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("make,kmax,s", [(lambda: synth.lap7(9), 5, 1), (_elast_small, 10, 2),
                                         (_aniso_small, 5, 2)])
def test_unit_diagonal_and_defining_equations(make, kmax, s):
    """diag(G A G^T) = I (eq. diagScal) and (A g_i)_j = 0 for j in P_i \\ {i} (eq. blocksys).
    Catches: 1/psi instead of psi^-1/2 scaling, a gather that misses entries."""
    A = make()
    G = oracle.setup(A, kmax, s, 1e-2)
    Gs = G.to_scipy()
    As = A.to_scipy()
    d = (Gs @ As @ Gs.T).diagonal()
    np.testing.assert_allclose(d, 1.0, rtol=1e-12)
    AGt = (As @ Gs.T).tocsc()  # column i = A g_i
    absA = abs(As)
    absG = abs(Gs)
    scale = (absA @ absG.T).tocsc()
    for i in range(A.n):
        P = G.col[G.row_ptr[i]:G.row_ptr[i + 1]]
        assert P[-1] == i and np.all(np.diff(P) > 0) and np.all(P <= i)
        col = AGt[:, i].toarray().ravel()
        sc = scale[:, i].toarray().ravel()
        for j in P[:-1]:
            assert abs(col[j]) <= 1e-12 * sc[j], (i, j)
        # (A g_i)_i = 1 / G_ii (eq. syst_3 with the scaling of eq. diagScal)
        assert abs(col[i] * G.val[G.row_ptr[i + 1] - 1] - 1.0) < 1e-12


# --------------------------------------------------------------------------------------
# P10: every row equals the last row of chol(A[P,P])^-1 computed by LAPACK
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("make,kmax,s", [(_elast_small, 10, 2), (_aniso_small, 5, 1)])
def test_rows_match_lapack(make, kmax, s):
    A = make()
    a = dense(A)
    G = oracle.setup(A, kmax, s, 1e-2)
    for i in range(0, A.n, 3):
        P = G.col[G.row_ptr[i]:G.row_ptr[i + 1]]
        L = sla.cholesky(a[np.ix_(P, P)], lower=True)
        want = sla.solve_triangular(L.T, np.eye(len(P))[-1], lower=False)
        got = G.val[G.row_ptr[i]:G.row_ptr[i + 1]]
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-14 * np.abs(want).max())
        # psi after the last step = L_mm^2 = Schur complement a_ii - A[i,Pb] A[Pb,Pb]^-1 A[Pb,i]
        k = G.rows.steps[i]
        if k > 0:
            Pb = P[:-1]
            schur = a[i, i] - a[i, Pb] @ np.linalg.solve(a[np.ix_(Pb, Pb)], a[Pb, i])
            assert abs(G.rows.psi[i, k] - schur) <= 1e-12 * a[i, i]


# --------------------------------------------------------------------------------------
# P4 / P5: diagonal matrix, k_max = 0 (Jacobi), identity preconditioner (plain CG)
# --------------------------------------------------------------------------------------
def test_diagonal_matrix():
    d = synth.uniform(5, 3, 37, 0.5, 9.0)
    A = synth.CSR.from_dense(np.diag(d))
    G = oracle.setup(A, 4, 2, 1e-2)
    np.testing.assert_array_equal(G.row_ptr, np.arange(38))
    np.testing.assert_allclose(G.val, d ** -0.5, rtol=1e-15)
    assert np.all(G.rows.reason == oracle.STOP_NOCAND) and np.all(G.rows.steps == 0)


def test_kmax0_is_jacobi_and_matches_scipy_cg():
    """k_max = 0 gives G = D^-1/2, so PCG is Jacobi-PCG (the paper's baseline, Sec. 5.2).
    Cross-checked against SciPy's CG with M = D^-1 (independent implementation)."""
    P = synth.poisson7(12)
    A = P.A
    G = oracle.setup(A, 0, 1, 1e-2)
    np.testing.assert_allclose(G.val, dense(A).diagonal() ** -0.5, rtol=1e-15)
    res = oracle.pcg(A, G, P.b, 1e-8)
    assert res.status == oracle.OK
    As = A.to_scipy()
    dinv = 1.0 / As.diagonal()
    M = spla.LinearOperator(As.shape, matvec=lambda v: dinv * v)
    its = []
    x_sc, info = spla.cg(As, P.b, rtol=1e-8, atol=0.0, M=M, maxiter=10 * A.n, callback=lambda xk: its.append(1))
    assert info == 0
    assert abs(len(its) - res.iters) <= 1
    assert np.linalg.norm(res.x - x_sc) <= 1e-6 * np.linalg.norm(x_sc)


@pytest.mark.parametrize("make", [lambda: synth.lap7(10), lambda: synth.elast27(4, 1.0, 3)])
def test_plain_cg_against_direct_solve(make):
    """M = I: plain CG; error against a sparse direct solve bounded by kappa_2(A) * rtol."""
    A = make()
    b = synth.matvec(A, synth.uniform(9, 1, A.n))
    res = oracle.pcg(A, None, b, 1e-10)
    assert res.status == oracle.OK
    xs = spla.spsolve(A.to_scipy().tocsc(), b)
    ev = np.linalg.eigvalsh(dense(A))
    kappa = ev[-1] / ev[0]
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) <= kappa * 1e-10
    assert res.true_relres <= 2e-10


def test_pcg_zero_rhs_and_x0_resume():
    P = synth.poisson7(8)
    G = oracle.setup(P.A, 3, 1, 1e-2)
    r0 = oracle.pcg(P.A, G, np.zeros(P.n))
    assert r0.iters == 0 and np.all(r0.x == 0)
    full = oracle.pcg(P.A, G, P.b, 1e-8)
    part = oracle.pcg(P.A, G, P.b, 1e-8, maxit=5)
    assert part.status == oracle.ERR_NOT_CONVERGED and part.iters == 5
    rest = oracle.pcg(P.A, G, P.b, 1e-8, x0=part.x)
    assert rest.status == oracle.OK
    assert np.linalg.norm(rest.x - P.x_true) <= 1e-6 * np.linalg.norm(P.x_true)
    assert np.linalg.norm(full.x - P.x_true) <= 1e-6 * np.linalg.norm(P.x_true)


# --------------------------------------------------------------------------------------
# P6: the Kaporin number (eqs. kap, kap2) is >= 1, equals (prod psi / det A)^(1/n), and
#     psi_{k,i} never increases along the adaptive steps
# --------------------------------------------------------------------------------------
def _kaporin_eig(G, a):
    ev = np.linalg.eigvalsh(G @ a @ G.T)
    return np.mean(ev) / np.exp(np.mean(np.log(ev)))


@pytest.mark.parametrize("make", [lambda: synth.lap7(5, 4, 3), lambda: synth.elast27(3, 1.0, 11),
                                  lambda: synth.CSR.from_dense(synth.random_spd_dense(9, 5))])
def test_kaporin_number(make):
    A = make()
    a = dense(A)
    n = A.n
    _, logdet = np.linalg.slogdet(a)
    prev = np.inf
    for kmax in range(0, 6):
        G = oracle.setup(A, kmax, 1, 0.0)
        Gd = G.to_scipy().toarray()
        kap = _kaporin_eig(Gd, a)
        last = G.rows.psi[np.arange(n), G.rows.steps]
        kap2 = np.exp((np.sum(np.log(last)) - logdet) / n)
        assert kap >= 1.0 - 1e-12
        assert abs(kap - kap2) <= 1e-10 * kap
        assert kap2 <= prev * (1 + 1e-12)
        prev = kap2
        ps = G.rows.psi
        for i in range(n):
            h = ps[i, : G.rows.steps[i] + 1]
            assert np.all(h[1:] <= h[:-1] * (1 + 1e-14))
            assert h[0] == a[i, i]


# --------------------------------------------------------------------------------------
# P7: step-1 closed form and the tie rule on the 7-point stencil
# --------------------------------------------------------------------------------------
def test_step1_closed_form_and_ties():
    """Step 1: v_j = a_ji a_ii^{-1/2}.  On the 7-point Laplacian the three lower neighbours
    tie exactly and the smallest column (the z-neighbour i - nx*ny) wins.  The row is then
    the 2x2 solve: G_ii = 1/sqrt(35/6), G_i,j = 1/(6 sqrt(35/6)), psi_1 = 35/6.
    Catches: a broken tie rule, a sign error in the solve, a wrong psi."""
    nx = 6
    A = synth.lap7(nx)
    G = oracle.setup(A, 1, 1, 0.0)
    c = math.sqrt(35.0 / 6.0)
    for i in range(A.n):
        x, y, z = i % nx, (i // nx) % nx, i // (nx * nx)
        lower = [j for j, ok in ((i - nx * nx, z > 0), (i - nx, y > 0), (i - 1, x > 0)) if ok]
        P = list(G.col[G.row_ptr[i]:G.row_ptr[i + 1]])
        if not lower:
            assert P == [i]
            continue
        assert P == [lower[0], i], (i, P)
        v = G.val[G.row_ptr[i]:G.row_ptr[i + 1]]
        assert abs(v[1] - 1 / c) < 1e-15 and abs(v[0] - 1 / (6 * c)) < 1e-15
        assert abs(G.rows.psi[i, 1] - 35.0 / 6.0) < 1e-14


def test_exit_criterion_direction():
    """psi_1/psi_0 = 35/36 = 0.9722 on interior 7-point rows: eps = 0.98 stops every row that
    grew after step 1, eps = 0.97 lets them continue (eq. exit_crit)."""
    A = synth.lap7(6)
    G98 = oracle.setup(A, 4, 1, 0.98)
    G97 = oracle.setup(A, 4, 1, 0.97)
    grew = G98.rows.steps > 0
    assert np.all(G98.rows.reason[grew] == oracle.STOP_EPS)
    assert np.all(G98.rows.m[grew] == 2)
    idx = np.arange(A.n)
    interior = (idx % 6 > 0) & ((idx // 6) % 6 > 0) & (idx // 36 > 0)
    assert np.all(G97.rows.steps[interior] >= 2) and np.all(G97.rows.m[interior] > 2)


# --------------------------------------------------------------------------------------
# P8: exact pattern counts on the 20^3 7-point problem
# --------------------------------------------------------------------------------------
def test_poisson20_exact_counts():
    """For the 7-point M-matrix every structural candidate has a nonzero gradient and the
    eps = 1e-2 test never fires (psi_k/psi_0 >= 1/2), so m_i = min(6, i+1) and
    nnz(G) = 1+2+3+4+5 + 6*7995 = 47,985."""
    P = synth.poisson7(20)
    G = oracle.setup(P.A, 5, 1, 1e-2)
    np.testing.assert_array_equal(G.rows.m, np.minimum(6, np.arange(P.n) + 1))
    assert G.nnz == 47985
    last = G.rows.psi[np.arange(P.n), G.rows.steps]
    assert np.all(last / 6.0 >= 0.5)


# --------------------------------------------------------------------------------------
# P11: application z = G^T (G r) against SciPy
# --------------------------------------------------------------------------------------
def test_apply_against_scipy():
    A = _elast_small()
    G = oracle.setup(A, 6, 2, 1e-2)
    r = synth.uniform(4, 2, A.n)
    Gs = G.to_scipy()
    np.testing.assert_allclose(oracle.apply(G, r), Gs.T @ (Gs @ r), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(oracle.spmv(A, r), A.to_scipy() @ r, rtol=1e-13, atol=1e-13)


# --------------------------------------------------------------------------------------
# brute force on tiny inputs: the selection is the top-s of |A g| outside the pattern
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_selection_brute_force(seed):
    """Re-derive one growth step with dense algebra: from the k-1 pattern, compute
    w = A g over all j < i, drop the pattern, and take the s largest |w| (no ties occur on
    random dense data); the k-step pattern must equal the (k-1) pattern plus those."""
    n = 9
    a = synth.random_spd_dense(n, 40 + seed)
    # sparsify while staying SPD: keep a band plus random entries, then add diagonal weight
    mask = (np.abs(np.subtract.outer(np.arange(n), np.arange(n))) <= 2)
    a = np.where(mask | mask.T, a, 0.0)
    a += np.diag(np.abs(a).sum(1))
    A = synth.CSR.from_dense(a)
    s = 2
    for k in range(1, 4):
        Gp = oracle.setup(A, k - 1, s, 0.0).to_scipy().toarray()
        Gk = oracle.setup(A, k, s, 0.0)
        for i in range(n):
            prevP = set(np.nonzero(Gp[i])[0])
            w = a @ Gp[i]
            cand = [j for j in range(i) if j not in prevP and abs(w[j]) > 2.0 ** -40 * max(
                [abs(w[q]) for q in range(i) if q not in prevP] + [0.0])]
            cand.sort(key=lambda j: (-abs(w[j]), j))
            want = sorted(prevP | set(cand[:s]))
            got = list(Gk.col[Gk.row_ptr[i]:Gk.row_ptr[i + 1]])
            assert got == want, (k, i)


# --------------------------------------------------------------------------------------
# error statuses
# --------------------------------------------------------------------------------------
def test_errors():
    bad = synth.CSR(np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0, 1.0]))
    assert oracle.check_csr(bad) == oracle.ERR_BAD_MATRIX
    unsorted = synth.CSR(np.array([0, 2, 4], np.int32), np.array([1, 0, 0, 1], np.int32), np.ones(4))
    assert oracle.check_csr(unsorted) == oracle.ERR_BAD_MATRIX
    indef = synth.CSR.from_dense(np.array([[1.0, 2.0], [2.0, 1.0]]))
    with pytest.raises(oracle.OracleError) as e:
        oracle.setup(indef, 1, 1, 0.0)
    assert e.value.code == oracle.ERR_NOT_SPD
    negd = synth.CSR.from_dense(np.array([[1.0, 0.0], [0.0, -1.0]]))
    with pytest.raises(oracle.OracleError) as e:
        oracle.setup(negd, 1, 1, 0.0)
    assert e.value.code == oracle.ERR_NOT_SPD
    with pytest.raises(oracle.OracleError):
        oracle.setup(negd, -1, 1, 0.0)


def test_row_subset_matches_full_and_thread_count():
    """Rows are independent (Sec. 2): any subset, in any order, on any number of threads
    gives the same rows bit for bit."""
    A = _elast_small()
    full = oracle.setup_rows(A, 8, 2, 1e-2, nthreads=1)
    rows = np.array([A.n - 1, 0, 17, 200, 201, 57], np.int32)
    sub = oracle.setup_rows(A, 8, 2, 1e-2, rows=rows, nthreads=3)
    np.testing.assert_array_equal(sub.cols, full.cols[rows])
    np.testing.assert_array_equal(sub.vals, full.vals[rows])
    many = oracle.setup_rows(A, 8, 2, 1e-2, nthreads=4)
    np.testing.assert_array_equal(many.vals, full.vals)
