"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Bars (from the method's arithmetic):
  * patterns of G: identical (the selection is an integer decision; both sides use the same
    tie band, so rounding noise in the gradient cannot flip it);
  * values of G: within 1e-10 relative per row (infinity norm), the independent bar.  The
    default (inverse-factor) form rounds differently from the oracle's Cholesky factorisation
    and meets only this bar; the Cholesky form (AFSAI_OPT_SETUP_FORM = 1) follows the oracle's
    rounding sequence (growth order, reciprocal pivots), so where it is forced the fraction of
    bitwise-equal values is checked too;
  * psi, steps and stop reasons per row: identical values / within 1e-12 relative;
  * PCG: the same iteration count and the solution within 1e-10 relative (FP64 G); with FP32
    storage of G: converged to the same rtol, iteration count within 2, and
    ||x - x_oracle|| / ||x_oracle|| <= 1e-6.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

G_RTOL = 1e-10
X_RTOL = 1e-10


@pytest.fixture(scope="module")
def af():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2010_14175_amd as af

    af.lib()
    return af


def _dev(af, A):
    return af.DeviceCSR.from_host(A)


def _vec(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()


def _gpu_factor(af, P):
    rp, ci, va = P.export()
    return rp.cpu().numpy(), ci.cpu().numpy(), va.cpu().numpy()


def compare_factor(af, A, kmax, s, eps, g_prec=0, rows=None, form=0):
    """Runs the GPU setup (form: 0 automatic, 1 Cholesky, 2 inverse factor) and the oracle;
    returns statistics; asserts the bars (vectorised over the rows, so that every row of the
    full-size workloads is checked)."""
    dA = _dev(af, A)
    try:
        af.set_option(af.OPT_SETUP_FORM, form)
        P = af.setup(dA, kmax, s, eps, g_prec=g_prec)
    finally:
        af.set_option(af.OPT_SETUP_FORM, 0)
    rp, ci, va = _gpu_factor(af, P)
    psi, steps, reason = (t.cpu().numpy() for t in P.export_rows())
    info = P.info()
    if rows is None:
        R = oracle.setup_rows(A, kmax, s, eps)
        rows = np.arange(A.n)
    else:
        R = oracle.setup_rows(A, kmax, s, eps, rows=rows)
    rows = np.asarray(rows, np.int64)
    lens = (rp[rows + 1] - rp[rows]).astype(np.int64)
    bad = np.nonzero(lens != R.m)[0]
    assert bad.size == 0, f"row {rows[bad[0]]}: pattern size {lens[bad[0]]} vs oracle {R.m[bad[0]]}"
    # the GPU rows padded like the oracle's (columns -1, values 0 past m)
    mmax = R.cols.shape[1]
    slot = np.arange(mmax)[None, :]
    live = slot < lens[:, None]
    src = np.where(live, rp[rows][:, None] + slot, 0)
    gcols = np.where(live, ci[src] if ci.size else 0, -1)
    gvals = np.where(live, va[src] if va.size else 0.0, 0.0)
    badc = np.nonzero((gcols != R.cols).any(axis=1))[0]
    assert badc.size == 0, f"row {rows[badc[0]]} pattern: {gcols[badc[0]]} vs oracle {R.cols[badc[0]]}"
    ov = np.where(live, R.vals, 0.0)
    if g_prec == 0:
        scale = np.max(np.abs(ov), axis=1)
        err = np.max(np.abs(gvals - ov), axis=1) / np.where(scale > 0, scale, 1.0)
        worst = int(np.argmax(err)) if err.size else 0
        assert err.size == 0 or err[worst] <= G_RTOL, f"row {rows[worst]}: relative error {err[worst]:.3e}"
        nbit = int(np.sum((gvals.view(np.int64) == ov.view(np.int64)) & live))
    else:
        # FP32 storage: the stored value is the FP64 result rounded to FP32 (half an FP32 ulp,
        # 2^-24 relative) of a value within rounding of the oracle's
        badv = np.nonzero((np.abs(gvals - ov) > 2.0 ** -23 * np.abs(ov)).any(axis=1))[0]
        assert badv.size == 0, f"row {rows[badv[0]]}: FP32 values beyond FP32 rounding of the oracle's"
        nbit = 0
    ntot = int(lens.sum())
    bads = np.nonzero((steps[rows] != R.steps) | (reason[rows] != R.reason))[0]
    assert bads.size == 0, f"row {rows[bads[0]]}: steps/reason"
    po = R.psi[np.arange(len(rows)), R.steps]
    badp = np.nonzero(np.abs(psi[rows] - po) > 1e-12 * np.abs(po))[0]
    assert badp.size == 0, f"row {rows[badp[0]]}: psi {psi[rows[badp[0]]]} vs oracle {po[badp[0]]}"
    return {"P": P, "dA": dA, "info": info, "bitwise": nbit / max(1, ntot), "nnz": ntot}


# --------------------------------------------------------------------------------------
# setup parity
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("form", [0, 1])
def test_setup_poisson20(af, form):
    """20^3 7-point Laplacian, k_max = 5, s = 1, eps = 1e-2 (nnz(G) = 47,985 exactly)."""
    Pb = synth.poisson7(20)
    r = compare_factor(af, Pb.A, 5, 1, 1e-2, form=form)
    assert r["info"].nnz_g == 47985
    if form == 1:
        assert r["bitwise"] == 1.0, r["bitwise"]


@pytest.mark.parametrize("case", ["tridiag3_k1", "tridiag3_k2", "dense8_full", "diag", "one", "two",
                                  "kmax0", "poisson_ragged", "aniso", "lognormal7"])
def test_setup_small_cases(af, case):
    if case.startswith("tridiag3"):
        A = synth.CSR.from_dense(np.array([[4.0, 1, 0], [1, 4, 1], [0, 1, 4]]))
        r = compare_factor(af, A, 1 if case.endswith("k1") else 2, 1, 0.0)
    elif case == "dense8_full":
        A = synth.CSR.from_dense(synth.random_spd_dense(8, 3))
        r = compare_factor(af, A, 7, 1, 0.0)
        G = np.zeros((8, 8))
        rp, ci, va = _gpu_factor(af, r["P"])
        for i in range(8):
            G[i, ci[rp[i]:rp[i + 1]]] = va[rp[i]:rp[i + 1]]
        a = A.to_scipy().toarray()
        np.testing.assert_allclose(G @ a @ G.T, np.eye(8), atol=1e-12)
    elif case == "diag":
        A = synth.CSR.from_dense(np.diag(synth.uniform(5, 3, 37, 0.5, 9.0)))
        compare_factor(af, A, 4, 2, 1e-2)
    elif case == "one":
        A = synth.CSR.from_dense(np.array([[2.5]]))
        compare_factor(af, A, 3, 1, 1e-2)
    elif case == "two":
        A = synth.CSR.from_dense(np.array([[2.0, -1.0], [-1.0, 2.0]]))
        compare_factor(af, A, 3, 2, 0.0)
    elif case == "kmax0":
        A = synth.elast27(4, 1.0, 3)
        compare_factor(af, A, 0, 1, 1e-2)
    elif case == "poisson_ragged":
        A = synth.lap7(13, 7, 5)
        compare_factor(af, A, 6, 2, 1e-2)
    elif case == "aniso":
        A = synth.lap7(11, 9, 7, (1.0, 1.0, 500.0))
        compare_factor(af, A, 5, 1, 1e-2)
    elif case == "lognormal7":
        A = synth.lap7_lognormal(12, 10, 9, 1.0, 4)
        compare_factor(af, A, 5, 2, 1e-2)


@pytest.mark.parametrize("form", [0, 1])
def test_setup_elasticity_reduced(af, form):
    """27-point 3-dof heterogeneous operator at 12^3 nodes (5,184 rows), k_max = 10, s = 2."""
    A = synth.elast27(12, 1.0, 2)
    r = compare_factor(af, A, 10, 2, 1e-2, form=form)
    if form == 1:
        assert r["bitwise"] == 1.0, r["bitwise"]


@pytest.mark.parametrize("form", [0, 1])
def test_setup_elasticity_24(af, form):
    """24^3 nodes (41,472 rows): the reduced form of the 64^3 workload, every row checked."""
    A = synth.elast27(24, 1.0, 2)
    r = compare_factor(af, A, 10, 2, 1e-2, form=form)
    if form == 1:
        assert r["bitwise"] == 1.0, r["bitwise"]


@pytest.mark.parametrize("form", [0, 1])
def test_setup_large_pattern(af, form):
    """k_max = 15, s = 3 (46 entries per row, the 150^3 workload's parameters) on a small grid,
    sigma = 2."""
    A = synth.elast27(7, 2.0, 5)
    compare_factor(af, A, 15, 3, 1e-2, form=form)


@pytest.mark.parametrize("make,kmax,s", [(lambda: synth.lap7(9, 8, 7), 5, 1), (lambda: synth.lap7(9, 8, 7), 7, 2),
                                         (lambda: synth.elast27(6, 1.0, 2), 5, 3),
                                         (lambda: synth.elast27(7, 2.0, 5), 10, 2),
                                         (lambda: synth.elast27(6, 2.0, 5), 21, 3),
                                         (lambda: synth.elast27(5, 1.0, 7), 9, 7)])
def test_setup_inverse_factor_shapes(af, make, kmax, s):
    """The inverse-factor form over its lane-group shapes (8, 16, 32 and 64 lanes per row) and
    block sizes (s above the rows appended per block), against the oracle."""
    A = make()
    compare_factor(af, A, kmax, s, 1e-2, form=2)


@pytest.mark.parametrize("make,kmax,s", [(lambda: synth.elast27(9, 1.0, 2), 10, 2), (lambda: synth.lap7(14), 5, 1),
                                         (lambda: synth.lap7(12), 5, 3),
                                         (lambda: synth.elast27(6, 2.0, 5), 15, 3)])
def test_setup_inverse_factor_table_sizes(af, make, kmax, s):
    """The inverse-factor form's result does not depend on the table size (slots only rank
    candidates; every table size gives the same G bit for bit) and agrees with the Cholesky
    form to rounding.  Tables of 128 and 256 slots put the 7-point rows (6 and 16 positions)
    on groups of 8 or 16 lanes, where a lane scans 8 or 16 slots (16 in unrolled steps rather
    than all at once); the 27-point rows run 64 lanes per row."""
    A = make()
    dA = _dev(af, A)
    outs = []
    try:
        af.set_option(af.OPT_SETUP_FORM, 2)
        for cap in (0, 128, 256, 1024):
            af.set_option(af.OPT_SETUP_TABLE, cap)
            outs.append(_gpu_factor(af, af.setup(dA, kmax, s, 1e-2)))
        af.set_option(af.OPT_SETUP_TABLE, 0)
        af.set_option(af.OPT_SETUP_FORM, 1)
        chol = _gpu_factor(af, af.setup(dA, kmax, s, 1e-2))
    finally:
        af.set_option(af.OPT_SETUP_FORM, 0)
        af.set_option(af.OPT_SETUP_TABLE, 0)
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(outs[0][0], chol[0])
    np.testing.assert_array_equal(outs[0][1], chol[1])
    np.testing.assert_allclose(outs[0][2], chol[2], rtol=G_RTOL, atol=G_RTOL * np.abs(chol[2]).max())


def test_setup_overflow_retry(af):
    """Random sparse SPD rows reaching all over the matrix, k_max*s = 63: patterns touch more
    candidate columns than the first on-chip table holds; those rows are redone with a larger
    table and must still match the oracle."""
    A = synth.random_sparse_spd(4000, 60, 8)
    rows = np.concatenate([np.arange(0, 4000, 97), np.arange(3990, 4000)]).astype(np.int32)
    r = compare_factor(af, A, 21, 3, 0.0, rows=rows)
    assert r["info"].rows_retried > 0


def test_setup_fp32_storage(af):
    A = synth.elast27(10, 1.0, 2)
    compare_factor(af, A, 10, 2, 1e-2, g_prec=1)


@pytest.mark.parametrize("make,kmax,s", [(lambda: synth.elast27(10, 1.0, 6), 10, 2), (lambda: synth.lap7(16), 5, 1),
                                         (lambda: synth.elast27(6, 2.0, 5), 7, 4)])
def test_setup_forms_identical(af, make, kmax, s):
    """Cholesky form: appending one or two rows per factor update instead of up to four, and
    any first table size, give G bit for bit identical."""
    A = make()
    dA = _dev(af, A)
    try:
        af.set_option(af.OPT_SETUP_FORM, 1)
        ref = _gpu_factor(af, af.setup(dA, kmax, s, 1e-2))
        outs = []
        for g in (1, 2):
            af.set_option(af.OPT_SETUP_GROUP, g)
            outs.append(_gpu_factor(af, af.setup(dA, kmax, s, 1e-2)))
        af.set_option(af.OPT_SETUP_GROUP, 0)
        af.set_option(af.OPT_SETUP_TABLE, 128)
        outs.append(_gpu_factor(af, af.setup(dA, kmax, s, 1e-2)))
    finally:
        af.set_option(af.OPT_SETUP_GROUP, 0)
        af.set_option(af.OPT_SETUP_TABLE, 0)
        af.set_option(af.OPT_SETUP_FORM, 0)
    for o in outs:
        for a, b in zip(ref, o):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("slots", [1, 2])
@pytest.mark.parametrize("make,kmax,s", [(lambda: synth.elast27(12, 1.0, 2), 10, 2), (lambda: synth.lap7(16), 5, 1),
                                         (lambda: synth.random_sparse_spd(3000, 40, 3), 10, 3),
                                         (lambda: synth.elast27(7, 2.0, 5), 15, 3),
                                         (lambda: synth.elast27(6, 1.0, 3), 21, 3)])
def test_setup_slot_lists(af, slots, make, kmax, s):
    """Cholesky form: the table slots of the pattern rows' entries kept in LDS (1) or in
    registers (2): both give the oracle's patterns and values (bitwise here), and equal each
    other bit for bit."""
    A = make()
    try:
        af.set_option(af.OPT_SETUP_SLOTS, slots)
        r = compare_factor(af, A, kmax, s, 1e-2, form=1)
        other = 1 if slots == 2 else 2
        af.set_option(af.OPT_SETUP_SLOTS, other)
        af.set_option(af.OPT_SETUP_FORM, 1)
        o = _gpu_factor(af, af.setup(r["dA"], kmax, s, 1e-2))
    finally:
        af.set_option(af.OPT_SETUP_SLOTS, 0)
        af.set_option(af.OPT_SETUP_FORM, 0)
    assert r["bitwise"] == 1.0, r["bitwise"]
    for a, b in zip(_gpu_factor(af, r["P"]), o):
        np.testing.assert_array_equal(a, b)


def test_setup_slot_lists_refused(af):
    """Register slot lists need rows of at most 128 entries: asked for on a matrix with longer
    rows the setup reports an invalid argument instead of running."""
    A = synth.random_sparse_spd(2000, 90, 4)
    assert np.diff(A.row_ptr).max() > 128
    dA = _dev(af, A)
    try:
        af.set_option(af.OPT_SETUP_SLOTS, 2)
        with pytest.raises(af.AfsaiError) as e:
            af.setup(dA, 2, 1, 1e-2)
        assert e.value.code == af.ERR_INVALID_ARG
    finally:
        af.set_option(af.OPT_SETUP_SLOTS, 0)


@pytest.mark.parametrize("make,kmax,s,min_same", [(lambda: synth.poisson7(16).A, 5, 1, 0.5),
                                                  (lambda: synth.elast27(8, 1.0, 2), 10, 2, 0.5),
                                                  (lambda: synth.lap7_lognormal(12, 11, 10, 1.0, 3), 5, 1, 0.5)])
def test_setup_f32_against_oracle(af, make, kmax, s, min_same):
    """Fully single-precision setup (gradient, selection, factorisation in FP32) against the FP64
    oracle, the evaluation the paper's single-precision remark calls for: the share of rows
    whose pattern is the oracle's, the relative error of G on those rows (FP32 rounding of
    small dense solves), and PCG to rtol 1e-8 with either G taking about the same number of
    iterations.  Rows may pick other columns where FP64 gradients tie within FP32 rounding."""
    A = make()
    dA = _dev(af, A)
    P = af.setup(dA, kmax, s, 1e-2, setup_f32=True)
    rp, ci, va = _gpu_factor(af, P)
    R = oracle.setup_rows(A, kmax, s, 1e-2)
    same, errs = 0, []
    for i in range(A.n):
        m = R.m[i]
        cols = ci[rp[i]:rp[i + 1]]
        if len(cols) == m and np.array_equal(cols, R.cols[i, :m]):
            same += 1
            ov = R.vals[i, :m]
            errs.append(np.max(np.abs(va[rp[i]:rp[i + 1]] - ov)) / np.max(np.abs(ov)))
    assert same / A.n >= min_same, f"only {same}/{A.n} rows with the oracle's pattern"
    assert max(errs) < 1e-4, max(errs)
    b = A.to_scipy() @ synth.uniform(3, 4, A.n, -1.0, 1.0)
    x32, i32 = af.pcg_solve(dA, P, _vec(b), rtol=1e-8)
    x64, i64 = af.pcg_solve(dA, af.setup(dA, kmax, s, 1e-2), _vec(b), rtol=1e-8)
    assert i32.converged and i32.true_relres < 2e-8
    assert abs(i32.iters - i64.iters) <= max(2, i64.iters // 10), (i32.iters, i64.iters)


@pytest.mark.parametrize("make,kmax,s", [(lambda: synth.elast27(12, 1.0, 2), 10, 2),
                                         (lambda: synth.lap7_lognormal(12, 11, 10, 1.0, 3), 5, 1),
                                         (lambda: synth.elast27(7, 2.0, 5), 15, 3),
                                         (lambda: synth.poisson7(14).A, 5, 1)])
def test_setup_grad_f32_against_oracle(af, make, kmax, s):
    """The precision form's gradient (FP32 values of A in the ranking product, FP64 systems,
    factorisation and g) against the FP64 oracle: nearly every row keeps the oracle's pattern
    (a row changes only where two candidates' gradients are within FP32 rounding of each
    other), and on those rows G is the FP64 result (within 1e-10 of the oracle, since the
    dense systems are gathered in FP64); PCG to rtol 1e-8 takes about the FP64 setup's
    iterations.  On the constant-coefficient Laplacian the FP32 values are exact, so every
    pattern is the oracle's."""
    A = make()
    dA = _dev(af, A)
    P = af.setup(dA, kmax, s, 1e-2, grad_f32=True)
    rp, ci, va = _gpu_factor(af, P)
    R = oracle.setup_rows(A, kmax, s, 1e-2)
    same, worst = 0, 0.0
    for i in range(A.n):
        m = R.m[i]
        cols = ci[rp[i]:rp[i + 1]]
        if len(cols) == m and np.array_equal(cols, R.cols[i, :m]):
            same += 1
            ov = R.vals[i, :m]
            worst = max(worst, np.max(np.abs(va[rp[i]:rp[i + 1]] - ov)) / np.max(np.abs(ov)))
    exact = np.array_equal(A.val.astype(np.float32).astype(np.float64), A.val)
    print(f"grad_f32: {same}/{A.n} rows with the oracle's pattern, worst G error on them {worst:.2e}")
    assert same == A.n if exact else same >= 0.98 * A.n, (same, A.n)
    assert worst <= G_RTOL, worst
    b = A.to_scipy() @ synth.uniform(3, 4, A.n, -1.0, 1.0)
    x32, i32 = af.pcg_solve(dA, P, _vec(b), rtol=1e-8)
    x64, i64 = af.pcg_solve(dA, af.setup(dA, kmax, s, 1e-2), _vec(b), rtol=1e-8)
    assert i32.converged and i32.true_relres < 2e-8
    assert abs(i32.iters - i64.iters) <= max(2, i64.iters // 10), (i32.iters, i64.iters)


def test_setup_grad_f32_refused(af):
    """The FP32 gradient belongs to the inverse-factor form with FP64 setup arithmetic."""
    A = synth.elast27(5, 1.0, 2)
    dA = _dev(af, A)
    with pytest.raises(af.AfsaiError) as e:
        af.setup(dA, 5, 2, 1e-2, grad_f32=True, setup_f32=True)
    assert e.value.code == af.ERR_INVALID_ARG
    try:
        af.set_option(af.OPT_SETUP_FORM, 1)
        with pytest.raises(af.AfsaiError) as e:
            af.setup(dA, 5, 2, 1e-2, grad_f32=True)
        assert e.value.code == af.ERR_INVALID_ARG
    finally:
        af.set_option(af.OPT_SETUP_FORM, 0)


def test_setup_f32_refused(af):
    A = synth.random_sparse_spd(2000, 90, 4)
    with pytest.raises(af.AfsaiError) as e:
        af.setup(_dev(af, A), 2, 1, 1e-2, setup_f32=True)
    assert e.value.code == af.ERR_INVALID_ARG


@pytest.mark.parametrize("gs,un", [(4, 1), (8, 2), (16, 8), (64, 4)])
def test_spmv_shapes(af, gs, un):
    """Every group size / unroll of the CSR products gives the oracle's y within rounding."""
    A = synth.elast27(7, 1.0, 2)
    r = synth.uniform(3, 8, A.n)
    try:
        af.set_option(af.OPT_SPMV_GROUP, gs)
        af.set_option(af.OPT_SPMV_UNROLL, un)
        y = af.spmv(_dev(af, A), _vec(r)).cpu().numpy()
    finally:
        af.set_option(af.OPT_SPMV_GROUP, 0)
        af.set_option(af.OPT_SPMV_UNROLL, 0)
    np.testing.assert_allclose(y, oracle.spmv(A, r), rtol=1e-13, atol=1e-13 * np.abs(y).max())


def test_setup_deterministic(af):
    A = synth.elast27(10, 1.0, 6)
    dA = _dev(af, A)
    P1 = af.setup(dA, 10, 2, 1e-2)
    P2 = af.setup(dA, 10, 2, 1e-2)
    for a, b in zip(_gpu_factor(af, P1), _gpu_factor(af, P2)):
        np.testing.assert_array_equal(a, b)


def test_setup_errors(af):
    indef = synth.CSR.from_dense(np.array([[1.0, 2.0], [2.0, 1.0]]))
    with pytest.raises(af.AfsaiError) as e:
        af.setup(_dev(af, indef), 1, 1, 0.0)
    assert e.value.code == af.ERR_NOT_SPD
    negd = synth.CSR.from_dense(np.array([[1.0, 0.0], [0.0, -1.0]]))
    with pytest.raises(af.AfsaiError) as e:
        af.setup(_dev(af, negd), 1, 1, 0.0)
    assert e.value.code == af.ERR_NOT_SPD
    nodiag = synth.CSR(np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0, 1.0]))
    with pytest.raises(af.AfsaiError) as e:
        af.setup(_dev(af, nodiag), 1, 1, 0.0)
    assert e.value.code == af.ERR_BAD_MATRIX
    unsorted = synth.CSR(np.array([0, 2, 4], np.int32), np.array([1, 0, 0, 1], np.int32), np.array([1.0, 4, 4, 1]))
    with pytest.raises(af.AfsaiError) as e:
        af.setup(_dev(af, unsorted), 1, 1, 0.0, validate=True)
    assert e.value.code == af.ERR_BAD_MATRIX
    asym = synth.CSR.from_dense(np.array([[4.0, 1.0], [1.5, 4.0]]))
    with pytest.raises(af.AfsaiError) as e:
        af.setup(_dev(af, asym), 1, 1, 0.0, validate=True)
    assert e.value.code == af.ERR_BAD_MATRIX
    ok = synth.lap7(5)
    P = af.setup(_dev(af, ok), 3, 1, 1e-2, validate=True)
    assert P.info().nnz_g > 0


# --------------------------------------------------------------------------------------
# apply / SpMV parity
# --------------------------------------------------------------------------------------
def _import_oracle_G(af, G, g_prec=0):
    return af.import_factor(af.DeviceCSR.from_host(G), g_prec=g_prec)


@pytest.mark.parametrize("make", [lambda: synth.lap7(17, 9, 5), lambda: synth.elast27(9, 1.0, 2)])
def test_spmv_and_apply(af, make):
    A = make()
    G = oracle.setup(A, 6, 2, 1e-2)
    r = synth.uniform(3, 4, A.n)
    y = af.spmv(_dev(af, A), _vec(r)).cpu().numpy()
    np.testing.assert_allclose(y, oracle.spmv(A, r), rtol=1e-13, atol=1e-13 * np.abs(y).max())
    P = _import_oracle_G(af, G)
    z = P.apply(_vec(r)).cpu().numpy()
    zo = oracle.apply(G, r)
    np.testing.assert_allclose(z, zo, rtol=1e-12, atol=1e-13 * np.abs(zo).max())


def test_apply_with_long_transpose_rows(af):
    """The 27-point operator with k_max = 15, s = 3 on a 12^3 grid (5,184 rows): 65 rows of G^T
    hold more than 128 entries (up to 190), which the transpose sorts four keys per lane.  The
    setup's G applied as G^T (G r) is within 1e-10 of the oracle's application of its own G, the
    oracle's G imported and applied within 1e-12 of it, and PCG takes the oracle's iterations."""
    Pb = synth.elasticity27(12, 2.0, 5, kmax=15, s=3)
    G = oracle.setup(Pb.A, 15, 3, 1e-2)
    assert np.bincount(np.asarray(G.col), minlength=Pb.n).max() > 128
    dA = _dev(af, Pb.A)
    P = af.setup(dA, 15, 3, 1e-2)
    r = synth.uniform(3, 8, Pb.n, -1.0, 1.0)
    z = P.apply(_vec(r)).cpu().numpy()
    zo = oracle.apply(G, r)
    assert np.linalg.norm(z - zo) <= 1e-10 * np.linalg.norm(zo)
    Pi = _import_oracle_G(af, G)
    zi = Pi.apply(_vec(r)).cpu().numpy()
    np.testing.assert_allclose(zi, zo, rtol=1e-12, atol=1e-13 * np.abs(zo).max())
    x, info = af.pcg_solve(dA, P, _vec(Pb.b), rtol=1e-8)
    ro = oracle.pcg(Pb.A, G, Pb.b, 1e-8)
    assert info.converged and info.iters == ro.iters, (info.iters, ro.iters)
    assert np.linalg.norm(x.cpu().numpy() - ro.x) <= X_RTOL * np.linalg.norm(ro.x)


# --------------------------------------------------------------------------------------
# PCG parity
# --------------------------------------------------------------------------------------
def _pcg_pair(af, Pb, kmax, s, eps=1e-2, g_prec=0, maxit=None):
    dA = _dev(af, Pb.A)
    P = af.setup(dA, kmax, s, eps, g_prec=g_prec)
    x, info = af.pcg_solve(dA, P, _vec(Pb.b), rtol=Pb.rtol, maxit=maxit)
    G = oracle.setup(Pb.A, kmax, s, eps)
    ro = oracle.pcg(Pb.A, G, Pb.b, Pb.rtol, maxit=maxit)
    return x.cpu().numpy(), info, ro


def test_pcg_poisson20(af):
    Pb = synth.poisson7(20)
    x, info, ro = _pcg_pair(af, Pb, 5, 1)
    assert info.converged and info.iters == ro.iters, (info.iters, ro.iters)
    assert np.linalg.norm(x - ro.x) <= X_RTOL * np.linalg.norm(ro.x)
    assert info.true_relres <= 1.1e-8


def test_pcg_elasticity_reduced(af):
    Pb = synth.elasticity27(16)
    x, info, ro = _pcg_pair(af, Pb, 10, 2)
    assert info.converged and info.iters == ro.iters, (info.iters, ro.iters)
    assert np.linalg.norm(x - ro.x) <= X_RTOL * np.linalg.norm(ro.x)


@pytest.mark.parametrize("make", [lambda: synth.elasticity27(16), lambda: synth.elasticity27(11, sigma=2.0, seed=5),
                                  lambda: synth.poisson7(12)])
def test_pcg_column_runs_layout(af, make):
    """A's SELL layout with one column index per run of three consecutive columns (every row of
    a 3-dof 27-point operator; the 11^3 grid leaves a ragged last slice) gives the per-entry
    layout's iterates bit for bit, and the oracle's iteration count and x within 1e-10; a
    matrix without such runs (7-point) keeps the per-entry layout."""
    Pb = make()
    dA = _dev(af, Pb.A)
    P = af.setup(dA, 10, 2, 1e-2)
    b = _vec(Pb.b)
    af.set_option(af.OPT_PCG_FORM, 1)  # the separate-update form multiplies with this layout
    try:
        x1, i1 = af.pcg_solve(dA, P, b, rtol=Pb.rtol)
        af.set_option(af.OPT_SELL_RUNS, 1)
        x0, i0 = af.pcg_solve(dA, P, b, rtol=Pb.rtol)
    finally:
        af.set_option(af.OPT_SELL_RUNS, 0)
        af.set_option(af.OPT_PCG_FORM, 0)
    assert i1.iters == i0.iters and i1.converged
    assert np.array_equal(x1.cpu().numpy(), x0.cpu().numpy())
    G = oracle.setup(Pb.A, 10, 2, 1e-2)
    ro = oracle.pcg(Pb.A, G, Pb.b, Pb.rtol)
    assert i1.iters == ro.iters, (i1.iters, ro.iters)
    assert np.linalg.norm(x1.cpu().numpy() - ro.x) <= X_RTOL * np.linalg.norm(ro.x)


def _broken_runs_elasticity():
    """8^3 27-point 3-dof operator with three symmetric pairs of entries removed from one
    interior row, each from a different run of three columns: the slices keep widths that are
    multiples of three, but that row's and three other rows' triples are no longer runs."""
    import scipy.sparse as sp

    A = synth.elast27(8, 1.0, 2)
    M = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n)).tolil()
    i = 3 * (4 * 64 + 4 * 8 + 4)  # first dof of an interior node
    cols = [c for c in M.rows[i] if c // 3 != i // 3]
    for j in (cols[0], cols[len(cols) // 2 + 1], cols[-1]):
        M[i, j] = 0.0
        M[j, i] = 0.0
    M = M.tocsr()
    M.eliminate_zeros()
    M.sort_indices()
    return synth.CSR(M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64))


def test_pcg_column_runs_rejected(af):
    """A matrix whose triples are not all runs keeps the per-entry layout: the separate-update
    PCG equals the run option switched off bit for bit and the oracle within 1e-10."""
    A = _broken_runs_elasticity()
    lens = np.diff(A.row_ptr)
    assert np.count_nonzero(lens % 3) == 3  # the three partner rows
    assert all(lens[k:k + 64].max() % 3 == 0 for k in range(0, A.n, 64))  # slice widths pass
    assert np.linalg.eigvalsh(_dense(A)).min() > 0.0  # still SPD
    xt = synth.uniform(31, 5, A.n, -1.0, 1.0)
    b = _spmv_host(A, xt)
    dA = _dev(af, A)
    P = af.setup(dA, 10, 2, 1e-2)
    af.set_option(af.OPT_PCG_FORM, 1)
    try:
        x1, i1 = af.pcg_solve(dA, P, _vec(b), rtol=1e-8)
        af.set_option(af.OPT_SELL_RUNS, 1)
        x0, i0 = af.pcg_solve(dA, P, _vec(b), rtol=1e-8)
    finally:
        af.set_option(af.OPT_SELL_RUNS, 0)
        af.set_option(af.OPT_PCG_FORM, 0)
    assert i1.iters == i0.iters and i1.converged
    assert np.array_equal(x1.cpu().numpy(), x0.cpu().numpy())
    G = oracle.setup(A, 10, 2, 1e-2)
    ro = oracle.pcg(A, G, b, 1e-8)
    assert i1.iters == ro.iters, (i1.iters, ro.iters)
    assert np.linalg.norm(x1.cpu().numpy() - ro.x) <= X_RTOL * np.linalg.norm(ro.x)


def _dense(A):
    D = np.zeros((A.n, A.n))
    for r in range(A.n):
        D[r, A.col[A.row_ptr[r]:A.row_ptr[r + 1]]] = A.val[A.row_ptr[r]:A.row_ptr[r + 1]]
    return D


def _spmv_host(A, x):
    y = np.zeros(A.n)
    for r in range(A.n):
        lo, hi = A.row_ptr[r], A.row_ptr[r + 1]
        y[r] = np.dot(A.val[lo:hi], x[A.col[lo:hi]])
    return y


def test_prepared_matrix_column_runs(af):
    """A prepared 3-dof matrix keeps run indices beside its per-entry columns: its PCG in the
    separate-update form (which multiplies with the run layout) and its block products (which
    read the per-entry columns) equal the unprepared calls bit for bit."""
    import torch

    Pb = synth.elasticity27(12, sigma=2.0, seed=7)
    dA = _dev(af, Pb.A)
    P = af.setup(dA, 10, 2, 1e-2)
    b = _vec(Pb.b)
    af.set_option(af.OPT_PCG_FORM, 1)
    try:
        M = af.PreparedMatrix(dA)
        x0, i0 = af.pcg_solve(dA, P, b, rtol=Pb.rtol)
        x1, i1 = M.pcg_solve(P, b, rtol=Pb.rtol)
    finally:
        af.set_option(af.OPT_PCG_FORM, 0)
    assert i0.iters == i1.iters and i1.converged
    assert torch.equal(x0, x1)
    X = torch.from_numpy(synth.uniform(29, 5, Pb.n * 4, -1.0, 1.0).reshape(Pb.n, 4)).cuda()
    assert torch.equal(M.spmm(X), af.spmm(dA, X))
    M.close()
    # the block PCG's products with A over run indices equal the per-entry layout's
    B2 = torch.from_numpy(synth.uniform(37, 5, Pb.n * 2, -1.0, 1.0).reshape(Pb.n, 2)).cuda()
    Xr, ir = af.pcg_solve_multi(dA, P, B2, rtol=1e-8)
    af.set_option(af.OPT_SELL_RUNS, 1)
    try:
        Xe, ie = af.pcg_solve_multi(dA, P, B2, rtol=1e-8)
    finally:
        af.set_option(af.OPT_SELL_RUNS, 0)
    assert [i.iters for i in ir] == [i.iters for i in ie]
    assert torch.equal(Xr, Xe)
    P.close()


def test_pcg_fp32_g(af):
    Pb = synth.elasticity27(16)
    x, info, ro = _pcg_pair(af, Pb, 10, 2, g_prec=1)
    assert info.converged and abs(info.iters - ro.iters) <= 2, (info.iters, ro.iters)
    assert np.linalg.norm(x - ro.x) <= 1e-6 * np.linalg.norm(ro.x)
    assert info.true_relres <= 1.5e-8


def test_pcg_plain_cg_and_jacobi(af):
    Pb = synth.poisson7(14)
    dA = _dev(af, Pb.A)
    x, info = af.pcg_solve(dA, None, _vec(Pb.b), rtol=1e-8)
    ro = oracle.pcg(Pb.A, None, Pb.b, 1e-8)
    assert info.iters == ro.iters
    assert np.linalg.norm(x.cpu().numpy() - ro.x) <= X_RTOL * np.linalg.norm(ro.x)
    xj, ij, roj = _pcg_pair(af, Pb, 0, 1)
    assert ij.iters == roj.iters
    assert np.linalg.norm(xj - roj.x) <= X_RTOL * np.linalg.norm(roj.x)


def test_pcg_edge_cases(af):
    import torch

    Pb = synth.poisson7(9)
    dA = _dev(af, Pb.A)
    P = af.setup(dA, 4, 1, 1e-2)
    G = oracle.setup(Pb.A, 4, 1, 1e-2)
    for maxit in (1, 2, 3, 7):
        xm, im = af.pcg_solve(dA, P, _vec(Pb.b), maxit=maxit)
        rom = oracle.pcg(Pb.A, G, Pb.b, 1e-8, maxit=maxit)
        assert im.iters == maxit
        assert np.linalg.norm(xm.cpu().numpy() - rom.x) <= X_RTOL * np.linalg.norm(rom.x), maxit
    # zero right-hand side
    x, info = af.pcg_solve(dA, P, torch.zeros(Pb.n, dtype=torch.float64, device="cuda"),
                           x=torch.ones(Pb.n, dtype=torch.float64, device="cuda"))
    assert info.iters == 0 and info.converged and float(x.abs().max()) == 0.0
    # maxit reached, then resume from the returned x
    G = oracle.setup(Pb.A, 4, 1, 1e-2)
    x5, info5 = af.pcg_solve(dA, P, _vec(Pb.b), maxit=5)
    ro5 = oracle.pcg(Pb.A, G, Pb.b, 1e-8, maxit=5)
    assert info5.status == af.ERR_NOT_CONVERGED and info5.iters == 5 and not info5.converged
    assert np.linalg.norm(x5.cpu().numpy() - ro5.x) <= X_RTOL * np.linalg.norm(ro5.x)
    x_r, info_r = af.pcg_solve(dA, P, _vec(Pb.b), x=x5.clone())
    ro_r = oracle.pcg(Pb.A, G, Pb.b, 1e-8, x0=ro5.x)
    assert info_r.converged and info_r.iters == ro_r.iters
    # maxit = 0
    x0, info0 = af.pcg_solve(dA, P, _vec(Pb.b), maxit=0)
    assert info0.status == af.ERR_NOT_CONVERGED and info0.iters == 0
    # an indefinite matrix is reported (p.Ap <= 0) by plain CG
    ind = synth.CSR.from_dense(np.diag([1.0, -1.0, 2.0]))
    x, info = af.pcg_solve(_dev(af, ind), None, _vec([1.0, 1.0, 1.0]), raise_on_error=False)
    assert info.status == af.ERR_NOT_SPD


@pytest.mark.parametrize("opt,make", [("separate", lambda: synth.elasticity27(10)), ("fused", lambda: synth.elasticity27(10)),
                                      ("csr_a", lambda: synth.elasticity27(10)), ("separate", lambda: synth.poisson7(9)),
                                      ("fused", lambda: synth.poisson7(9)), ("csr_a", lambda: synth.poisson7(9))])
def test_pcg_forms_identical(af, opt, make):
    """Fused products and separate update kernels give the same iterates bit for bit; the CSR
    product for A agrees with the SELL-64 one to rounding (same iteration count).  The 9^3
    Poisson matrix has enough short boundary rows to get a split SELL layout for A."""
    Pb = make()
    dA = _dev(af, Pb.A)
    P = af.setup(dA, 10, 2, 1e-2)
    x1, i1 = af.pcg_solve(dA, P, _vec(Pb.b))
    o, v = {"separate": (af.OPT_PCG_FORM, 1), "fused": (af.OPT_PCG_FORM, 2), "csr_a": (af.OPT_PCG_CSR_A, 1)}[opt]
    try:
        af.set_option(o, v)
        x2, i2 = af.pcg_solve(dA, P, _vec(Pb.b))
    finally:
        af.set_option(o, 0)
    assert i1.iters == i2.iters
    if opt != "csr_a":
        assert bool((x1 == x2).all())
    else:
        assert float((x1 - x2).norm() / x1.norm()) < X_RTOL


@pytest.mark.parametrize("width", [1, 3, 8, 17])
@pytest.mark.parametrize("make", [lambda: synth.elasticity27(10), lambda: synth.random_sparse_spd(3000, 40, 3)])
def test_split_layouts_identical(af, make, width):
    """SELL layouts split at any width (the slices keep each row's last w entries, a sorted
    second layout the leading ones, multiplied first) give G^T(G r) and the PCG iterates bit
    for bit equal to the automatic layouts: each row is one sequential chain either way."""
    Pb = make()
    A = Pb.A if hasattr(Pb, "A") else Pb
    b = Pb.b if hasattr(Pb, "b") else A.to_scipy() @ synth.uniform(7, 2, A.n, -1.0, 1.0)
    dA = _dev(af, A)
    r = _vec(synth.uniform(5, 9, A.n))
    try:
        af.set_option(af.OPT_SELL_UNEVEN, 1)  # split layouts, automatic width
        P1 = af.setup(dA, 6, 2, 1e-2)
        z1 = P1.apply(r)
        x1, i1 = af.pcg_solve(dA, P1, _vec(b), maxit=2000)
        af.set_option(af.OPT_SELL_WIDTH, width)
        P2 = af.setup(dA, 6, 2, 1e-2)
        z2 = P2.apply(r)
        x2, i2 = af.pcg_solve(dA, P2, _vec(b), maxit=2000)
    finally:
        af.set_option(af.OPT_SELL_WIDTH, 0)
        af.set_option(af.OPT_SELL_UNEVEN, 0)
    assert bool((z1 == z2).all())
    assert i1.iters == i2.iters
    assert bool((x1 == x2).all())


@pytest.mark.parametrize("make", [lambda: synth.elasticity27(10), lambda: synth.random_sparse_spd(3000, 40, 3),
                                  lambda: synth.poisson7(9)])
def test_sorted_slices_against_split(af, make):
    """Uneven rows (G^T; A of small Poisson grids) ordered by length within windows of slices,
    every lane reading only its own row, against split layouts: G^T(G r) and A x bit for bit
    equal (each row is the same sequential chain), PCG iterates equal to rounding of the fused
    dots and both within the oracle's tolerance."""
    Pb = make()
    A = Pb.A if hasattr(Pb, "A") else Pb
    b = Pb.b if hasattr(Pb, "b") else A.to_scipy() @ synth.uniform(7, 2, A.n, -1.0, 1.0)
    dA = _dev(af, A)
    r = _vec(synth.uniform(5, 9, A.n))
    out = []
    try:
        for mode in (0, 1):
            af.set_option(af.OPT_SELL_UNEVEN, mode)
            P = af.setup(dA, 6, 2, 1e-2)
            z = P.apply(r)
            y = af.spmv(dA, r)
            x, i = af.pcg_solve(dA, P, _vec(b), maxit=2000)
            out.append((z, y, x, i))
    finally:
        af.set_option(af.OPT_SELL_UNEVEN, 0)
    (z0, y0, x0, i0), (z1, y1, x1, i1) = out
    assert bool((z0 == z1).all()) and bool((y0 == y1).all())
    assert abs(i0.iters - i1.iters) <= 1 and i0.converged and i1.converged
    assert float((x0 - x1).norm() / x1.norm()) < X_RTOL
    G = oracle.setup(A, 6, 2, 1e-2)
    ro = oracle.pcg(A, G, b, 1e-8, maxit=2000)
    assert float(np.linalg.norm(x0.cpu().numpy() - ro.x) / np.linalg.norm(ro.x)) < 10 * X_RTOL


@pytest.mark.parametrize("width", [0, 3, 8])
@pytest.mark.parametrize("make", [lambda: synth.elasticity27(10), lambda: synth.random_sparse_spd(3000, 40, 3)])
def test_split_tail_fused_identical(af, make, width):
    """The leading entries of split rows run inside the slices' product or in a launch of their
    own before it: G^T(G r) and the PCG iterates are bit for bit the same (width 0: the
    automatic split)."""
    Pb = make()
    A = Pb.A if hasattr(Pb, "A") else Pb
    b = Pb.b if hasattr(Pb, "b") else A.to_scipy() @ synth.uniform(7, 2, A.n, -1.0, 1.0)
    dA = _dev(af, A)
    r = _vec(synth.uniform(5, 9, A.n))
    try:
        af.set_option(af.OPT_SELL_WIDTH, width)
        P = af.setup(dA, 6, 2, 1e-2)
        out = []
        for tail in (0, 1):
            af.set_option(af.OPT_SELL_TAIL, tail)
            z = P.apply(r)
            x, i = af.pcg_solve(dA, P, _vec(b), maxit=2000)
            out.append((z, x, i.iters))
    finally:
        af.set_option(af.OPT_SELL_WIDTH, 0)
        af.set_option(af.OPT_SELL_TAIL, 0)
    (z0, x0, i0), (z1, x1, i1) = out
    assert bool((z0 == z1).all())
    assert i0 == i1
    assert bool((x0 == x1).all())


@pytest.mark.parametrize("make", [lambda: synth.elasticity27(8), lambda: synth.poisson7(9),
                                  lambda: synth.random_sparse_spd(3000, 40, 3)])
def test_spmm_against_oracle(af, make):
    """Y = A X for blocks of 1, 2, 4 and 8 right-hand sides (plain and length-ordered layouts,
    ragged last slices): every column within 1e-13 of the oracle's product and bit for bit the
    single-vector product of that column."""
    import torch

    Pb = make()
    A = Pb.A if hasattr(Pb, "A") else Pb
    dA = _dev(af, A)
    X8 = synth.uniform(13, 5, A.n * 8, -1.0, 1.0).reshape(A.n, 8)
    for k in (1, 2, 4, 8):
        Y = af.spmm(dA, torch.from_numpy(np.ascontiguousarray(X8[:, :k])).cuda()).cpu().numpy()
        for j in range(k):
            yo = oracle.spmv(A, X8[:, j])
            assert np.linalg.norm(Y[:, j] - yo) <= 1e-13 * np.linalg.norm(yo), (k, j)
            y1 = af.spmm(dA, torch.from_numpy(np.ascontiguousarray(X8[:, j:j + 1])).cuda()).cpu().numpy()
            assert np.array_equal(Y[:, j].view(np.int64), y1[:, 0].view(np.int64)), (k, j)
    with pytest.raises(af.AfsaiError):
        af.spmm(dA, torch.zeros((A.n, 3), dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("make", [lambda: synth.elasticity27(8), lambda: synth.random_sparse_spd(3000, 40, 3)])
def test_prepared_matrix_matches_unprepared(af, make):
    """A prepared once: its block products and its PCG solves (preconditioned and plain, two
    right-hand sides in a row) equal the unprepared calls bit for bit, with the same iteration
    counts; A's device arrays may be overwritten after preparing without changing them."""
    import torch

    Pb = make()
    A = Pb.A if hasattr(Pb, "A") else Pb
    dA = _dev(af, A)
    M = af.PreparedMatrix(dA)
    X8 = torch.from_numpy(synth.uniform(19, 5, A.n * 8, -1.0, 1.0).reshape(A.n, 8)).cuda()
    for k in (1, 4, 8):
        Xk = X8[:, :k].contiguous()
        assert torch.equal(M.spmm(Xk), af.spmm(dA, Xk)), k
    P = af.setup(dA, 6, 2, 1e-2)
    bs = [_vec(synth.uniform(23 + t, 5, A.n, -1.0, 1.0)) for t in range(2)]
    for Pc in (P, None):
        for b in bs:
            x0, i0 = af.pcg_solve(dA, Pc, b, rtol=1e-8, maxit=3000)
            x1, i1 = M.pcg_solve(Pc, b, rtol=1e-8, maxit=3000)
            assert i0.iters == i1.iters and i0.converged == i1.converged
            assert torch.equal(x0, x1)
    ref = af.spmm(dA, X8)
    x_ref, i_ref = M.pcg_solve(P, bs[0], rtol=1e-8, maxit=3000)
    dA.val.zero_()  # the prepared copy does not read A's arrays again
    assert torch.equal(M.spmm(X8), ref)
    x2, i2 = M.pcg_solve(P, bs[0], rtol=1e-8, maxit=3000)
    assert i2.iters == i_ref.iters and torch.equal(x2, x_ref)
    M.close()
    P.close()


@pytest.mark.parametrize("precond", [True, False])
@pytest.mark.parametrize("make", [lambda: synth.elasticity27(8), lambda: synth.random_sparse_spd(3000, 40, 3)])
def test_pcg_multi_against_oracle(af, make, precond):
    """PCG over blocks of 1, 2, 4 and 8 right-hand sides (one column zero, one a multiple of
    another): each column's true residual below the stopping bound, A (x - x_oracle) within
    the sum of the two residuals, the zero column x = 0 after 0 iterations; preconditioned,
    every column takes the oracle's iteration count and x is within 1e-10 of the oracle's
    (the bar of the single-vector solver); plain CG amplifies the rounding of the dots (the
    block sums each column's terms in a fixed tree order, the oracle in row order), so there
    its count is held within one.  A second solve of the block of eight gives the same
    iterates bit for bit."""
    import torch

    Pb = make()
    A = Pb.A if hasattr(Pb, "A") else Pb
    dA = _dev(af, A)
    P = af.setup(dA, 6, 2, 1e-2) if precond else None
    G = oracle.setup(A, 6, 2, 1e-2) if precond else None
    Xt = synth.uniform(17, 3, A.n * 8, -1.0, 1.0).reshape(A.n, 8)
    B8 = np.ascontiguousarray(np.column_stack([A.to_scipy() @ Xt[:, j] for j in range(8)]))
    B8[:, 3] = 0.0
    B8[:, 5] = 4.0 * B8[:, 1]
    for k in (1, 2, 4, 8):
        X, infos = af.pcg_solve_multi(dA, P, torch.from_numpy(np.ascontiguousarray(B8[:, :k])).cuda(),
                                      rtol=1e-8, maxit=3000)
        X = X.cpu().numpy()
        for j in range(k):
            if j == 3:
                assert infos[j].iters == 0 and infos[j].converged and not X[:, j].any()
                continue
            ro = oracle.pcg(A, G, B8[:, j], 1e-8, maxit=3000)
            assert infos[j].converged and abs(infos[j].iters - ro.iters) <= (0 if precond else 1), \
                (k, j, infos[j].iters, ro.iters)
            # both stop at ||b - A x|| <= 1e-8 ||b||, so ||A (x - x_o)|| is bounded by the sum of
            # the two true residuals (each measured with the oracle's product)
            nb = np.linalg.norm(B8[:, j])
            r_gpu = np.linalg.norm(B8[:, j] - oracle.spmv(A, X[:, j]))
            r_o = np.linalg.norm(B8[:, j] - oracle.spmv(A, ro.x))
            assert r_gpu <= 1.01e-8 * nb and abs(infos[j].true_relres - r_gpu / nb) <= 1e-12, (k, j)
            assert np.linalg.norm(oracle.spmv(A, X[:, j] - ro.x)) <= (r_gpu + r_o) * (1 + 1e-6), (k, j)
            if precond:
                assert np.linalg.norm(X[:, j] - ro.x) <= X_RTOL * np.linalg.norm(ro.x), (k, j)
        if k == 8:
            X2, i2 = af.pcg_solve_multi(dA, P, torch.from_numpy(np.ascontiguousarray(B8)).cuda(), rtol=1e-8,
                                        maxit=3000)
            assert [i.iters for i in i2] == [i.iters for i in infos]
            assert np.array_equal(X2.cpu().numpy().view(np.int64), X.view(np.int64))


def test_pcg_deterministic(af):
    Pb = synth.elasticity27(12)
    dA = _dev(af, Pb.A)
    P = af.setup(dA, 10, 2, 1e-2)
    x1, _ = af.pcg_solve(dA, P, _vec(Pb.b))
    x2, _ = af.pcg_solve(dA, P, _vec(Pb.b))
    assert bool((x1 == x2).all())


# --------------------------------------------------------------------------------------
# full size (64^3 nodes, 786,432 rows): the launch configuration of the benchmark
# --------------------------------------------------------------------------------------
def test_full_size_elasticity64(af):
    """Every launch at the full 64^3 size (786,432 rows): G row by row against the oracle's
    setup of all rows (patterns identical, values within 1e-10), then the GPU's PCG against the
    oracle's PCG on the oracle's G: the same iteration count and x within 1e-10."""
    Pb = synth.elasticity27(64)
    r = compare_factor(af, Pb.A, 10, 2, 1e-2)
    dA, P = r["dA"], r["P"]
    x, info = af.pcg_solve(dA, P, _vec(Pb.b), rtol=1e-8)
    assert info.converged and info.true_relres <= 1.1e-8
    ro = oracle.pcg(Pb.A, oracle.setup(Pb.A, 10, 2, 1e-2), Pb.b, 1e-8)
    assert info.iters == ro.iters, (info.iters, ro.iters)
    err = np.linalg.norm(x.cpu().numpy() - ro.x) / np.linalg.norm(ro.x)
    assert err <= X_RTOL, err


def test_full_size_elasticity150_sampled(af):
    """The largest configuration (150^3 nodes x 3 dof: 10,125,000 rows, 809,238,528 nonzeros,
    log-normal sigma = 2, k_max = 15, s = 3, patterns of up to 46 entries) with G stored in FP32:
    3,000 sampled rows against the oracle (pattern identical, values within FP32 rounding of
    the oracle's), and the solve by its true residual."""
    import time

    t0 = time.time()
    Pb = synth.elasticity27(150, 2.0, 5, kmax=15, s=3)
    rows = np.unique(np.concatenate([np.arange(0, 30), np.arange(Pb.n - 30, Pb.n),
                                     synth.raw_u64(150, 5, 2940).astype(np.int64) % Pb.n])).astype(np.int32)
    r = compare_factor(af, Pb.A, 15, 3, 1e-2, g_prec=1, rows=rows)
    dA, P = r["dA"], r["P"]
    x, info = af.pcg_solve(dA, P, _vec(Pb.b), rtol=1e-8)
    assert info.converged and info.true_relres <= 1.1e-8
    print(f"150^3 27-point: setup {r['info'].ms:.0f} ms, nnz(G) {r['info'].nnz_g}, PCG {info.iters} iterations "
          f"{info.ms:.0f} ms, test {time.time() - t0:.0f} s")
