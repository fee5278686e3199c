"""GPU parity of the solver, filters and orthonormalisation against the oracle.

CG has many correct answers: the GPU solution must satisfy the residual
bound when the oracle measures it, and sit within kappa * tol of the oracle's
CG solution.  The Chebyshev filter, the series, Gram-Schmidt and the power
method with a fixed iteration count are unique up to rounding and are
compared directly.
"""

import numpy as np
import pytest

import synth
from oracle import krylov, lattice as L
from tests.gpu_util import M5, MF, dev_tensor, make_operator, pack, rel, rel_per_rhs, unpack

pytestmark = pytest.mark.gpu

F64, F32, F16S = 0, 1, 2
EVEN, ODD, BOTH = 0, 1, 2
C1 = ((4, 4, 4, 4), 8)


def even_fields(dims, Ls, n, seed):
    return np.stack([L.on_parity(f, EVEN) for f in synth.gaussian_fermion_batch(dims, Ls, n, seed)])


def oracle_A(U):
    return lambda v: L.mpcdagmpc(U, v, M5, MF)


@pytest.mark.parametrize("nrhs", [1, 2])
def test_cg_f64_c1(nrhs):
    dims, Ls = C1
    op, U = make_operator(dims, Ls, eps=0.3, seed=0)
    b = even_fields(dims, Ls, nrhs, seed=1)
    x = op.new_field(nrhs)
    code, iters, res = op.cg(pack(op, b, EVEN), x, nrhs, tol=1e-10, maxiter=5000)
    xg = unpack(op, x, nrhs, EVEN)
    A = oracle_A(U)
    for k in range(nrhs):
        true = np.linalg.norm((b[k] - A(xg[k])).ravel()) / np.linalg.norm(b[k].ravel())
        assert true < 1e-10 * 1.5
        assert abs(true - res[k]) < 1e-11
        ref = krylov.cg(A, b[k], tol=1e-10, maxiter=5000)
        assert rel(xg[k], ref.x) < 1e-6  # kappa(C1) ~ 1e3: both within kappa * tol of the solution
        assert abs(iters[k] - ref.iterations) <= 3


def test_cg_initial_guess_is_used():
    dims, Ls = C1
    op, U = make_operator(dims, Ls, seed=0)
    b = even_fields(dims, Ls, 1, seed=2)
    A = oracle_A(U)
    ref = krylov.cg(A, b[0], tol=1e-10)
    x = pack(op, ref.x[None], EVEN)
    code, iters, res = op.cg(pack(op, b, EVEN), x, 1, tol=1e-8)
    assert iters[0] == 0 and res[0] < 1e-8


def test_solve_rb_c1():
    dims, Ls = C1
    op, U = make_operator(dims, Ls, seed=0)
    eta = synth.gaussian_fermion(dims, Ls, seed=1)
    psi = op.new_field(1, both=True)
    iters, res = op.solve_rb(pack(op, eta[None], BOTH), psi, tol=1e-10)
    got = unpack(op, psi, 1, BOTH)[0]
    assert res < 1e-10 * 1.5
    # full-operator residual measured by the oracle
    r = np.linalg.norm((L.ddw(U, got, M5, MF) - eta).ravel()) / np.linalg.norm(eta.ravel())
    assert r < 1e-7
    # the oracle's own red-black solve
    b = L.mpc_dag(U, L.schur_source(U, eta, M5, MF), M5, MF)
    xe = krylov.cg(oracle_A(U), b, tol=1e-12).x
    ref = xe + L.reconstruct_odd(U, xe, eta, M5, MF)
    assert rel(got, ref) < 1e-6


@pytest.mark.parametrize("prec", [F32, F16S])
def test_mixed_precision_cg_reaches_fp64_residual(prec):
    dims, Ls = C1
    op, U = make_operator(dims, Ls, seed=0, prec=prec)
    b = even_fields(dims, Ls, 2, seed=3)
    x = op.new_field(2, prec=F64)
    b_dev = op.new_field(2, prec=F64)
    # b in FP64 packed layout: pack through an FP64 handle
    op64, _ = make_operator(dims, Ls, seed=0, prec=F64)
    b_dev = pack(op64, b, EVEN)
    code, iters, res = op.cg(b_dev, x, 2, tol=1e-10, maxiter=20000)
    xg = unpack(op64, x, 2, EVEN)
    A = oracle_A(U)
    for k in range(2):
        true = np.linalg.norm((b[k] - A(xg[k])).ravel()) / np.linalg.norm(b[k].ravel())
        assert true < 1.5e-10
        assert res[k] < 1.5e-10


def test_cg_status_codes():
    import paper_2103_05034_amd as dwf

    dims, Ls = C1
    op, U = make_operator(dims, Ls, seed=0)
    b = even_fields(dims, Ls, 1, seed=4)
    x = op.new_field(1)
    code, iters, res = op.cg(pack(op, b, EVEN), x, 1, tol=1e-12, maxiter=1, allow_noconv=True)
    assert code == dwf.DWF_ENOCONV and iters[0] == 1
    bad = b.copy()
    bad.reshape(-1)[5] = np.nan
    x = op.new_field(1)
    with pytest.raises(dwf.DWFError) as e:
        op.cg(pack(op, bad, EVEN), x, 1, tol=1e-10, maxiter=50)
    assert e.value.code == dwf.DWF_EBREAKDOWN
    zero = np.zeros_like(b)
    x = op.new_field(1)
    code, iters, res = op.cg(pack(op, zero, EVEN), x, 1, tol=1e-10)
    assert code == 0 and iters[0] == 0
    assert not unpack(op, x, 1, EVEN).any()


def test_power_method_fixed_iterations():
    dims, Ls = (2, 2, 2, 2), 4
    op, U = make_operator(dims, Ls, eps=0.6, seed=12)
    v0 = even_fields(dims, Ls, 1, seed=5)
    v = pack(op, v0, EVEN)
    lam, it = op.power(v, iters=40, rtol=0.0)
    ref, it_ref = krylov.power_method(oracle_A(U), v0[0], iters=40, rtol=0.0)
    assert it == 40
    assert abs(lam - ref) < 1e-12 * abs(ref)


@pytest.mark.parametrize("prec,tol", [(F64, 1e-11), (F32, 1e-5)])
def test_chebyshev_filter(prec, tol):
    dims, Ls = C1
    op, U = make_operator(dims, Ls, seed=0, prec=prec, max_nrhs=2)
    v = even_fields(dims, Ls, 3, seed=6)
    buf = pack(op, v, EVEN)
    src = unpack(op, buf, 3, EVEN)
    op.chebyshev_filter(buf, 3, order=16, lo=0.1, hi=60.0)  # 3 vectors, chunks of 2
    got = unpack(op, buf, 3, EVEN)
    exp = np.stack([krylov.chebyshev_filter(oracle_A(U), s, 16, 0.1, 60.0)[0] for s in src])
    assert rel_per_rhs(got, exp) < tol


def test_chebyshev_series():
    dims, Ls = (2, 2, 2, 2), 4
    op, U = make_operator(dims, Ls, eps=0.6, seed=12)
    eta = even_fields(dims, Ls, 1, seed=7)
    m, lo, lmax, delta, nvec = 20, 0.05, 30.0, 5, 4
    out = op.new_field(nvec)
    op.chebyshev_series(pack(op, eta, EVEN), out, m, lo, lmax, delta, nvec)
    got = unpack(op, out, nvec, EVEN)
    phis, _ = krylov.chebyshev_series(oracle_A(U), eta[0], m, lo, lmax, delta, nvec)
    for k in range(nvec):
        assert rel(got[k], phis[k]) < 1e-11


@pytest.mark.parametrize("prec,tol", [(F64, 1e-12), (F32, 2e-5)])
def test_gram_schmidt(prec, tol):
    dims, Ls = C1
    op, U = make_operator(dims, Ls, seed=0, prec=prec)
    n = 6
    v = even_fields(dims, Ls, n, seed=8)
    v[3] = v[3] + 30.0 * v[0]  # poorly conditioned set
    buf = pack(op, v, EVEN)
    src = unpack(op, buf, n, EVEN)
    R = op.gram_schmidt(buf, n)
    Q = unpack(op, buf, n, EVEN)
    Qo, Ro = krylov.gram_schmidt(list(src))
    for k in range(n):
        assert rel(Q[k], Qo[k]) < tol
    assert np.max(np.abs(R - Ro)) < tol * np.max(np.abs(Ro))
    G = np.array([[np.vdot(Q[i].ravel(), Q[j].ravel()) for j in range(n)] for i in range(n)])
    assert np.max(np.abs(G - np.eye(n))) < (1e-13 if prec == F64 else 1e-5)


@pytest.mark.parametrize("prec,tol,nrhs", [(F64, 1e-12, 1), (F64, 1e-12, 3), (F32, 1e-5, 2)])
def test_chebyshev_smoother(prec, tol, nrhs):
    """S_cheb([0.5, 60], 12) -- the smoother of the paper's two-level runs -- against the
    oracle's term-by-term evaluation (the library uses Clenshaw's recurrence)."""
    dims, Ls = C1
    op, U = make_operator(dims, Ls, seed=0, prec=prec, max_nrhs=2)
    r = even_fields(dims, Ls, nrhs, seed=27)
    src = pack(op, r, EVEN)
    vals = unpack(op, src, nrhs, EVEN)
    out = op.new_field(nrhs)
    op.chebyshev_smoother(src, out, 12, 0.5, 60.0, nrhs)
    got = unpack(op, out, nrhs, EVEN)
    mdag = lambda v: L.mpc_dag(U, v, M5, MF)
    exp = np.stack([krylov.chebyshev_smoother(oracle_A(U), mdag, v, 0.5, 60.0, 12) for v in vals])
    assert rel_per_rhs(got, exp) < tol


@pytest.mark.parametrize("prec", [F64, F16S])
def test_cg_progress_reports_and_stops(prec):
    import paper_2103_05034_amd as dwf

    dims, Ls = C1
    op, U = make_operator(dims, Ls, seed=0, prec=prec)
    op64 = op if prec == F64 else make_operator(dims, Ls, seed=0, prec=F64)[0]
    b = pack(op64, even_fields(dims, Ls, 1, seed=31), EVEN)
    seen = []
    op.set_progress(lambda it, rel: seen.append((it, rel[0])) and False, every=16)
    x = op.new_field(1, prec=F64)
    code, iters, res = op.cg(b, x, 1, tol=1e-10, maxiter=20000)
    assert code == 0 and res[0] < 1.5e-10
    assert len(seen) >= 2
    its = [s[0] for s in seen]
    assert all(b2 - b1 >= 16 for b1, b2 in zip(its, its[1:])) and its[-1] <= iters[0]
    assert seen[0][1] > 1e-10 and all(np.isfinite(r) for _, r in seen)
    # a nonzero return stops the solve with x holding the current iterate
    op.set_progress(lambda it, rel: it >= 40, every=8)
    x = op.new_field(1, prec=F64)
    code, iters, res = op.cg(b, x, 1, tol=1e-10, maxiter=20000, allow_noconv=True)
    assert code == dwf.DWF_ENOCONV and "progress" in dwf.last_error()
    assert 40 <= iters[0] <= 48 and 1e-10 < res[0] < 1.0
    op.set_progress(None)
    code, iters, res = op.cg(b, x, 1, tol=1e-10, maxiter=20000)  # resumes from the stopped iterate
    assert code == 0 and res[0] < 1.5e-10


@pytest.mark.parametrize("dims,Ls,prec,slack", [((16, 16, 16, 32), 16, F32, 1.3), ((8, 8, 8, 16), 12, F16S, 4.0)])
def test_mixed_cg_near_physical_mass(dims, Ls, prec, slack):
    """mf = 0.00078, links exp(0.15 iH): FP32 fields with FP64 reliable updates need about the FP64
    iteration count (re-orthogonalising p after each update keeps the recursion conjugate); FP16
    fields still converge on the smaller lattice.  Both reach the FP64 true residual."""
    mf = 0.00078
    U = synth.gauge_links(dims, eps=0.15, seed=0)
    op64, _ = make_operator(dims, Ls, prec=F64, mf=mf, U=U, max_nrhs=1, max_cg_rhs=1)
    b = op64.pack(__import__("torch").from_numpy(synth.gaussian_fermion_batch(dims, Ls, 1, 5)).cuda(), EVEN)
    x = op64.new_field(1)
    code, it64, res64 = op64.cg(b, x, 1, tol=1e-10, maxiter=5000)
    assert code == 0 and res64[0] < 1.5e-10
    op, _ = make_operator(dims, Ls, prec=prec, mf=mf, U=U, max_nrhs=1, max_cg_rhs=1)
    x = op.new_field(1, prec=F64)
    code, it, res = op.cg(b, x, 1, tol=1e-10, maxiter=int(slack * it64[0]) + 50)
    assert code == 0 and res[0] < 1.5e-10
    assert it[0] <= slack * it64[0]


def test_filter_warns_when_its_top_is_below_the_measured_lambda_max():
    """After dwf_power, a filter, series or smoother whose upper bound lies below the
    measured lambda_max still computes its result (the oracle's, for that bound) but
    returns DWF_WLAMBDA; a bound above it, or a changed operator, gives no warning."""
    import warnings

    import paper_2103_05034_amd as dwf

    dims, Ls = C1
    op, U = make_operator(dims, Ls, prec=F64, max_nrhs=2)
    v = pack(op, even_fields(dims, Ls, 1, seed=70), EVEN)
    lam, _ = op.power(v, iters=200, rtol=1e-10)
    A = lambda w: L.mpcdagmpc(U, w, M5, MF)  # noqa: E731
    x = even_fields(dims, Ls, 1, seed=71)
    low = 0.5 * lam
    buf = pack(op, x, EVEN)
    with pytest.warns(RuntimeWarning, match="below the measured lambda_max"):
        op.chebyshev_filter(buf, 1, 6, 0.1, low)
    want, _ = krylov.chebyshev_filter(A, x[0], 6, 0.1, low)
    assert rel(unpack(op, buf, 1, EVEN)[0], want) < 1e-12
    out = op.new_field(1)
    with pytest.warns(RuntimeWarning):
        op.chebyshev_smoother(pack(op, x, EVEN), out, 4, 0.1, low)
    code = op.lib.dwf_chebyshev_filter(op.h, 3, 0.1, low, dwf._ptr(pack(op, x, EVEN)), 1)
    assert code == dwf.DWF_WLAMBDA
    with warnings.catch_warnings():
        warnings.simplefilter("error")
        op.chebyshev_filter(pack(op, x, EVEN), 1, 3, 0.1, 1.01 * lam)
        op.update_links(dev_tensor(U))  # the operator may have changed: the estimate is dropped
        op.chebyshev_filter(pack(op, x, EVEN), 1, 3, 0.1, low)


@pytest.mark.parametrize("prec", [F64, F32, F16S])
def test_cg_independent_of_launch_shape(prec):
    """CG's reductions are sums per site (over s in order) added in site order, so the
    whole solve -- iteration counts and the solution, bit for bit -- is the same for
    every launch shape (sites per workgroup, pipeline depth, rhs per workgroup) and
    traversal order."""
    import torch

    dims, Ls = (8, 4, 4, 8), 6
    op, U = make_operator(dims, Ls, seed=0, prec=prec, max_nrhs=2, max_cg_rhs=2)
    op64, _ = make_operator(dims, Ls, seed=0, prec=F64)
    b_dev = pack(op64, even_fields(dims, Ls, 2, seed=7), EVEN)
    ref = None
    for order in (0, 1, 2, (1, 2, 2)):
        if isinstance(order, tuple):
            op.set_order_box(*order)
        else:
            op.set_order(order)
        for spb, depth, rpb in ((4, 2, 1), (8, 3, 1), (16, 3, 2), (42, 1, 1)):
            op.set_tile(spb, depth, rpb)
            x = op.new_field(2, prec=F64)
            code, iters, res = op.cg(b_dev, x, 2, tol=1e-10, maxiter=20000)
            torch.cuda.synchronize()
            assert code == 0 and max(res) < 1.5e-10
            if ref is None:
                ref = (iters, res, x.clone())
            else:
                assert iters == ref[0], (order, spb, depth, rpb)
                assert res == ref[1]
                assert torch.equal(x, ref[2]), (order, spb, depth, rpb)


@pytest.mark.parametrize("nrhs", [1, 2])
def test_cg_fixed_iteration_counts(nrhs):
    """CG stopped after 1..9 iterations (the FP64 solver adds its search
    directions to x four iterations at a time, so these counts end with every
    number of directions still pending) against the oracle's CG run for the
    same number of iterations: the iterates are unique up to rounding."""
    dims, Ls = C1
    op, U = make_operator(dims, Ls, eps=0.3, seed=0)
    b = even_fields(dims, Ls, nrhs, seed=7)
    A = oracle_A(U)
    b_dev = pack(op, b, EVEN)
    for k in range(1, 10):
        x = op.new_field(nrhs)
        code, iters, res = op.cg(b_dev, x, nrhs, tol=1e-14, maxiter=k, allow_noconv=True)
        xg = unpack(op, x, nrhs, EVEN)
        for j in range(nrhs):
            ref = krylov.cg(A, b[j], tol=1e-14, maxiter=k)
            assert iters[j] == k == ref.iterations
            assert rel(xg[j], ref.x) < 1e-12, (k, j)
            assert abs(res[j] - ref.true_rel_residual) < 1e-12 * max(1.0, ref.true_rel_residual), (k, j)


@pytest.mark.parametrize("prec,tol", [(F64, 1e-12), (F32, 2e-5), (F16S, 3e-3)])
@pytest.mark.parametrize("n", [1, 17, 40, 64, 65])
def test_gram_schmidt_set_sizes(prec, tol, n):
    """Sets of up to 64 vectors go through Cholesky QR twice, larger sets through
    CGS2: both against the oracle's CGS2 of the stored inputs (Q R with a positive
    real diagonal is unique), on a set with a spread of norms and two near-parallel
    pairs.  FP16 + scale: the output is rounded to FP16 (2^-11 relative per value);
    CGS2 also stores every intermediate direction in FP16, and the 40x near-parallel
    pair amplifies that rounding, hence its looser bound."""
    if prec == F16S and n > 64:
        tol = 3e-2
    dims, Ls = C1
    op, U = make_operator(dims, Ls, seed=0, prec=prec)
    v = even_fields(dims, Ls, n, seed=20 + n)
    v *= np.exp(np.linspace(-3.0, 3.0, n))[:, None, None, None, None, None, None, None]
    if n > 3:
        v[2] = v[2] + 40.0 * v[1]
        v[n - 1] = v[n - 1] + 25.0 * v[0] * np.exp(3.0 - (-3.0))
    buf = pack(op, v, EVEN)
    src = unpack(op, buf, n, EVEN)
    R = op.gram_schmidt(buf, n)
    Q = unpack(op, buf, n, EVEN)
    Qo, Ro = krylov.gram_schmidt(list(src))
    for k in range(n):
        assert rel(Q[k], Qo[k]) < tol, k
    assert np.max(np.abs(R - Ro)) < tol * np.max(np.abs(Ro))
    assert np.all(np.abs(np.diag(R).imag) == 0) and np.all(np.diag(R).real > 0)
    G = np.array([[np.vdot(Q[i].ravel(), Q[j].ravel()) for j in range(n)] for i in range(n)])
    assert np.max(np.abs(G - np.eye(n))) < {F64: 1e-13, F32: 1e-5, F16S: 5e-3}[prec]


def test_gram_schmidt_nearly_dependent_set_falls_back():
    """A set too ill-conditioned for Cholesky QR (condition number ~1e9) is left to
    CGS2, which still returns an orthonormal Q with Q R = V."""
    dims, Ls = C1
    op, U = make_operator(dims, Ls, seed=0, prec=F64)
    n = 8
    v = even_fields(dims, Ls, n, seed=40)
    v[5] = v[2] + 1e-9 * v[5]
    buf = pack(op, v, EVEN)
    src = unpack(op, buf, n, EVEN)
    R = op.gram_schmidt(buf, n)
    Q = unpack(op, buf, n, EVEN)
    G = np.array([[np.vdot(Q[i].ravel(), Q[j].ravel()) for j in range(n)] for i in range(n)])
    assert np.max(np.abs(G - np.eye(n))) < 1e-12
    V = np.stack([s.ravel() for s in src], axis=1)
    QR = np.stack([q.ravel() for q in Q], axis=1) @ R
    assert np.linalg.norm(QR - V) < 1e-12 * np.linalg.norm(V)
    assert np.all(np.diag(R).real > 0)
