"""Pins of the oracle's CG, power method, Chebyshev filters and Gram-Schmidt.

The references are independent of the oracle's recurrences: dense solves and
eigendecompositions, the closed form T_n(x) = cos(n arccos x) of the
Chebyshev smoothers section (continued with cosh outside [-1, 1]), the CG
convergence bound of the Spectrum section, the numbers printed in the
caption of the paper's Chebyshev filter figure, and numpy's QR.
"""

import os

import numpy as np
import pytest

import synth
from oracle import krylov, lattice as L

M5, MF = 1.8, 0.01
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def cheb_closed(n, x):
    """T_n(x) from its trigonometric definition, continued outside [-1, 1]."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1
    out[inside] = np.cos(n * np.arccos(x[inside]))
    hi = x > 1
    out[hi] = np.cosh(n * np.arccosh(x[hi]))
    lo = x < -1
    out[lo] = (-1.0) ** n * np.cosh(n * np.arccosh(-x[lo]))
    return out


@pytest.fixture(scope="module")
def dense_A():
    dims, Ls = (2, 2, 2, 2), 4
    U = synth.gauge_links(dims, eps=0.6, seed=12)
    shape = (Ls, 2, 2, 2, 2, 4, 3)
    even = L.parity_entry_mask(shape, L.EVEN)
    A = L.dense_matrix(lambda v: L.mpcdagmpc(U, v, M5, MF), shape, even)
    idx = np.flatnonzero(even.ravel())

    def apply(v):
        out = np.zeros(v.shape, dtype=np.complex128)  # C-contiguous, so reshape(-1) is a view
        out.reshape(-1)[idx] = A @ v.reshape(-1)[idx]
        return out

    w, V = np.linalg.eigh(A)
    return dict(U=U, dims=dims, Ls=Ls, shape=shape, even=even, idx=idx, A=A, apply=apply, w=w, V=V)


def test_cg_matches_dense_solve_and_bound(dense_A):
    d = dense_A
    b = L.on_parity(synth.gaussian_fermion(d["dims"], d["Ls"], seed=20), L.EVEN)
    tol = 1e-12
    res = krylov.cg(d["apply"], b, tol=tol, maxiter=5000)
    assert res.converged and res.true_rel_residual < 10 * tol
    x_dense = np.linalg.solve(d["A"], b.reshape(-1)[d["idx"]])
    err = np.linalg.norm(res.x.reshape(-1)[d["idx"]] - x_dense) / np.linalg.norm(x_dense)
    kappa = d["w"].max() / d["w"].min()
    assert err < kappa * tol
    # convergence bound of the Spectrum section, in the A-norm form:
    # iterations <= ln(2 sqrt(kappa)/tol) / -ln(sigma)
    sigma = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    assert res.iterations <= np.log(2 * np.sqrt(kappa) / tol) / -np.log(sigma) + 1
    assert res.iterations <= len(x_dense)


def test_cg_with_initial_guess(dense_A):
    d = dense_A
    b = L.on_parity(synth.gaussian_fermion(d["dims"], d["Ls"], seed=21), L.EVEN)
    full = krylov.cg(d["apply"], b, tol=1e-12)
    half = krylov.cg(d["apply"], b, tol=1e-4)
    resumed = krylov.cg(d["apply"], b, tol=1e-12, x0=half.x)
    assert resumed.converged and resumed.iterations < full.iterations
    assert resumed.true_rel_residual < 1e-11


def test_power_method(dense_A):
    d = dense_A
    v0 = L.on_parity(synth.gaussian_fermion(d["dims"], d["Ls"], seed=22), L.EVEN)
    lam, it = krylov.power_method(d["apply"], v0, iters=2000, rtol=1e-12)
    assert abs(lam - d["w"].max()) < 1e-6 * d["w"].max()


@pytest.mark.parametrize("order,lo,hi", [(0, 0.1, 60.0), (1, 0.1, 60.0), (16, 0.1, 60.0), (7, 0.5, 30.0)])
def test_chebyshev_filter_vs_eigendecomposition(dense_A, order, lo, hi):
    d = dense_A
    v = L.on_parity(synth.gaussian_fermion(d["dims"], d["Ls"], seed=23), L.EVEN)
    out, count = krylov.chebyshev_filter(d["apply"], v, order, lo, hi)
    assert count == order
    x = 2 * (d["w"] - lo) / (hi - lo) - 1
    c = d["V"].conj().T @ v.reshape(-1)[d["idx"]]
    expect = d["V"] @ (cheb_closed(order, x) * c)
    got = out.reshape(-1)[d["idx"]]
    assert np.linalg.norm(got - expect) < 1e-11 * np.linalg.norm(expect)


def test_chebyshev_series_vs_eigendecomposition(dense_A):
    d = dense_A
    eta = L.on_parity(synth.gaussian_fermion(d["dims"], d["Ls"], seed=24), L.EVEN)
    m, lam_lo, lam_max, delta, nvec = 20, 0.05, 30.0, 5, 4
    phis, count = krylov.chebyshev_series(d["apply"], eta, m, lam_lo, lam_max, delta, nvec)
    assert count == m + (nvec - 1) * delta
    c = d["V"].conj().T @ eta.reshape(-1)[d["idx"]]
    pre = cheb_closed(m, 2 * (d["w"] - lam_lo) / (lam_max - lam_lo) - 1)
    xs = 2 * d["w"] / lam_max - 1
    for k, phi in enumerate(phis):
        expect = d["V"] @ (cheb_closed(k * delta, xs) * pre * c)
        got = phi.reshape(-1)[d["idx"]]
        assert np.linalg.norm(got - expect) < 1e-10 * np.linalg.norm(expect)


def test_fig2_filter_numbers():
    """The caption's numbers: an order-500 low-pass over [0.02, 60] lifts the
    zero mode by ~1e8 relative to the passband, and 16 series vectors at
    Delta = 100 cost 1500 applications beyond the prefilter."""
    g = read_golden("fig2_chebyshev_filter.txt")
    lam = np.array([0.0])  # a 1x1 operator at eigenvalue 0
    apply0 = lambda v: lam * v
    amp, _ = krylov.chebyshev_filter(apply0, np.array([1.0]), int(g["m"]), g["lambda_lo"], g["lambda_max"])
    # |T_m| <= 1 on the passband, so the gain is the value at 0
    order_of_mag = np.log10(abs(amp[0]))
    assert abs(order_of_mag - np.log10(g["low_mode_enhancement"])) < 0.5
    closed = cheb_closed(int(g["m"]), np.array([2 * (0 - g["lambda_lo"]) / (g["lambda_max"] - g["lambda_lo"]) - 1]))
    assert abs(amp[0] - closed[0]) < 1e-9 * abs(closed[0])
    apply1 = lambda v: 7.0 * v
    _, count = krylov.chebyshev_series(
        apply1, np.array([1.0]), int(g["m"]), g["lambda_lo"], g["lambda_max"], int(g["delta"]), int(g["nvec"])
    )
    assert count - int(g["m"]) == int(g["further_multiplies"])


def test_gram_schmidt_vs_qr():
    rng = np.random.default_rng(25)
    vecs = [rng.standard_normal((5, 7, 3)) + 1j * rng.standard_normal((5, 7, 3)) for _ in range(9)]
    # make the set ill-conditioned so that one pass alone would lose orthogonality
    for k in range(1, 9):
        vecs[k] = vecs[k] + 1e3 * vecs[0]
    Q, R = krylov.gram_schmidt(vecs)
    Qm = np.stack([q.ravel() for q in Q], 1)
    Vm = np.stack([v.ravel() for v in vecs], 1)
    assert np.max(np.abs(Qm.conj().T @ Qm - np.eye(9))) < 1e-13
    assert np.max(np.abs(Qm @ R - Vm)) < 1e-12 * np.max(np.abs(Vm))
    assert np.all(np.abs(np.diag(R).imag) == 0) and np.all(np.diag(R).real > 0)
    q2, r2 = np.linalg.qr(Vm)
    ph = np.diag(r2) / np.abs(np.diag(r2))
    q2 = q2 * ph[None, :]
    r2 = r2 * ph.conj()[:, None]
    assert np.max(np.abs(q2 - Qm)) < 1e-9
    assert np.max(np.abs(r2 - R)) < 1e-9 * np.max(np.abs(R))


def test_rb_counting_golden(monkeypatch):
    """The counting rule the benchmark uses: one red-black CG iteration applies
    M_pc twice (4 half-lattice hops) and counts as 2 full matrix multiplies.  The
    paper's Krylov-table rows obey it; the oracle's CG on M_pc^dag M_pc makes exactly
    that many hopping applications per iteration (counted by wrapping the oracle's
    hop); and bench.py's site-update count is that many full matrix multiplies of
    V5 sites per iteration."""
    import bench

    g = read_golden("rb_counting.txt")
    assert g["rb_cgnr_form1_matmuls"] == g["full_matmuls_per_rb_iteration"] * g["rb_cgnr_form1_iterations"]
    assert g["rb_cgnr_form2_matmuls"] == g["full_matmuls_per_rb_iteration"] * g["rb_cgnr_form2_iterations"]
    assert g["half_dhop_per_rb_iteration"] == 2 * g["full_matmuls_per_rb_iteration"]
    # hops per oracle CG iteration
    dims, Ls = (2, 2, 2, 4), 4
    U = synth.gauge_links(dims, eps=0.3, seed=0)
    b = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=1), L.EVEN)
    calls = [0]
    real_dhop = L.dhop

    def counted(*args, **kwargs):
        calls[0] += 1
        return real_dhop(*args, **kwargs)

    monkeypatch.setattr(L, "dhop", counted)
    iters = 7
    res = krylov.cg(lambda v: L.mpcdagmpc(U, v, M5, MF), b, tol=1e-30, maxiter=iters)
    assert res.iterations == iters
    # one application per iteration plus the true residual at exit
    assert calls[0] == g["half_dhop_per_rb_iteration"] * (iters + 1)
    # the bench's count
    V5 = int(np.prod(dims)) * Ls
    assert bench.FULL_MATMULS_PER_RB_ITERATION == g["full_matmuls_per_rb_iteration"]
    assert bench.rb_site_updates(V5, g["rb_cgnr_form1_iterations"]) == g["rb_cgnr_form1_matmuls"] * V5


def test_smoother_coefficients_match_numpy_interpolation():
    """The coefficients are Chebyshev interpolation of 1/y at the first-kind nodes:
    numpy's chebinterpolate on the same N nodes gives c_0/2, c_1, ..., c_{N-1}, and c_N = 0."""
    a, b, N = 0.5, 60.0, 12
    c = krylov.chebyshev_smoother_coeffs(a, b, N)
    ref = np.polynomial.chebyshev.chebinterpolate(lambda x: 1.0 / (a + (b - a) * (x + 1) / 2), N - 1)
    assert np.allclose(c[0] / 2, ref[0], rtol=1e-13, atol=0)
    assert np.allclose(c[1:N], ref[1:], rtol=1e-10, atol=1e-15)
    assert abs(c[N]) < 1e-14 * abs(c[0])


def test_smoother_vs_eigendecomposition_and_inverse(dense_A):
    """S_cheb r = V p(Lambda) V^dag M^dag r with p the interpolant of 1/y, and on a
    spectrum inside [a, b] it approaches (M^dag M)^{-1} M^dag r = M^{-1} r as N grows."""
    d = dense_A
    U = d["U"]
    r = L.on_parity(synth.gaussian_fermion(d["dims"], d["Ls"], seed=26), L.EVEN)
    mdag = lambda v: L.mpc_dag(U, v, M5, MF)
    a, b = 0.9 * d["w"].min(), 1.1 * d["w"].max()
    N = 24
    got = krylov.chebyshev_smoother(d["apply"], mdag, r, a, b, N)
    c = krylov.chebyshev_smoother_coeffs(a, b, N)
    x = 2 * (d["w"] - a) / (b - a) - 1
    poly = 0.5 * c[0] + sum(c[j] * cheb_closed(j, x) for j in range(1, N + 1))
    wv = d["V"].conj().T @ mdag(r).reshape(-1)[d["idx"]]
    expect = d["V"] @ (poly * wv)
    assert np.linalg.norm(got.reshape(-1)[d["idx"]] - expect) < 1e-11 * np.linalg.norm(expect)
    # accuracy of the polynomial approximation to 1/y improves with N on [a, b]
    errs = []
    for N in (8, 32, 128):
        s = krylov.chebyshev_smoother(d["apply"], mdag, r, a, b, N)
        exact = d["V"] @ (wv / d["w"])
        errs.append(np.linalg.norm(s.reshape(-1)[d["idx"]] - exact) / np.linalg.norm(exact))
    assert errs[0] > errs[1] > errs[2]
