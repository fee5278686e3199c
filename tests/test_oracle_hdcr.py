"""Pins of the HDCR oracle against facts that do not come from the oracle itself:

* the little Dirac operator is nearest neighbour in the block grid (well separated
  blocks do not couple) and Hermitian (H_DW is);
* the squared-coarse-operator identity of the Spectrum section for a Gamma_5-compatible
  (chirally split) basis, built independently from D_DW and D_DW^dag;
* the V(1,1) sequence equals the closed form S (1 - MQ) + Q + (1 - QM) S + S (MQM - M) S
  of the Composite V(1,1) section (its first form; in the rewriting with P_L = 1 - MQ
  and P_R = 1 - QM the last term is -S P_L M S), and P_L M P = 0;
* with a basis spanning a whole block the cycle is the exact inverse;
* the smoother on H_DW is the interpolating polynomial of 1/y evaluated in the
  eigenbasis of the dense H_DW (numpy's eigh and chebval);
* GCR without a preconditioner minimises the residual over the Krylov space
  (least squares over an explicit Krylov basis), GCR with the exact inverse as
  preconditioner ends in one step, and HDCR solves D_DW psi = eta.
"""

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

import synth
from oracle import coarse as C
from oracle import hdcr as H
from oracle import krylov
from oracle import lattice as L

M5, MF = 1.8, 0.01


def chiral_basis(dims, Ls, block, nraw, seed):
    raw = list(synth.gaussian_fermion_batch(dims, Ls, nraw, seed))
    split = []
    for v in raw:
        split.extend(C.chiral_split(v))
    Q, _ = C.block_orthonormalize(split, dims, block)
    return Q


def block_coords(dims, block):
    X, Y, Z, T = dims
    n = [X // block[0], Y // block[1], Z // block[2], T // block[3]]
    nb = int(np.prod(n))
    coords = []
    for b in range(nb):
        bx = b % n[0]
        by = (b // n[0]) % n[1]
        bz = (b // (n[0] * n[1])) % n[2]
        bt = b // (n[0] * n[1] * n[2])
        coords.append((bx, by, bz, bt))
    return coords, n


def test_coarse_operator_nearest_neighbour_and_hermitian():
    dims, Ls, block = (4, 2, 2, 8), 2, (2, 2, 2, 2)  # block grid 2 x 1 x 1 x 4
    U = synth.gauge_links(dims, 0.3, seed=1)
    basis = chiral_basis(dims, Ls, block, 2, seed=2)
    n = len(basis)
    A = H.coarse_operator(lambda v: L.hdw(U, v, M5, MF), basis, dims, block)
    assert np.max(np.abs(A - A.conj().T)) < 1e-13 * np.max(np.abs(A))
    coords, ng = block_coords(dims, block)
    for a, ca in enumerate(coords):
        for b, cb in enumerate(coords):
            dist = []
            for mu in range(4):
                d = (cb[mu] - ca[mu]) % ng[mu]
                dist.append(min(d, ng[mu] - d))
            blk = A[a * n : (a + 1) * n, b * n : (b + 1) * n]
            if sum(dist) <= 1:
                assert np.max(np.abs(blk)) > 1e-3
            else:
                assert np.max(np.abs(blk)) == 0.0  # blocks two apart in t never couple


def test_squared_coarse_operator_identity():
    """P^dag Gamma5 D P P^dag Gamma5 D P = P^dag D^dag P P^dag D P for a chirally split basis."""
    dims, Ls, block = (4, 2, 2, 4), 4, (2, 2, 2, 2)
    U = synth.gauge_links(dims, 0.3, seed=3)
    basis = chiral_basis(dims, Ls, block, 2, seed=4)
    A = H.coarse_operator(lambda v: L.hdw(U, v, M5, MF), basis, dims, block)
    Dc = H.coarse_operator(lambda v: L.ddw(U, v, M5, MF), basis, dims, block)
    Ddc = H.coarse_operator(lambda v: L.ddw(U, v, M5, MF, dag=True), basis, dims, block)
    lhs, rhs = A @ A, Ddc @ Dc
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(lhs))
    # a basis that is not chirally split breaks it
    raw = list(synth.gaussian_fermion_batch(dims, Ls, 4, 5))
    Qr, _ = C.block_orthonormalize(raw, dims, block)
    A2 = H.coarse_operator(lambda v: L.hdw(U, v, M5, MF), Qr, dims, block)
    Dc2 = H.coarse_operator(lambda v: L.ddw(U, v, M5, MF), Qr, dims, block)
    Ddc2 = H.coarse_operator(lambda v: L.ddw(U, v, M5, MF, dag=True), Qr, dims, block)
    assert np.max(np.abs(A2 @ A2 - Ddc2 @ Dc2)) > 1e-3 * np.max(np.abs(A2 @ A2))


@pytest.fixture(scope="module")
def level():
    dims, Ls, block = (4, 2, 2, 4), 4, (2, 2, 2, 2)
    U = synth.gauge_links(dims, 0.3, seed=6)
    basis = chiral_basis(dims, Ls, block, 3, seed=7)
    A = H.coarse_operator(lambda v: L.hdw(U, v, M5, MF), basis, dims, block)
    return H.Level(U, M5, MF, basis, A, dims, block, lo=0.5, hi=40.0, order=6, coarse_tol=None)


def test_vcycle_closed_form(level):
    lv = level
    r0 = synth.gaussian_fermion(lv.dims, 4, seed=8)
    M, S, Q = lv.M, lv.S, lv.Q
    PL = lambda v: v - M(Q(v))  # noqa: E731
    PR = lambda v: v - Q(M(v))  # noqa: E731
    closed = S(PL(r0)) + Q(r0) + PR(S(r0)) + S(M(Q(M(S(r0)))) - M(S(r0)))
    got = H.vcycle(lv, r0)
    assert np.max(np.abs(got - closed)) < 1e-11 * np.max(np.abs(closed))
    # the same terms with +S P_L M S (the sign of the rewritten form) do not match
    wrong = S(PL(r0)) + Q(r0) + PR(S(r0)) + S(PL(M(S(r0))))
    assert np.max(np.abs(got - wrong)) > 1e-3 * np.max(np.abs(closed))


def test_left_projector_annihilates_the_subspace(level):
    lv = level
    c = np.random.default_rng(9).standard_normal(lv.A.shape[0]) + 0j
    Pc = H.prolong(lv.basis, c, lv.dims, lv.block)
    out = lv.M(Pc) - lv.M(lv.Q(lv.M(Pc)))  # P_L M P c
    assert np.max(np.abs(out)) < 1e-11 * np.max(np.abs(lv.M(Pc)))


def test_vcycle_exact_with_a_complete_basis():
    """One block holding the whole lattice and every unit vector: Q = M^{-1}, so
    r1 is removed exactly and the post-smoother acts on a zero residual."""
    dims, Ls, block = (2, 2, 2, 2), 2, (2, 2, 2, 2)
    U = synth.gauge_links(dims, 0.3, seed=10)
    shape = (Ls,) + tuple(reversed(dims)) + (4, 3)
    basis = []
    for i in range(int(np.prod(shape))):
        e = np.zeros(int(np.prod(shape)), dtype=np.complex128)
        e[i] = 1.0
        basis.append(e.reshape(shape))
    A = H.coarse_operator(lambda v: L.hdw(U, v, M5, MF), basis, dims, block)
    lv = H.Level(U, M5, MF, basis, A, dims, block, lo=0.5, hi=40.0, order=4, coarse_tol=None)
    r0 = synth.gaussian_fermion(dims, Ls, seed=11)
    x = H.vcycle(lv, r0)
    assert np.max(np.abs(lv.M(x) - r0)) < 1e-11 * np.max(np.abs(r0))


def test_smoother_on_hdw_in_its_eigenbasis():
    dims, Ls = (2, 2, 2, 4), 2
    U = synth.gauge_links(dims, 0.3, seed=12)
    shape = (Ls,) + tuple(reversed(dims)) + (4, 3)
    Hd = L.dense_matrix(lambda v: L.hdw(U, v, M5, MF), shape)
    assert np.max(np.abs(Hd - Hd.conj().T)) < 1e-13
    lam, V = np.linalg.eigh(Hd)
    lo, hi, N = 0.3, 30.0, 7
    c = krylov.chebyshev_smoother_coeffs(lo, hi, N).copy()
    c[0] *= 0.5
    p = npcheb.chebval((2 * lam**2 - (hi + lo)) / (hi - lo), c)
    r = synth.gaussian_fermion(dims, Ls, seed=13)
    want = V @ (p * lam * (V.conj().T @ r.ravel()))
    got = H.smoother(U, r, M5, MF, lo, hi, N).ravel()
    assert np.max(np.abs(got - want)) < 1e-11 * np.max(np.abs(want))


def test_gcr_minimises_the_residual_over_the_krylov_space():
    dims, Ls = (2, 2, 2, 4), 2
    U = synth.gauge_links(dims, 0.3, seed=14)
    M = lambda v: L.hdw(U, v, M5, MF)  # noqa: E731
    b = synth.gaussian_fermion(dims, Ls, seed=15)
    res = H.gcr(M, lambda r: r, b, tol=1e-30, maxiter=6, nkrylov=10)
    # residual of the least-squares problem over span{M b, M^2 b, ...}
    K, v = [], b.ravel()
    for k in range(1, 7):
        v = M(v.reshape(b.shape)).ravel()
        K.append(v / np.linalg.norm(v))
        Qk, _ = np.linalg.qr(np.stack(K, axis=1))
        best = np.linalg.norm(b.ravel() - Qk @ (Qk.conj().T @ b.ravel())) / np.linalg.norm(b.ravel())
        assert abs(res.history[k] - best) < 1e-10
    assert res.history[6] < res.history[1]


def test_gcr_with_the_exact_inverse_needs_one_step_and_restarts_are_exact():
    dims, Ls = (2, 2, 2, 4), 2
    U = synth.gauge_links(dims, 0.3, seed=16)
    shape = (Ls,) + tuple(reversed(dims)) + (4, 3)
    Hd = L.dense_matrix(lambda v: L.hdw(U, v, M5, MF), shape)
    M = lambda v: (Hd @ v.ravel()).reshape(shape)  # noqa: E731
    inv = lambda r: np.linalg.solve(Hd, r.ravel()).reshape(shape)  # noqa: E731
    b = synth.gaussian_fermion(dims, Ls, seed=17)
    res = H.gcr(M, inv, b, tol=1e-12)
    assert res.iterations == 1 and res.true_rel_residual < 1e-12
    # restarted every 3 directions on the positive definite H^2 (restarted GCR can
    # stall on an indefinite matrix): still converges to the dense solution
    H2 = Hd @ Hd
    M2 = lambda v: (H2 @ v.ravel()).reshape(shape)  # noqa: E731
    res = H.gcr(M2, lambda r: r, b, tol=1e-10, maxiter=20000, nkrylov=3)
    assert res.converged and res.true_rel_residual < 2e-10
    want = np.linalg.solve(H2, b.ravel())
    assert np.max(np.abs(res.x.ravel() - want)) < 1e-6 * np.max(np.abs(want))


def filtered_chiral_basis(U, dims, Ls, block, nraw, order, lo, hi, seed):
    """The setup of Algorithms A / B in miniature: Gaussian vectors low-pass
    filtered with T_order of D_DW^dag D_DW over [lo, hi], split by chirality and
    orthonormalised in every block."""
    A2 = lambda v: H.hdw_normal(U, v, M5, MF)  # noqa: E731
    split = []
    for g in synth.gaussian_fermion_batch(dims, Ls, nraw, seed):
        v, _ = krylov.chebyshev_filter(A2, g, order, lo, hi)
        split.extend(C.chiral_split(v / np.linalg.norm(v)))
    Q, _ = C.block_orthonormalize(split, dims, block)
    return Q


def test_hdcr_solves_ddw():
    """4^4, Ls = 4: H^2 has 12 light modes below 0.01 and a band from 0.16, so the
    setup keeps 12 filtered vectors (24 after the split) and the smoother covers
    [0.15, 70] (lambda_max = 56.5)."""
    dims, Ls, block = (4, 4, 4, 4), 4, (2, 2, 2, 2)
    U = synth.gauge_links(dims, 0.3, seed=18)
    basis = filtered_chiral_basis(U, dims, Ls, block, 12, 100, 0.15, 70.0, seed=19)
    A = H.coarse_operator(lambda v: L.hdw(U, v, M5, MF), basis, dims, block)
    lv = H.Level(U, M5, MF, basis, A, dims, block, lo=0.15, hi=70.0, order=12, coarse_tol=0.02)
    eta = synth.gaussian_fermion(dims, Ls, seed=20)
    res = H.hdcr_solve(lv, eta, tol=1e-10, maxiter=60, nkrylov=8)
    assert res.converged and res.iterations <= 30
    psi = res.x
    assert np.linalg.norm((L.ddw(U, psi, M5, MF) - eta).ravel()) / np.linalg.norm(eta.ravel()) < 2e-10
    # GCR without the preconditioner is still far from converged after many more steps
    plain = H.gcr(lv.M, lambda r: r, L.Gamma5(eta), tol=1e-10, maxiter=200, nkrylov=8)
    assert not plain.converged and plain.history[-1] > 1e-3


def test_coarse_solve_is_cgnr():
    rng = np.random.default_rng(21)
    n = 40
    B = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = B + B.conj().T + 0.5 * np.eye(n)  # Hermitian indefinite
    d = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    res = H.coarse_solve(A, d, tol=1e-12)
    assert np.linalg.norm(A @ res.x - d) / np.linalg.norm(d) < 1e-8
    loose = H.coarse_solve(A, d, tol=0.02)
    Ah = A.conj().T
    assert np.linalg.norm(Ah @ (d - A @ loose.x)) <= 0.02 * np.linalg.norm(Ah @ d) * (1 + 1e-12)
    assert loose.iterations < res.iterations
