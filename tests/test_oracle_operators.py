"""Pins of the oracle's operators against facts the paper and the algebra fix.

Each test checks the oracle against something other than itself: the gamma
algebra, the free-field plane-wave symbol of D_W, the paper's free 5D
Wilson spectrum (Spectrum of domain wall fermions section), the Ls = 1
reduction to Wilson, Gamma5-hermiticity (Chiral Fermion Actions section),
gauge covariance, the closed-form inverse of the fifth-dimension matrix,
and the Schur determinant / solve identities of the red-black form.
"""

import numpy as np
import pytest

import synth
from oracle import lattice as L

M5, MF = 1.8, 0.01


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


# ----------------------------------------------------------------------------- gamma
def test_gamma_algebra():
    for mu in range(4):
        g = L.GAMMA[mu]
        assert np.allclose(g, g.conj().T)
        for nu in range(4):
            anti = g @ L.GAMMA[nu] + L.GAMMA[nu] @ g
            assert np.allclose(anti, 2.0 * (mu == nu) * np.eye(4))
        assert np.allclose(g @ L.GAMMA5 + L.GAMMA5 @ g, 0)
    assert np.allclose(L.GAMMA5, np.diag([1, 1, -1, -1]))
    assert np.allclose(L.P_PLUS + L.P_MINUS, np.eye(4))
    assert np.allclose(L.P_PLUS @ L.P_MINUS, 0)


def test_synthetic_links_are_su3():
    U = synth.gauge_links((4, 4, 4, 4), eps=0.3, seed=0)
    u = U.reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.max(np.abs(u.conj().transpose(0, 2, 1) @ u - eye)) < 1e-13
    assert np.max(np.abs(np.linalg.det(u) - 1)) < 1e-13


# ------------------------------------------------------------------------ Wilson D_W
def test_wilson_free_plane_wave_symbol():
    """U = 1: D_W(M) e^{ipx} u = [M + sum(1 - cos p) + i sum gamma_mu sin p_mu] e^{ipx} u."""
    dims = (4, 6, 2, 8)
    X, Y, Z, T = dims
    U = synth.unit_links(dims)
    rng = np.random.default_rng(3)
    n = (1, 5, 1, 3)  # momentum integers in x, y, z, t
    p = [2 * np.pi * n[0] / X, 2 * np.pi * n[1] / Y, 2 * np.pi * n[2] / Z, 2 * np.pi * n[3] / T]
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = phase[..., None, None] * u
    M = -0.7
    symbol = (M + sum(1 - np.cos(q) for q in p)) * np.eye(4) + 1j * sum(
        L.GAMMA[mu] * np.sin(p[mu]) for mu in range(4)
    )
    expect = phase[..., None, None] * (symbol @ u)
    assert rel(L.wilson(U, psi, M), expect) < 1e-14


def test_dhop_adjoint_and_gamma5_hermiticity():
    dims = (4, 2, 6, 4)
    U = synth.gauge_links(dims, eps=0.7, seed=1)
    chi = synth.gaussian_fermion(dims, 3, seed=2)
    psi = synth.gaussian_fermion(dims, 3, seed=3)
    # the dagger flag is the adjoint: <chi, D psi> = <D^dag chi, psi>
    lhs = L.inner(chi, L.dhop(U, psi))
    rhs = L.inner(L.dhop(U, chi, dag=True), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # gamma5-hermiticity: g5 D_hop g5 = D_hop^dag
    assert rel(L.gamma5(L.dhop(U, L.gamma5(psi))), L.dhop(U, psi, dag=True)) < 1e-14


def test_gauge_covariance_of_ddw():
    """U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag, psi -> g psi  =>  D[U^g] psi^g = (D[U] psi)^g."""
    dims = (4, 4, 2, 6)
    U = synth.gauge_links(dims, eps=0.5, seed=4)
    g = synth.gauge_transform(dims, seed=5)
    psi = synth.gaussian_fermion(dims, 4, seed=6)
    Ug = np.empty_like(U)
    for mu in range(4):
        g_fwd = L.shift(g, mu, +1)  # g(x + mu)
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ L.dagger(g_fwd)
    gpsi = lambda f: f @ np.swapaxes(g, -1, -2)  # colour rotation per site
    lhs = L.ddw(Ug, gpsi(psi), M5, MF)
    rhs = gpsi(L.ddw(U, psi, M5, MF))
    assert rel(lhs, rhs) < 1e-14


# ------------------------------------------------------------------------- D_DW
def test_ddw_Ls1_is_wilson():
    """At Ls = 1 both corner terms land on the diagonal: D_DW = D_W(1 + m - M5)."""
    dims = (4, 4, 2, 2)
    U = synth.gauge_links(dims, eps=0.4, seed=7)
    psi = synth.gaussian_fermion(dims, 1, seed=8)
    expect = L.wilson(U, psi[0], 1.0 + MF - M5)[None]
    assert rel(L.ddw(U, psi, M5, MF), expect) < 1e-14


def test_ddw_gamma5_hermiticity():
    """Gamma_5 D_DW Gamma_5 = D_DW^dag, checked through inner products."""
    dims = (2, 4, 4, 2)
    U = synth.gauge_links(dims, eps=0.8, seed=9)
    chi = synth.gaussian_fermion(dims, 5, seed=10)
    psi = synth.gaussian_fermion(dims, 5, seed=11)
    a = L.inner(chi, L.hdw(U, psi, M5, MF))
    b = L.inner(L.hdw(U, chi, M5, MF), psi)
    assert abs(a - b) < 1e-13 * abs(a)
    # and the dag flag of ddw is the adjoint
    a = L.inner(chi, L.ddw(U, psi, M5, MF))
    b = L.inner(L.ddw(U, chi, M5, MF, dag=True), psi)
    assert abs(a - b) < 1e-13 * abs(a)


@pytest.mark.parametrize("mf,antiperiodic", [(-1.0, False), (1.0, True)])
def test_free_5d_wilson_spectrum(mf, antiperiodic):
    """mf = -1 (+1): D_DW is the periodic (antiperiodic) free 5D Wilson operator at
    mass -M5, whose eigenvalues are Re = -M5 + 5 - sum cos p, |Im|^2 = sum sin^2 p
    over the five momenta (the paper's free-field formula)."""
    dims = (3, 3, 2, 2)
    Ls = 2
    X, Y, Z, T = dims
    U = synth.unit_links(dims)
    shape = (Ls, T, Z, Y, X, 4, 3)
    D = L.dense_matrix(lambda v: L.ddw(U, v, M5, mf), shape)
    ev = np.linalg.eigvals(D)
    expect = []
    for nx in range(X):
        for ny in range(Y):
            for nz in range(Z):
                for nt in range(T):
                    for k in range(Ls):
                        p5 = 2 * np.pi * (k + (0.5 if antiperiodic else 0.0)) / Ls
                        ps = [2 * np.pi * nx / X, 2 * np.pi * ny / Y, 2 * np.pi * nz / Z, 2 * np.pi * nt / T, p5]
                        re = -M5 + 5 - sum(np.cos(q) for q in ps)
                        im = np.sqrt(sum(np.sin(q) ** 2 for q in ps))
                        expect += [re + 1j * im] * 6 + [re - 1j * im] * 6
    expect = np.array(expect)
    key = lambda z: np.lexsort((np.round(z.imag, 9), np.round(z.real, 9)))
    assert len(ev) == len(expect)
    assert np.max(np.abs(ev[key(ev)] - expect[key(expect)])) < 1e-10


def test_zero_momentum_domain_wall_roots():
    """Free field, p = 0: D_par = 1 - M5 and the P_+ block is (1 - M5) - S with the
    cyclic shift S^Ls = -m, so its eigenvalues are (1 - M5) - z, z^Ls = -m."""
    Ls, mf = 5, 0.03
    U = synth.unit_links((1, 1, 1, 1))  # one site: every hop returns to it, p = 0
    shape = (Ls, 1, 1, 1, 1, 4, 3)
    D = L.dense_matrix(lambda v: L.ddw(U, v, M5, mf), shape)
    ev = np.linalg.eigvals(D)
    roots = (mf ** (1.0 / Ls)) * np.exp(1j * np.pi * (2 * np.arange(Ls) + 1) / Ls)
    expect = np.repeat((1 - M5) - roots, 12)  # 2 spins x 3 colours x 2 chiralities
    key = lambda z: np.lexsort((np.round(z.imag, 9), np.round(z.real, 9)))
    assert np.max(np.abs(ev[key(ev)] - expect[key(expect)])) < 1e-12


def test_m5d_inverse_closed_form():
    """Per chirality, (d - S)^{-1} = sum_{k<Ls} d^{-k} S^k / (d (1 + m d^{-Ls})), d = 5 - M5,
    with S the cyclic shift (lower for P_+, upper for P_-) carrying -m on the wrap."""
    for Ls, mf in [(1, 0.01), (2, 0.5), (8, 0.01), (16, 0.00078), (5, -1.0 + 1e-3)]:
        d = 5 - M5
        K = L.m5d_matrix(Ls, M5, mf).reshape(Ls, 4, Ls, 4)
        Kinv = np.linalg.inv(L.m5d_matrix(Ls, M5, mf)).reshape(Ls, 4, Ls, 4)
        S_low = np.zeros((Ls, Ls))
        for s in range(1, Ls):
            S_low[s, s - 1] = 1.0
        S_low[0, Ls - 1] = -mf
        closed = sum(np.linalg.matrix_power(S_low, k) / d**k for k in range(Ls))
        closed /= d * (1 + mf * d ** (-Ls))
        assert np.max(np.abs(Kinv[:, 0, :, 0] - closed)) < 1e-14
        assert np.max(np.abs(Kinv[:, 2, :, 2] - closed.T)) < 1e-14
        assert np.max(np.abs(Kinv[:, 0, :, 2])) == 0
        # the forward matrix itself: P_+ block = d - S_low
        assert np.max(np.abs(K[:, 0, :, 0] - (d * np.eye(Ls) - S_low))) < 1e-15


# ------------------------------------------------------------- Schur / red-black
@pytest.fixture(scope="module")
def small():
    dims = (2, 2, 2, 2)
    Ls = 4
    U = synth.gauge_links(dims, eps=0.6, seed=12)
    shape = (Ls, 2, 2, 2, 2, 4, 3)
    return dims, Ls, U, shape


def test_schur_determinant(small):
    """det D_DW = det M_oo * det M_pc on a 2^4 x 4 lattice (dims 768 and 384)."""
    dims, Ls, U, shape = small
    D = L.dense_matrix(lambda v: L.ddw(U, v, M5, MF), shape)
    even = L.parity_entry_mask(shape, L.EVEN)
    Mpc = L.dense_matrix(lambda v: L.mpc(U, v, M5, MF), shape, even)
    K = L.m5d_matrix(Ls, M5, MF)
    s_D, ld_D = np.linalg.slogdet(D)
    s_P, ld_P = np.linalg.slogdet(Mpc)
    s_K, ld_K = np.linalg.slogdet(K)
    n_odd_colour = 8 * 3  # odd 4D sites x colours, each carrying one copy of K
    assert abs(ld_D - (ld_P + n_odd_colour * ld_K)) < 1e-10 * abs(ld_D)
    assert abs(s_D - s_P * s_K**n_odd_colour) < 1e-9


def test_mpc_adjoint_and_Gamma5(small):
    dims, Ls, U, shape = small
    even = L.parity_entry_mask(shape, L.EVEN)
    Mpc = L.dense_matrix(lambda v: L.mpc(U, v, M5, MF), shape, even)
    Mdag = L.dense_matrix(lambda v: L.mpc_dag(U, v, M5, MF), shape, even)
    assert np.max(np.abs(Mdag - Mpc.conj().T)) < 1e-13
    psi = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=13), L.EVEN)
    assert rel(L.Gamma5(L.mpc(U, L.Gamma5(psi), M5, MF)), L.mpc_dag(U, psi, M5, MF)) < 1e-14


def test_mpc_free_field_momentum_block():
    """U = 1: M_pc e^{ipx}|_even u = [M5D - Dh(p) M5D^{-1} Dh(p) / 4] u e^{ipx}|_even,
    Dh(p) = 2 sum cos p - 2 i sum gamma_mu sin p_mu (acting on spin; colour trivial)."""
    dims = (4, 2, 6, 2)
    X, Y, Z, T = dims
    Ls = 3
    U = synth.unit_links(dims)
    n = (1, 1, 2, 0)
    p = [2 * np.pi * n[0] / X, 2 * np.pi * n[1] / Y, 2 * np.pi * n[2] / Z, 2 * np.pi * n[3] / T]
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    rng = np.random.default_rng(4)
    u = rng.standard_normal((Ls, 4, 3)) + 1j * rng.standard_normal((Ls, 4, 3))
    psi = L.on_parity(u[:, None, None, None, None] * phase[None, ..., None, None], L.EVEN)
    Dh = 2 * sum(np.cos(q) for q in p) * np.eye(4) - 2j * sum(L.GAMMA[m] * np.sin(p[m]) for m in range(4))
    Dh5 = np.kron(np.eye(Ls), Dh)
    K = L.m5d_matrix(Ls, M5, MF)
    block = K - 0.25 * Dh5 @ np.linalg.inv(K) @ Dh5
    v = (block @ u.reshape(Ls * 4, 3)).reshape(Ls, 4, 3)
    expect = L.on_parity(v[:, None, None, None, None] * phase[None, ..., None, None], L.EVEN)
    assert rel(L.mpc(U, psi, M5, MF), expect) < 1e-14


def test_red_black_solve_matches_dense_solve(small):
    from oracle import krylov

    dims, Ls, U, shape = small
    eta = synth.gaussian_fermion(dims, Ls, seed=14)
    D = L.dense_matrix(lambda v: L.ddw(U, v, M5, MF), shape)
    psi_dense = np.linalg.solve(D, eta.ravel()).reshape(shape)
    b = L.mpc_dag(U, L.schur_source(U, eta, M5, MF), M5, MF)
    res = krylov.cg(lambda v: L.mpcdagmpc(U, v, M5, MF), b, tol=1e-13, maxiter=2000)
    assert res.converged
    psi_o = L.reconstruct_odd(U, res.x, eta, M5, MF)
    psi = res.x + psi_o
    assert rel(psi, psi_dense) < 1e-10
    assert rel(L.ddw(U, psi, M5, MF), eta) < 1e-11


def test_mpcdagmpc_dense_spectrum(small):
    dims, Ls, U, shape = small
    even = L.parity_entry_mask(shape, L.EVEN)
    A = L.dense_matrix(lambda v: L.mpcdagmpc(U, v, M5, MF), shape, even)
    assert np.max(np.abs(A - A.conj().T)) < 1e-12
    w = np.linalg.eigvalsh(A)
    assert w.min() > 0
    Mpc = L.dense_matrix(lambda v: L.mpc(U, v, M5, MF), shape, even)
    sv = np.linalg.svd(Mpc, compute_uv=False)
    assert np.max(np.abs(np.sort(sv**2) - w)) < 1e-11 * w.max()


def test_mpc2_adjoint(small):
    """The second Schur form's adjoint, assembled from adjoint blocks in reverse order,
    is the conjugate transpose of its dense matrix."""
    dims, Ls, U, shape = small
    even = L.parity_entry_mask(shape, L.EVEN)
    M2 = L.dense_matrix(lambda v: L.mpc2(U, v, M5, MF), shape, even)
    M2dag = L.dense_matrix(lambda v: L.mpc2_dag(U, v, M5, MF), shape, even)
    assert np.max(np.abs(M2dag - M2.conj().T)) < 1e-13
    # det(1 - M_ee^{-1} M_eo M_oo^{-1} M_oe) = det M_pc / det M_ee, M_ee = K on each even site and colour
    Mpc = L.dense_matrix(lambda v: L.mpc(U, v, M5, MF), shape, even)
    ld2 = np.linalg.slogdet(M2)[1]
    ld1 = np.linalg.slogdet(Mpc)[1]
    ldK = np.linalg.slogdet(L.m5d_matrix(Ls, M5, MF))[1]
    assert abs(ld2 - (ld1 - 8 * 3 * ldK)) < 1e-10 * abs(ld1)


def test_red_black_solve_form2_matches_dense_solve(small):
    from oracle import krylov

    dims, Ls, U, shape = small
    eta = synth.gaussian_fermion(dims, Ls, seed=15)
    D = L.dense_matrix(lambda v: L.ddw(U, v, M5, MF), shape)
    psi_dense = np.linalg.solve(D, eta.ravel()).reshape(shape)
    b = L.mpc2_dag(U, L.schur_source2(U, eta, M5, MF), M5, MF)
    res = krylov.cg(lambda v: L.mpc2dagmpc2(U, v, M5, MF), b, tol=1e-13, maxiter=2000)
    assert res.converged
    psi = res.x + L.reconstruct_odd(U, res.x, eta, M5, MF)
    assert rel(psi, psi_dense) < 1e-10


def test_unpreconditioned_cgnr_matches_dense_solve(small):
    """CGNR on D_DW^dag D_DW over both parities (the Krylov table's unpreconditioned row)."""
    from oracle import krylov

    dims, Ls, U, shape = small
    eta = synth.gaussian_fermion(dims, Ls, seed=16)
    D = L.dense_matrix(lambda v: L.ddw(U, v, M5, MF), shape)
    psi_dense = np.linalg.solve(D, eta.ravel()).reshape(shape)
    b = L.ddw(U, eta, M5, MF, dag=True)
    res = krylov.cg(lambda v: L.ddw(U, L.ddw(U, v, M5, MF), M5, MF, dag=True), b, tol=1e-13, maxiter=5000)
    assert res.converged
    assert rel(res.x, psi_dense) < 1e-10
