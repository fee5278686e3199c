"""Pins of the oracle's pseudofermion force: finite differences of the action
with dense solves (so the only error is O(eps^2) and rounding), the resolvent
identity, gauge covariance, and the phi-gradient."""

import numpy as np
import pytest

import synth
from oracle import force as F, lattice as L

M5, MF = 1.8, 0.01


@pytest.fixture(scope="module")
def setup():
    dims, Ls = (2, 2, 2, 2), 4
    U = synth.gauge_links(dims, eps=0.5, seed=30)
    phi = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=31), L.EVEN)
    G, gphi = F.force(U, phi, M5, MF, dense=True)
    return dims, Ls, U, phi, G, gphi


def _dense_mpc(U, shape):
    even = L.parity_entry_mask(shape, L.EVEN)
    return L.dense_matrix(lambda v: L.mpc(U, v, M5, MF), shape, even), np.flatnonzero(even.ravel())


def _action_dense(U, phi):
    M, idx = _dense_mpc(U, phi.shape)
    p = phi.reshape(-1)[idx]
    y = np.linalg.solve(M.conj().T, p)  # M^{-dag} phi
    return float(np.vdot(y, y).real)  # phi^dag (M^dag M)^{-1} phi


def test_force_vs_central_differences(setup):
    dims, Ls, U, phi, G, _ = setup
    rng = np.random.default_rng(32)
    eps = 1e-5
    for trial in range(3):
        E = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
        if trial == 2:  # a single link only
            mask = np.zeros(U.shape[:5], dtype=bool)
            mask[1, 0, 1, 0, 2] = True
            E = E * mask[..., None, None]
        s_p = _action_dense(U + eps * E, phi)
        s_m = _action_dense(U - eps * E, phi)
        fd = (s_p - s_m) / (2 * eps)
        an = float(np.sum(np.conj(G) * E).real)
        assert abs(fd - an) < 1e-7 * max(abs(an), 1e-3 * np.abs(G).max())


def test_force_resolvent_identity(setup):
    """S(U+) - S(U-) = X+^dag (A(U-) - A(U+)) X- exactly; no cancellation."""
    dims, Ls, U, phi, G, _ = setup
    rng = np.random.default_rng(33)
    eps = 1e-5
    E = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
    Up, Um = U + eps * E, U - eps * E
    Xp = F.solve_normal(Up, phi, M5, MF, dense=True)
    Xm = F.solve_normal(Um, phi, M5, MF, dense=True)
    diff = L.inner(Xp, L.mpcdagmpc(Um, Xm, M5, MF) - L.mpcdagmpc(Up, Xm, M5, MF)).real
    an = float(np.sum(np.conj(G) * E).real)
    assert abs(diff / (2 * eps) - an) < 1e-8 * abs(an)


def test_force_gauge_covariance(setup):
    dims, Ls, U, phi, G, _ = setup
    g = synth.gauge_transform(dims, seed=34)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ L.dagger(L.shift(g, mu, +1))
    phig = phi @ np.swapaxes(g, -1, -2)
    Gg, _ = F.force(Ug, phig, M5, MF, dense=True)
    for mu in range(4):
        expect = g @ G[..., mu, :, :] @ L.dagger(L.shift(g, mu, +1))
        assert np.max(np.abs(Gg[..., mu, :, :] - expect)) < 1e-10 * np.abs(G).max()


def test_phi_gradient(setup):
    dims, Ls, U, phi, G, gphi = setup
    rng = np.random.default_rng(35)
    eps = 1e-6
    E = L.on_parity(rng.standard_normal(phi.shape) + 1j * rng.standard_normal(phi.shape), L.EVEN)
    fd = (_action_dense(U, phi + eps * E) - _action_dense(U, phi - eps * E)) / (2 * eps)
    an = float(np.sum(np.conj(gphi) * E).real)
    assert abs(fd - an) < 1e-6 * abs(an)


def test_su3_generators():
    T = F.su3_generators()
    for a in range(8):
        assert np.allclose(T[a], T[a].conj().T) and abs(np.trace(T[a])) < 1e-15
        for b in range(8):
            assert abs(np.trace(T[a] @ T[b]) - 0.5 * (a == b)) < 1e-15
    # [T^1, T^2] = i T^3 (structure constant f_123 = 1)
    assert np.allclose(T[0] @ T[1] - T[1] @ T[0], 1j * T[2])


def _expi(H, eps):
    """exp(i eps H) for Hermitian H from its eigendecomposition."""
    w, V = np.linalg.eigh(H)
    return (V * np.exp(1j * eps * w)) @ V.conj().T


def test_lie_force_vs_central_differences(setup):
    """F^a_mu(x) against central differences of the dense action along
    U_mu(x) -> exp(+-i eps T^a) U_mu(x), the eight directions on two links of
    different directions and parities (the update keeps the links in SU(3))."""
    dims, Ls, U, phi, G, _ = setup
    T = F.su3_generators()
    Fl = F.lie_force(U, G)
    eps = 1e-5
    links = [(0, 0, 0, 0, 0), (0, 1, 1, 1, 3)]
    scale = np.abs(Fl).max()
    for link in links:
        for a in range(8):
            Up, Um = U.copy(), U.copy()
            Up[link] = _expi(T[a], eps) @ U[link]
            Um[link] = _expi(T[a], -eps) @ U[link]
            fd = (_action_dense(Up, phi) - _action_dense(Um, phi)) / (2 * eps)
            assert abs(fd - Fl[link][a]) < 1e-7 * max(abs(Fl[link][a]), 1e-2 * scale), (link, a)
