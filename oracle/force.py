"""Pseudofermion action and its gauge-link gradient (oracle; test infrastructure).

The Conclusions motivate the method by HMC with the two-flavour
determinant det(M^dag M); its pseudofermion estimator is
S(U) = phi^dag (M_pc^dag M_pc)^{-1} phi.  The paper gives no force formula,
so it is derived here from the Schur blocks:

    X = A^{-1} phi,  A = M_pc^dag M_pc,   Y = M_pc X,
    dS = -X^dag dA X = -2 Re(Y^dag dM_pc X),
    dM_pc = -dM_eo M_oo^{-1} M_oe - M_eo M_oo^{-1} dM_oe,  dM_eo = -dD_hop^{eo}/2.

With Z = M_oo^{-1} M_oe X and W = M_oo^{-dag} M_eo^dag Y on odd sites and
the full-lattice fields a = (Y even, W odd), b = (X even, Z odd):

    dS = -Re(a^dag dD_hop b),

so for the link U_mu(x) (both terms of D_hop that contain it):

    G_mu(x) = -sum_s sum_spin [ a(x,s) ((1 - g_mu) b(x+mu,s))^dag
                               + ((1 + g_mu) b(x,s)) a(x+mu,s)^dag ],

the colour outer products summed over spin.  G follows PyTorch's complex
gradient convention, G = dS/dRe U + i dS/dIm U, so that
dS = Re sum conj(G) dU for any complex perturbation dU.
"""

from __future__ import annotations

import numpy as np

from . import lattice as L
from . import krylov


def action(U, phi, M5, mf, tol=1e-14, maxiter=100000, dense=False):
    """S = Re phi^dag A^{-1} phi, with A^{-1} phi by CG (or by a dense solve)."""
    X = solve_normal(U, phi, M5, mf, tol, maxiter, dense)
    return float(np.vdot(phi.ravel(), X.ravel()).real), X


def solve_normal(U, phi, M5, mf, tol=1e-14, maxiter=100000, dense=False):
    def A(v):
        return L.mpcdagmpc(U, v, M5, mf)

    if dense:
        mask = L.parity_entry_mask(phi.shape, L.EVEN)
        M = L.dense_matrix(A, phi.shape, mask)
        x = np.zeros(phi.shape, dtype=np.complex128)  # C-contiguous: reshape(-1) is a view
        flat = x.reshape(-1)
        idx = np.flatnonzero(mask.ravel())
        flat[idx] = np.linalg.solve(M, phi.ravel()[idx])
        return x
    return krylov.cg(A, phi, tol=tol, maxiter=maxiter).x


def outer_sum(v, w):
    """sum over s and spin of v w^dag per 4D site: out[..., a, b] = sum v[a] conj(w[b])."""
    return np.einsum("s...ia,s...ib->...ab", v, np.conj(w))


def link_gradient(U, X, Y, M5, mf):
    """G_mu(x) from X = A^{-1} phi and Y = M_pc X (both on even sites)."""
    Z = L.m5d_inv(L.m_oe(U, X), M5, mf)
    W = L.m5d_inv(L.m_eo(U, Y, dag=True), M5, mf, dag=True)
    a = L.on_parity(Y, L.EVEN) + L.on_parity(W, L.ODD)
    b = L.on_parity(X, L.EVEN) + L.on_parity(Z, L.ODD)
    G = np.zeros_like(U)
    for mu in range(4):
        b_fwd = L.shift(b, mu, +1)
        a_fwd = L.shift(a, mu, +1)
        term1 = outer_sum(a, L.spin_mul(L.IDENT4 - L.GAMMA[mu], b_fwd))
        term2 = outer_sum(L.spin_mul(L.IDENT4 + L.GAMMA[mu], b), a_fwd)
        G[..., mu, :, :] = -(term1 + term2)
    return G


def force(U, phi, M5, mf, tol=1e-14, maxiter=100000, dense=False):
    """dS/dU (PyTorch convention) and dS/dphi = 2 X for S = phi^dag A^{-1} phi."""
    X = solve_normal(U, phi, M5, mf, tol, maxiter, dense)
    Y = L.mpc(U, X, M5, mf)
    return link_gradient(U, X, Y, M5, mf), 2.0 * X


def su3_generators():
    """T^a = lambda^a / 2 with the Gell-Mann matrices lambda^a, a = 1..8 (index 0..7):
    Hermitian, traceless, tr(T^a T^b) = delta_ab / 2."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return lam / 2


def lie_force(U, G):
    """Derivative of S along the Lie-algebra directions of each link:
    F^a_mu(x) = dS/d omega at omega = 0 for U_mu(x) -> exp(i omega T^a) U_mu(x).

    The variation is dU = i omega T^a U, and dS = Re sum conj(G) dU = Re tr(G^dag dU)
    in the gradient convention above, so F^a = Re tr(i T^a U G^dag) = -Im tr(T^a U G^dag).
    Returns F[..., mu, a] (real)."""
    T = su3_generators()
    M = np.einsum("...ab,...cb->...ac", U, np.conj(G))  # U G^dag
    return -np.einsum("kab,...ba->...k", T, M).imag
