"""Domain-wall operators in plain NumPy complex128 (oracle; test infrastructure).

Every function follows a definition of the paper's "Chiral Fermion Actions"
section, written out without blocking, fusion or spin-projection tricks:

* ``dhop``   -- the Wilson hopping term (the D_hop equation): forward hop
  with (1 - gamma_mu) U_mu(x), backward hop with (1 + gamma_mu) U_mu(x-mu)^dag,
  summed over mu = x, y, z, t.  The adjoint is written from the matrix
  elements (projector signs swap), not through gamma5.
* ``wilson`` -- D_W(M) = M + 4 - D_hop / 2.
* ``m5d_matrix`` -- the fifth-dimension part of the D_DW matrix with the
  hopping term removed: (5 - M5) on the diagonal, -P_- above it, -P_+ below
  it, m P_+ in the top-right and m P_- in the bottom-left corner.
* ``ddw``    -- D_DW = M5D - D_hop / 2 on every s slice (D_par = 5 - M5 - D_hop/2).
* ``Gamma5`` -- gamma5 times the reflection s -> Ls-1-s.
* the Schur blocks M_ee = M_oo = M5D, M_eo = -D_hop^{eo}/2, M_oe = -D_hop^{oe}/2
  and the preconditioned operator M_pc = M_ee - M_eo M_oo^{-1} M_oe that the
  Results section's red-black CGNR solves with (normal form M_pc^dag M_pc).

M5D^{-1} is the dense inverse of the 4Ls x 4Ls matrix; it is the same at
every 4D site and does not touch colour.

Readings where the paper is silent: chiral gamma basis (below), P_+- =
(1 +- gamma5)/2, the sum over mu implicit in D_hop, periodic 4D boundaries,
4D (not 5D) checkerboarding, parity = (x+y+z+t) mod 2 with even = 0.
"""

from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# Gamma matrices: chiral basis, mu = x, y, z, t.  Each gamma_mu has zero
# diagonal 2x2 blocks; gamma5 = gamma_x gamma_y gamma_z gamma_t = diag(1,1,-1,-1).
# ---------------------------------------------------------------------------
_i = 1j
GAMMA = np.array(
    [
        [[0, 0, 0, _i], [0, 0, _i, 0], [0, -_i, 0, 0], [-_i, 0, 0, 0]],  # x
        [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],  # y
        [[0, 0, _i, 0], [0, 0, 0, -_i], [-_i, 0, 0, 0], [0, _i, 0, 0]],  # z
        [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],  # t
    ],
    dtype=np.complex128,
)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
IDENT4 = np.eye(4, dtype=np.complex128)
P_PLUS = 0.5 * (IDENT4 + GAMMA5)
P_MINUS = 0.5 * (IDENT4 - GAMMA5)


# ---------------------------------------------------------------------------
# Small helpers on natural-layout arrays.  A 4D fermion is [T,Z,Y,X,4,3]; a
# 5D fermion has a leading Ls axis.  Lattice axis of direction mu, counted
# from the end: x -> -3, y -> -4, z -> -5, t -> -6 (links [T,Z,Y,X,3,3] use
# the same offsets).
# ---------------------------------------------------------------------------
def _axis(mu: int) -> int:
    return -3 - mu


def shift(field: np.ndarray, mu: int, step: int) -> np.ndarray:
    """``out(x) = field(x + step * mu_hat)`` with periodic boundaries."""
    return np.roll(field, -step, axis=_axis(mu))


def spin_mul(g: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """Apply a 4x4 spin matrix to every site: out[.., a, c] = g[a, b] psi[.., b, c]."""
    return g @ psi


def colour_mul(u: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """Apply a per-site 3x3 colour matrix: out[.., s, a] = u[.., a, b] psi[.., s, b]."""
    return psi @ np.swapaxes(u, -1, -2)


def dagger(u: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(u, -1, -2))


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    """<a, b> = sum conj(a) b."""
    return complex(np.vdot(a.ravel(), b.ravel()))


def norm2(a: np.ndarray) -> float:
    return float(np.vdot(a.ravel(), a.ravel()).real)


def dims_of(U: np.ndarray):
    T, Z, Y, X = U.shape[:4]
    return (X, Y, Z, T)


# ---------------------------------------------------------------------------
# Wilson hopping term and Wilson operator.
# ---------------------------------------------------------------------------
def dhop(U: np.ndarray, psi: np.ndarray, dag: bool = False) -> np.ndarray:
    """D_hop psi (or D_hop^dag psi) on every slice of ``psi``.

    Non-adjoint: sum_mu (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu).
    Adjoint: the same hops with (1 + g_mu) forward and (1 - g_mu) backward,
    which is the conjugate transpose of the matrix elements above.
    """
    out = np.zeros_like(psi)
    for mu in range(4):
        u = U[..., mu, :, :]
        u_back = dagger(shift(u, mu, -1))  # U_mu(x - mu)^dag
        fwd = colour_mul(u, shift(psi, mu, +1))
        bwd = colour_mul(u_back, shift(psi, mu, -1))
        if not dag:
            out += spin_mul(IDENT4 - GAMMA[mu], fwd) + spin_mul(IDENT4 + GAMMA[mu], bwd)
        else:
            out += spin_mul(IDENT4 + GAMMA[mu], fwd) + spin_mul(IDENT4 - GAMMA[mu], bwd)
    return out


def wilson(U: np.ndarray, psi: np.ndarray, M: float, dag: bool = False) -> np.ndarray:
    """D_W(M) psi = (M + 4) psi - D_hop psi / 2."""
    return (M + 4.0) * psi - 0.5 * dhop(U, psi, dag)


def gamma5(psi: np.ndarray) -> np.ndarray:
    return spin_mul(GAMMA5, psi)


# ---------------------------------------------------------------------------
# Fifth dimension: M5D (the D_DW matrix without D_hop) as an explicit
# (Ls*4) x (Ls*4) matrix acting on (s, spin), identical at every 4D site.
# ---------------------------------------------------------------------------
def m5d_matrix(Ls: int, M5: float, mf: float) -> np.ndarray:
    """The Ls x Ls block matrix of D_DW with D_par replaced by 5 - M5.

    Blocks are 4x4 spin matrices; entries are accumulated so that at Ls = 1
    and Ls = 2 the corner blocks add onto the diagonal / off-diagonal ones.
    """
    K = np.zeros((Ls, 4, Ls, 4), dtype=np.complex128)
    for s in range(Ls):
        K[s, :, s, :] += (5.0 - M5) * IDENT4
        if s + 1 < Ls:
            K[s, :, s + 1, :] += -P_MINUS
        if s - 1 >= 0:
            K[s, :, s - 1, :] += -P_PLUS
    K[0, :, Ls - 1, :] += mf * P_PLUS
    K[Ls - 1, :, 0, :] += mf * P_MINUS
    return K.reshape(4 * Ls, 4 * Ls)


def apply_fifth(K: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """out[s, .., a, c] = sum_{s', b} K[(s,a), (s',b)] psi[s', .., b, c]."""
    Ls = psi.shape[0]
    rest = psi.shape[1:-2]
    x = np.moveaxis(psi, -2, 1)  # [Ls, 4, ..., 3]
    flat = x.reshape(Ls * 4, -1)
    y = (K @ flat).reshape((Ls, 4) + rest + (3,))
    return np.ascontiguousarray(np.moveaxis(y, 1, -2))


def m5d(psi, M5, mf, dag=False):
    K = m5d_matrix(psi.shape[0], M5, mf)
    return apply_fifth(K.conj().T if dag else K, psi)


def m5d_inv(psi, M5, mf, dag=False):
    K = np.linalg.inv(m5d_matrix(psi.shape[0], M5, mf))
    return apply_fifth(K.conj().T if dag else K, psi)


# ---------------------------------------------------------------------------
# Shamir domain-wall operator, Gamma5, H_DW.
# ---------------------------------------------------------------------------
def ddw(U, psi, M5, mf, dag=False):
    """D_DW psi: on each slice D_par = 5 - M5 - D_hop/2 plus the s couplings."""
    return m5d(psi, M5, mf, dag) - 0.5 * dhop(U, psi, dag)


def reflect5(psi):
    return psi[::-1].copy()


def Gamma5(psi):
    """Gamma_5 = gamma_5 R_5."""
    return gamma5(reflect5(psi))


def hdw(U, psi, M5, mf):
    """H_DW = Gamma_5 D_DW."""
    return Gamma5(ddw(U, psi, M5, mf))


# ---------------------------------------------------------------------------
# Checkerboarding (4D parity) and the Schur complement.
# ---------------------------------------------------------------------------
def parity_of_sites(dims) -> np.ndarray:
    """(x + y + z + t) mod 2 on the [T,Z,Y,X] grid."""
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    return (x + y + z + t) % 2


def on_parity(psi: np.ndarray, parity: int) -> np.ndarray:
    """Keep the sites of one parity, zero the others."""
    T, Z, Y, X = psi.shape[-6:-2]
    keep = parity_of_sites((X, Y, Z, T)) == parity
    return psi * keep[..., None, None]


EVEN, ODD = 0, 1


def m_eo(U, v_odd, dag=False):
    """M_eo v = -D_hop^{e<-o} v / 2; with dag, (M_eo)^dag v = -(D_hop^dag)^{o<-e} v / 2."""
    if not dag:
        return -0.5 * on_parity(dhop(U, on_parity(v_odd, ODD)), EVEN)
    return -0.5 * on_parity(dhop(U, on_parity(v_odd, EVEN), dag=True), ODD)


def m_oe(U, v_even, dag=False):
    """M_oe v = -D_hop^{o<-e} v / 2; with dag, (M_oe)^dag v = -(D_hop^dag)^{e<-o} v / 2."""
    if not dag:
        return -0.5 * on_parity(dhop(U, on_parity(v_even, EVEN)), ODD)
    return -0.5 * on_parity(dhop(U, on_parity(v_even, ODD), dag=True), EVEN)


def mpc(U, psi_e, M5, mf):
    """M_pc psi_e = M_ee psi_e - M_eo M_oo^{-1} M_oe psi_e (first Schur form)."""
    t = m5d_inv(m_oe(U, psi_e), M5, mf)
    return m5d(psi_e, M5, mf) - m_eo(U, t)


def mpc_dag(U, psi_e, M5, mf):
    """M_pc^dag = M_ee^dag - M_oe^dag M_oo^{-dag} M_eo^dag, assembled from adjoint blocks."""
    t = m5d_inv(m_eo(U, psi_e, dag=True), M5, mf, dag=True)
    return m5d(psi_e, M5, mf, dag=True) - m_oe(U, t, dag=True)


def mpcdagmpc(U, psi_e, M5, mf):
    return mpc_dag(U, mpc(U, psi_e, M5, mf), M5, mf)


def mpc2(U, psi_e, M5, mf):
    """Second Schur form (Results, Krylov table): 1 - M_ee^{-1} M_eo M_oo^{-1} M_oe."""
    t = m5d_inv(m_oe(U, psi_e), M5, mf)
    return psi_e - m5d_inv(m_eo(U, t), M5, mf)


def mpc2_dag(U, psi_e, M5, mf):
    """(1 - M_ee^{-1} M_eo M_oo^{-1} M_oe)^dag = 1 - M_oe^dag M_oo^{-dag} M_eo^dag M_ee^{-dag}."""
    y = m5d_inv(psi_e, M5, mf, dag=True)
    t = m5d_inv(m_eo(U, y, dag=True), M5, mf, dag=True)
    return psi_e - m_oe(U, t, dag=True)


def mpc2dagmpc2(U, psi_e, M5, mf):
    return mpc2_dag(U, mpc2(U, psi_e, M5, mf), M5, mf)


def schur_source2(U, eta, M5, mf):
    """Right-hand side of the second form: M_ee^{-1} eta'."""
    return m5d_inv(schur_source(U, eta, M5, mf), M5, mf)


def schur_source(U, eta, M5, mf):
    """eta' = eta_e - M_eo M_oo^{-1} eta_o (the even-site source of the Schur system)."""
    eta_e = on_parity(eta, EVEN)
    eta_o = on_parity(eta, ODD)
    return eta_e - m_eo(U, m5d_inv(eta_o, M5, mf))


def reconstruct_odd(U, psi_e, eta, M5, mf):
    """psi_o = M_oo^{-1} (eta_o - M_oe psi_e)."""
    eta_o = on_parity(eta, ODD)
    return m5d_inv(eta_o - m_oe(U, psi_e), M5, mf)


# ---------------------------------------------------------------------------
# Dense matrices of small operators (for eigen-decompositions and solves).
# ---------------------------------------------------------------------------
def dense_matrix(apply, shape, sites_mask=None) -> np.ndarray:
    """The matrix of a linear map on arrays of ``shape`` (optionally restricted
    to the entries where ``sites_mask`` is True), built column by column."""
    n_all = int(np.prod(shape))
    if sites_mask is None:
        idx = np.arange(n_all)
    else:
        idx = np.flatnonzero(np.broadcast_to(sites_mask, shape).ravel())
    cols = []
    for k in idx:
        e = np.zeros(n_all, dtype=np.complex128)
        e[k] = 1.0
        cols.append(apply(e.reshape(shape)).ravel()[idx])
    return np.stack(cols, axis=1)


def parity_entry_mask(shape, parity) -> np.ndarray:
    """Boolean mask over a 5D field's entries that lie on one 4D parity."""
    T, Z, Y, X = shape[-6:-2]
    m = parity_of_sites((X, Y, Z, T)) == parity
    return np.broadcast_to(m[..., None, None], shape)
