"""Two-level HDCR solver on the full lattice (oracle; test infrastructure).

HDCR coarsens the Hermitian domain-wall operator M = H_DW = Gamma_5 D_DW
(Spectrum of domain wall fermions section) over blocks of 4D sites taken with
all Ls slices, and solves D_DW psi = eta through H_DW psi = Gamma_5 eta with
an outer preconditioned GCR whose preconditioner is the composite V(1,1) cycle
(Algorithms A and B: pGCR(H_DW), Chebyshev smoother, CGNR coarse solve).

* ``hdw_normal`` -- M^dag M = H_DW^2 = D_DW^dag D_DW.
* ``smoother`` -- S_cheb([a,b],N) of the Chebyshev smoothers section with
  M = H_DW: the Chebyshev approximation of 1/y on [a, b] in M^dag M, applied
  to M^dag r = H_DW r.
* ``coarse_operator`` -- the little Dirac operator
  A^{ab}_{jk} = <phi_j^a | M | phi_k^b> (Two level preconditioner section),
  as a dense [nb * n, nb * n] matrix, row (a, j) and column (b, k) at
  a * n + j and b * n + k: column (b, k) is the restriction of M phi_k^b.
* ``coarse_solve`` -- A c = d by conjugate gradients on the normal residual
  system A^dag A c = A^dag d from c = 0 (the coarse solver of Algorithms A / B),
  stopped on the relative residual of the normal system.
* ``coarse_correction`` -- Q r = P A^{-1} P^dag r with the prolongator P and
  restrictor P^dag of the blocked basis.
* ``vcycle`` -- the V(1,1) sequence of the Composite V(1,1) section:
  x1 = S r0, x2 = x1 + Q (r0 - M x1), x3 = x2 + S (r0 - M x2), from x0 = 0.
* ``gcr`` -- generalised conjugate residuals with a (possibly varying) right
  preconditioner K: z_k = K r, w_k = M z_k, w_k made orthonormal to the earlier
  w_i by modified Gram-Schmidt (the same combination applied to z_k), then
  x += <w_k, r> z_k and r -= <w_k, r> w_k; restarted from the true residual
  after ``nkrylov`` directions.  The paper calls it pGCR and leaves its
  details to the literature; this is the flexible variant, which a
  preconditioner containing an inexact inner solve needs.
* ``hdcr_solve`` -- psi with D_DW psi = eta: gcr on H_DW with the V(1,1)
  preconditioner for the source Gamma_5 eta.

Fields are natural-layout complex128 arrays [Ls, T, Z, Y, X, 4, 3] on both
parities; coarse vectors are [nb * n] complex128, block-major.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from oracle import coarse as C
from oracle import krylov
from oracle import lattice as L


def _dot(a, b) -> complex:
    return complex(np.vdot(a.ravel(), b.ravel()))


def _nrm(a) -> float:
    return float(np.sqrt(np.vdot(a.ravel(), a.ravel()).real))


def hdw_normal(U, v, M5, mf):
    """H_DW^2 v = D_DW^dag D_DW v."""
    return L.ddw(U, L.ddw(U, v, M5, mf), M5, mf, dag=True)


def smoother(U, r, M5, mf, lo, hi, N):
    """S_cheb([lo, hi], N) r with M = H_DW: polynomial in M^dag M applied to M^dag r = H_DW r."""
    return krylov.chebyshev_smoother(
        lambda v: hdw_normal(U, v, M5, mf), lambda v: L.hdw(U, v, M5, mf), r, lo, hi, N
    )


def blocked(phi, b, dims, block):
    """phi^b: phi on the sites of block b, zero elsewhere."""
    mask = (C.block_of_sites(dims, block) == b)[..., None, None]
    return np.where(mask, phi, 0)


def coarse_operator(apply_M, basis, dims, block):
    """Dense little Dirac operator of apply_M on the blocked basis."""
    n = len(basis)
    nb = C.nblocks(dims, block)
    A = np.zeros((nb * n, nb * n), dtype=np.complex128)
    for b in range(nb):
        for k in range(n):
            col = C.restrict(basis, apply_M(blocked(basis[k], b, dims, block)), dims, block)  # [nb, n]
            A[:, b * n + k] = col.reshape(-1)
    return A


def restrict(basis, v, dims, block):
    return C.restrict(basis, v, dims, block).reshape(-1)


def prolong(basis, c, dims, block):
    return C.prolong(basis, c.reshape(-1, len(basis)), dims, block)


@dataclass
class CoarseResult:
    x: np.ndarray
    iterations: int


def coarse_solve(A, d, tol, maxiter=10000):
    """CGNR on A: CG on A^dag A c = A^dag d from c = 0, relative residual of the normal system."""
    Ah = A.conj().T
    res = krylov.cg(lambda v: Ah @ (A @ v), Ah @ d, tol=tol, maxiter=maxiter)
    return CoarseResult(res.x, res.iterations)


def coarse_correction(A, basis, r, dims, block, tol=None, maxiter=10000):
    """Q r = P A^{-1} P^dag r; tol None takes the exact dense inverse."""
    d = restrict(basis, r, dims, block)
    c = np.linalg.solve(A, d) if tol is None else coarse_solve(A, d, tol, maxiter).x
    return prolong(basis, c, dims, block)


@dataclass
class Level:
    """Everything one V(1,1) cycle needs."""

    U: np.ndarray
    M5: float
    mf: float
    basis: list
    A: np.ndarray
    dims: tuple
    block: tuple
    lo: float
    hi: float
    order: int
    coarse_tol: float | None
    coarse_maxiter: int = 10000

    def M(self, v):
        return L.hdw(self.U, v, self.M5, self.mf)

    def S(self, r):
        return smoother(self.U, r, self.M5, self.mf, self.lo, self.hi, self.order)

    def Q(self, r):
        return coarse_correction(self.A, self.basis, r, self.dims, self.block, self.coarse_tol, self.coarse_maxiter)


def vcycle(lv: Level, r0):
    """x3 of the V(1,1) sequence from x0 = 0 (pre-smoother, coarse correction, post-smoother)."""
    x1 = lv.S(r0)
    r1 = r0 - lv.M(x1)
    x2 = x1 + lv.Q(r1)
    r2 = r0 - lv.M(x2)
    return x2 + lv.S(r2)


@dataclass
class GCRResult:
    x: np.ndarray
    iterations: int
    converged: bool
    true_rel_residual: float
    history: list = field(default_factory=list)


def gcr(apply_M, precond, b, tol=1e-10, maxiter=1000, nkrylov=8, x0=None) -> GCRResult:
    """Flexible right-preconditioned GCR with restarts (see the module notes)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bn = _nrm(b)
    r = b - apply_M(x) if x0 is not None else b.copy()
    hist = [_nrm(r) / bn if bn > 0 else 0.0]
    it = 0
    converged = bn == 0 or hist[0] <= tol
    while not converged and it < maxiter:
        Z, W = [], []
        for _ in range(nkrylov):
            z = precond(r)
            w = apply_M(z)
            for zi, wi in zip(Z, W):
                beta = _dot(wi, w)
                w = w - beta * wi
                z = z - beta * zi
            nw = _nrm(w)
            if nw == 0:
                raise FloatingPointError("GCR breakdown: M z = 0")
            w, z = w / nw, z / nw
            alpha = _dot(w, r)
            x = x + alpha * z
            r = r - alpha * w
            Z.append(z)
            W.append(w)
            it += 1
            hist.append(_nrm(r) / bn)
            if hist[-1] <= tol or it >= maxiter:
                converged = hist[-1] <= tol
                break
        if not converged:
            r = b - apply_M(x)  # restart from the true residual
    true = _nrm(b - apply_M(x)) / bn if bn > 0 else 0.0
    return GCRResult(x, it, converged, true, hist)


def hdcr_solve(lv: Level, eta, tol=1e-10, maxiter=1000, nkrylov=8) -> GCRResult:
    """D_DW psi = eta via pGCR(H_DW) on H_DW psi = Gamma_5 eta with the V(1,1) preconditioner."""
    return gcr(lv.M, lambda r: vcycle(lv, r), L.Gamma5(eta), tol=tol, maxiter=maxiter, nkrylov=nkrylov)
