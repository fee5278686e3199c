"""Krylov solver, power method, Chebyshev filters, Gram-Schmidt (oracle; test infrastructure).

* ``cg`` -- Hestenes-Stiefel conjugate gradients on a Hermitian positive
  definite operator (the Spectrum section solves M_pc^dag M_pc psi = eta
  this way; the Results section calls it red-black CGNR).  Stops on the
  recursive relative residual and reports the true one.
* ``power_method`` -- the upper spectral bound lambda_max of M^dag M used by
  the subspace setup (Deflation basis setup section).
* ``chebyshev_filter`` -- T_n(x(A)) v with the interval map
  x = 2 (y - a) / (b - a) - 1 of the Chebyshev smoothers section and the
  three-term recurrence T_{k+1} = 2 x T_k - T_{k-1}.
* ``chebyshev_series`` -- the recursive series of the setup: a low-pass
  prefilter T_m over [lambda_lo, lambda_max], then
  phi_k = T_{k Delta}(2A/lambda_max - 1) applied to the prefiltered vector,
  k = 0..N-1, all from one recurrence (Deflation basis setup section).
* ``gram_schmidt`` -- classical Gram-Schmidt applied twice (CGS2), FP64,
  in vector-index order, giving Q R = V with a positive real diagonal of R.
* ``chebyshev_smoother`` -- S_cheb([a,b],N) r = [c_0/2 + sum_{j=1}^N c_j
  T_j(x(M^dag M))] M^dag r with the coefficients of the Chebyshev
  approximation of 1/y at theta_k = pi (k + 1/2) / N (Chebyshev smoothers
  section); evaluated term by term with T_j from the three-term recurrence.

Vectors are NumPy arrays of any shape; operators are callables.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _dot(a, b) -> complex:
    return complex(np.vdot(a.ravel(), b.ravel()))


def _nrm2(a) -> float:
    return float(np.vdot(a.ravel(), a.ravel()).real)


@dataclass
class CGResult:
    x: np.ndarray
    iterations: int
    converged: bool
    true_rel_residual: float
    history: list = field(default_factory=list)


def cg(apply_A, b, tol=1e-10, maxiter=10000, x0=None) -> CGResult:
    """Solve A x = b (A Hermitian positive definite) by Hestenes-Stiefel CG.

    Convergence test: ||r_k|| / ||b|| < tol on the recursively updated
    residual r_k.  The returned ``true_rel_residual`` is ||b - A x|| / ||b||.
    """
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    p = r.copy()
    bb = _nrm2(b)
    rr = _nrm2(r)
    history = [np.sqrt(rr / bb)]
    it = 0
    converged = rr <= tol * tol * bb
    while not converged and it < maxiter:
        Ap = apply_A(p)
        alpha = rr / _dot(p, Ap).real
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = _nrm2(r)
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
        it += 1
        history.append(np.sqrt(rr / bb))
        converged = rr <= tol * tol * bb
    true = np.sqrt(_nrm2(b - apply_A(x)) / bb)
    return CGResult(x, it, converged, true, history)


def power_method(apply_A, v0, iters=100, rtol=1e-6):
    """Largest eigenvalue of a Hermitian positive operator.

    v <- A v / ||A v|| from the start vector ``v0``; the estimate is the
    Rayleigh quotient <v, A v>.  Stops after ``iters`` steps or when the
    estimate changes by less than ``rtol`` relatively.
    """
    v = v0 / np.sqrt(_nrm2(v0))
    lam = 0.0
    for k in range(iters):
        w = apply_A(v)
        lam_new = _dot(v, w).real
        v = w / np.sqrt(_nrm2(w))
        if k > 0 and abs(lam_new - lam) < rtol * abs(lam_new):
            return lam_new, k + 1
        lam = lam_new
    return lam, iters


def chebyshev_filter(apply_A, v, order: int, lo: float, hi: float):
    """T_order(x(A)) v, x(A) = 2 (A - lo) / (hi - lo) - 1, by the three-term recurrence.

    ``order`` applications of A; no normalisation.  Returns (vector, count).
    """
    if order == 0:
        return v.copy(), 0

    def xA(w):
        return (2.0 * apply_A(w) - (hi + lo) * w) / (hi - lo)

    t_prev = v.copy()
    t_cur = xA(v)
    for _ in range(order - 1):
        t_prev, t_cur = t_cur, 2.0 * xA(t_cur) - t_prev
    return t_cur, order


def chebyshev_series(apply_A, eta, m: int, lam_lo: float, lam_max: float, delta: int, nvec: int):
    """The recursive setup series phi_k = T_{k Delta}(2A/lam_max - 1) T_m(x_lo(A)) eta.

    The prefilter maps [lam_lo, lam_max] to [-1, 1].  The later filters map
    [0, lam_max] to [-1, 1] and are all taken from one three-term recurrence
    started at the prefiltered vector, recording every ``delta`` steps, so
    phi_0 is the prefiltered vector itself.

    Returns (list of nvec vectors, number of applications of A).
    """
    v0, count = chebyshev_filter(apply_A, eta, m, lam_lo, lam_max)
    phis = [v0.copy()]
    if nvec == 1:
        return phis, count

    def xA(w):
        return (2.0 * apply_A(w) - lam_max * w) / lam_max

    t_prev = v0
    t_cur = xA(v0)
    count += 1
    n = 1
    while len(phis) < nvec:
        if n % delta == 0:
            phis.append(t_cur.copy())
            if len(phis) == nvec:
                break
        t_prev, t_cur = t_cur, 2.0 * xA(t_cur) - t_prev
        count += 1
        n += 1
    return phis, count


def gram_schmidt(vectors):
    """CGS2 in FP64: returns (Q, R) with Q R = V column-wise and R_ii > 0.

    ``vectors`` is a list of equal-shaped arrays; Q is returned as a list of
    arrays of that shape.
    """
    shape = vectors[0].shape
    V = np.stack([np.asarray(v, dtype=np.complex128).ravel() for v in vectors], axis=1)
    n, k = V.shape
    Q = np.zeros_like(V)
    R = np.zeros((k, k), dtype=np.complex128)
    for j in range(k):
        w = V[:, j].copy()
        for _ in range(2):
            h = Q[:, :j].conj().T @ w
            w = w - Q[:, :j] @ h
            R[:j, j] += h
        rjj = np.sqrt(np.vdot(w, w).real)
        R[j, j] = rjj
        Q[:, j] = w / rjj
    return [Q[:, j].reshape(shape) for j in range(k)], R


def chebyshev_smoother_coeffs(a: float, b: float, N: int):
    """c_j = (2/N) sum_{k<N} f(y(cos theta_k)) cos(j theta_k), j = 0..N, f(y) = 1/y,
    theta_k = pi (k + 1/2) / N, y(x) = a + (b - a)(x + 1)/2 (the inverse of the interval map)."""
    theta = np.pi * (np.arange(N) + 0.5) / N
    y = a + (b - a) * (np.cos(theta) + 1.0) / 2.0
    f = 1.0 / y
    return np.array([2.0 / N * np.sum(f * np.cos(j * theta)) for j in range(N + 1)])


def chebyshev_smoother(apply_A, apply_Mdag, r, a: float, b: float, N: int):
    """S_cheb([a,b],N) r: the polynomial sum_j c_j T_j(x(A)) (c_0 halved) applied to M^dag r."""
    c = chebyshev_smoother_coeffs(a, b, N)
    w = apply_Mdag(r)

    def xA(v):
        return (2.0 * apply_A(v) - (b + a) * v) / (b - a)

    t_prev = w
    out = 0.5 * c[0] * w
    if N >= 1:
        t_cur = xA(w)
        out = out + c[1] * t_cur
        for j in range(2, N + 1):
            t_prev, t_cur = t_cur, 2.0 * xA(t_cur) - t_prev
            out = out + c[j] * t_cur
    return out
