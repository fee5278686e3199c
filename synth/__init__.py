"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module draws random numbers and nothing else: it holds none of the
arithmetic of the domain-wall operator, its solvers or its filters.  Both
the CPU oracle (through the tests) and the HIP path (through the tests and
the benchmark) take their inputs from here, in the natural lattice layout:

* gauge links  ``U[T][Z][Y][X][mu][a][b]``, complex128, mu = x, y, z, t;
* 5D fermions  ``psi[Ls][T][Z][Y][X][spin][colour]``, complex128
  (with a leading ``nrhs`` axis for batches).

Lattice extents are given as ``dims = (X, Y, Z, T)``.

The paper measures on gauge configurations of an RBC/UKQCD ensemble
(Results section); those are not available, so links are synthetic:
``U = exp(i * eps * H)`` with ``H`` a traceless Hermitian 3x3 matrix whose
independent entries are standard normal.  A gauge transformation field
(for covariance checks) is drawn the same way.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "gauge_links",
    "gauge_transform",
    "unit_links",
    "gaussian_fermion",
    "gaussian_fermion_batch",
    "gaussian_fermion_device",
    "random_link_sites",
]


def _random_su3(rng: np.random.Generator, n: int, eps: float) -> np.ndarray:
    """``n`` matrices ``exp(i eps H)``, H traceless Hermitian with N(0,1) entries.

    Draw order per matrix: the 3 diagonal entries, then the 3 real parts and
    the 3 imaginary parts of the upper triangle (01, 02, 12).
    """
    g = rng.standard_normal((n, 9))
    h = np.zeros((n, 3, 3), dtype=np.complex128)
    h[:, 0, 0], h[:, 1, 1], h[:, 2, 2] = g[:, 0], g[:, 1], g[:, 2]
    upper = g[:, 3:6] + 1j * g[:, 6:9]
    for k, (i, j) in enumerate(((0, 1), (0, 2), (1, 2))):
        h[:, i, j] = upper[:, k]
        h[:, j, i] = np.conj(upper[:, k])
    tr = np.trace(h, axis1=1, axis2=2).real / 3.0
    for i in range(3):
        h[:, i, i] -= tr
    w, v = np.linalg.eigh(h)
    phase = np.exp(1j * eps * w)
    return np.einsum("nab,nb,ncb->nac", v, phase, np.conj(v))


def gauge_links(dims, eps: float, seed: int = 0) -> np.ndarray:
    """Synthetic SU(3) links ``U[T][Z][Y][X][4][3][3]`` (complex128).

    Links are drawn site by site (x fastest), and within a site for
    mu = x, y, z, t in that order.
    """
    X, Y, Z, T = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    u = _random_su3(rng, T * Z * Y * X * 4, eps)
    return u.reshape(T, Z, Y, X, 4, 3, 3)


def unit_links(dims) -> np.ndarray:
    """The free field: every link is the identity."""
    X, Y, Z, T = (int(d) for d in dims)
    u = np.zeros((T, Z, Y, X, 4, 3, 3), dtype=np.complex128)
    for a in range(3):
        u[..., a, a] = 1.0
    return u


def gauge_transform(dims, eps: float = 1.0, seed: int = 7) -> np.ndarray:
    """A random SU(3) matrix per 4D site, ``g[T][Z][Y][X][3][3]``."""
    X, Y, Z, T = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    return _random_su3(rng, T * Z * Y * X, eps).reshape(T, Z, Y, X, 3, 3)


def gaussian_fermion(dims, Ls: int, seed: int) -> np.ndarray:
    """Complex Gaussian 5D field ``psi[Ls][T][Z][Y][X][4][3]``; Re, Im ~ N(0,1)."""
    X, Y, Z, T = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((Ls, T, Z, Y, X, 4, 3, 2))
    return g[..., 0] + 1j * g[..., 1]


def gaussian_fermion_batch(dims, Ls: int, nrhs: int, seed: int) -> np.ndarray:
    """``nrhs`` Gaussian fields drawn in sequence from one generator."""
    X, Y, Z, T = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((nrhs, Ls, T, Z, Y, X, 4, 3, 2))
    return g[..., 0] + 1j * g[..., 1]


def gaussian_fermion_device(dims, Ls: int, nrhs: int, seed: int, device="cuda"):
    """``nrhs`` complex Gaussian fields ``[nrhs][Ls][T][Z][Y][X][4][3]`` (complex128, Re, Im
    ~ N(0,1)) drawn on a torch device from a generator seeded with ``seed``.  For lattices
    whose host-side draw would take minutes; a different stream of numbers from
    ``gaussian_fermion_batch`` with the same seed."""
    import torch

    X, Y, Z, T = (int(d) for d in dims)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    g = torch.randn((nrhs, Ls, T, Z, Y, X, 4, 3, 2), dtype=torch.float64, device=device, generator=gen)
    return torch.view_as_complex(g)


def random_link_sites(dims, count: int, seed: int):
    """``count`` distinct (t, z, y, x, mu) link coordinates, uniform."""
    X, Y, Z, T = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    flat = rng.choice(T * Z * Y * X * 4, size=count, replace=False)
    out = []
    for f in flat:
        mu = int(f % 4)
        site = int(f // 4)
        x = site % X
        y = (site // X) % Y
        z = (site // (X * Y)) % Z
        t = site // (X * Y * Z)
        out.append((t, z, y, x, mu))
    return out
