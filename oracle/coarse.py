"""Coarse-space transfer of the two-level method (oracle; test infrastructure).

* ``chiral_split`` -- each subspace vector v becomes the two chiral halves
  (1 + Gamma_5) v / 2 and (1 - Gamma_5) v / 2 with (Gamma_5 v)_s =
  gamma_5 v_{Ls-1-s}, the five-dimensional chirality used when the domain-wall
  operator itself is coarsened (Deflation basis setup section, after the
  filter; Gamma_5 as in the Chiral Fermion Actions section).
* ``block_of_sites`` -- the blocks b of the Two level preconditioner section:
  4D boxes of bx*by*bz*bt sites tiling the lattice, each taken with all Ls
  slices (the Algorithm A / B table uses 4x2x4x2x16 and 2^4x16 at Ls = 16).
* ``block_orthonormalize`` -- the blocked basis phi_k^b (the vector
  restricted to block b) made orthonormal inside every block: classical
  Gram-Schmidt applied twice, in vector-index order, independently per block,
  so that Q^b R^b = V^b with R^b upper triangular and a positive real
  diagonal.
* ``restrict`` / ``prolong`` -- the restrictor <phi_k^b| and the prolongator
  |phi_k^b> of the Two level preconditioner section: c_k^b = <phi_k^b, v> and
  v = sum_{b,k} c_k^b phi_k^b.

Fields are natural-layout complex128 arrays [..., Ls, T, Z, Y, X, 4, 3];
coarse vectors are [nblocks, nvec] complex128 with blocks numbered
lexicographically (bx-block index fastest).
"""

from __future__ import annotations

import numpy as np

from oracle import lattice as L


def chiral_split(v: np.ndarray):
    """(P+ v, P- v) with P+- = (1 +- Gamma_5) / 2."""
    g = L.Gamma5(v)
    return 0.5 * (v + g), 0.5 * (v - g)


def block_of_sites(dims, block) -> np.ndarray:
    """Block number of every 4D site, as an array [T, Z, Y, X]."""
    X, Y, Z, T = dims
    bx, by, bz, bt = block
    if X % bx or Y % by or Z % bz or T % bt:
        raise ValueError("block extents must divide the lattice extents")
    nx, ny, nz = X // bx, Y // by, Z // bz
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    return ((t // bt * nz + z // bz) * ny + y // by) * nx + x // bx


def nblocks(dims, block) -> int:
    return int(np.prod([d // b for d, b in zip(dims, block)]))


def block_inner(a: np.ndarray, b: np.ndarray, dims, block) -> np.ndarray:
    """[nblocks] array of sum over x in block b (all s, spin, colour) of conj(a) b."""
    blk = block_of_sites(dims, block)
    # sum over s, spin and colour first, then bin the 4D sites by block
    site = np.einsum("stzyxac,stzyxac->tzyx", a.conj(), b)
    return np.bincount(blk.ravel(), weights=site.real.ravel(), minlength=nblocks(dims, block)) + 1j * np.bincount(
        blk.ravel(), weights=site.imag.ravel(), minlength=nblocks(dims, block)
    )


def _spread(c: np.ndarray, dims, block) -> np.ndarray:
    """Per-block scalars c[nblocks] as a [T, Z, Y, X, 1, 1] array over the sites."""
    return c[block_of_sites(dims, block)][..., None, None]


def restrict(basis, v: np.ndarray, dims, block) -> np.ndarray:
    """c[b, k] = <phi_k^b, v>."""
    return np.stack([block_inner(phi, v, dims, block) for phi in basis], axis=1)


def prolong(basis, c: np.ndarray, dims, block) -> np.ndarray:
    """v = sum_k c[b(x), k] phi_k(x)."""
    out = np.zeros_like(basis[0])
    for k, phi in enumerate(basis):
        out = out + _spread(c[:, k], dims, block) * phi
    return out


def block_orthonormalize(vectors, dims, block):
    """CGS2 inside every block; returns (Q list, R [nblocks, n, n])."""
    n = len(vectors)
    nb = nblocks(dims, block)
    R = np.zeros((nb, n, n), dtype=np.complex128)
    Q = []
    for k in range(n):
        v = np.array(vectors[k], dtype=np.complex128)
        for _ in range(2):
            if not Q:
                break
            c = restrict(Q, v, dims, block)  # [nb, k]
            v = v - prolong(Q, c, dims, block)
            R[:, :k, k] += c
        nrm = np.sqrt(block_inner(v, v, dims, block).real)
        if np.any(nrm == 0):
            raise ValueError("a block of the vector set is linearly dependent")
        R[:, k, k] = nrm
        Q.append(v / _spread(nrm, dims, block))
    return Q, R
