"""Pins of the coarse-space oracle (chirality split, blocks, block orthonormalisation,
restriction and prolongation) against facts that do not come from the oracle itself:
hand-computed values, numpy's QR run block by block, and the algebraic identities the
Two level preconditioner section relies on (P_S a projector, Gamma_5 commuting with
restriction for a chirally split basis)."""

import numpy as np
import pytest

import synth
from oracle import coarse as C
from oracle import lattice as L

DIMS, LS, BLOCK = (4, 4, 4, 4), 4, (2, 2, 2, 2)


def even_vectors(n, seed, dims=DIMS, Ls=LS):
    return [L.on_parity(f, L.EVEN) for f in synth.gaussian_fermion_batch(dims, Ls, n, seed)]


def test_chiral_split_by_hand():
    """A unit upper-spin entry at s = 0: P+- put +-1/2 of it back at s = 0 and
    gamma_5 (+1 on upper spins) / 2 of it at the mirrored slice s = Ls - 1."""
    v = np.zeros((LS, 4, 4, 4, 4, 4, 3), dtype=np.complex128)
    v[0, 1, 2, 3, 0, 1, 2] = 2.0 + 4.0j  # s=0, t=1, z=2, y=3, x=0 (even), spin 1 (upper), colour 2
    v[2, 1, 2, 3, 0, 3, 0] = 1.0j  # s=2, spin 3 (lower): mirrored to s = 1 with gamma_5 = -1
    p, m = C.chiral_split(v)
    assert p[0, 1, 2, 3, 0, 1, 2] == 1.0 + 2.0j and p[LS - 1, 1, 2, 3, 0, 1, 2] == 1.0 + 2.0j
    assert m[0, 1, 2, 3, 0, 1, 2] == 1.0 + 2.0j and m[LS - 1, 1, 2, 3, 0, 1, 2] == -(1.0 + 2.0j)
    assert p[2, 1, 2, 3, 0, 3, 0] == 0.5j and p[1, 1, 2, 3, 0, 3, 0] == -0.5j
    assert m[2, 1, 2, 3, 0, 3, 0] == 0.5j and m[1, 1, 2, 3, 0, 3, 0] == 0.5j
    assert np.count_nonzero(p) == 4 and np.count_nonzero(m) == 4


def test_chiral_halves_are_complementary_orthogonal_eigenvectors():
    v, w = even_vectors(2, seed=11)
    p, m = C.chiral_split(v)
    assert np.max(np.abs(p + m - v)) < 1e-15 * np.max(np.abs(v))  # equal up to the rounding of the halves
    assert np.allclose(L.Gamma5(p), p, atol=1e-15) and np.allclose(L.Gamma5(m), -m, atol=1e-15)
    pw, mw = C.chiral_split(w)
    assert abs(L.inner(p, mw)) < 1e-12 * np.sqrt(L.norm2(p) * L.norm2(mw))


def test_block_numbering_by_hand():
    blk = C.block_of_sites((4, 2, 2, 2), (2, 1, 1, 2))
    assert C.nblocks((4, 2, 2, 2), (2, 1, 1, 2)) == 8
    # site x=3, y=1, z=0, t=1: block coordinates (1, 1, 0, 0) -> 1 + 2*1 + 4*0 + 8*0
    assert blk[1, 0, 1, 3] == 3
    assert blk[0, 1, 0, 2] == 1 + 0 + 4 * 1 + 0
    counts = np.bincount(blk.ravel())
    assert np.all(counts == 4)
    with pytest.raises(ValueError):
        C.block_of_sites((4, 4, 4, 4), (3, 2, 2, 2))


def _block_rows(v, blk, b):
    """Entries of v on the sites of block b, all s / spin / colour, as a flat vector."""
    return v[:, blk == b].ravel()


@pytest.mark.parametrize("block", [BLOCK, (4, 2, 4, 2), (4, 4, 4, 4)])
def test_block_orthonormalize_matches_numpy_qr_per_block(block):
    V = even_vectors(5, seed=12)
    V[3] = V[3] + 20.0 * V[1]  # an ill-conditioned set
    Q, R = C.block_orthonormalize(V, DIMS, block)
    blk = C.block_of_sites(DIMS, block)
    for b in range(C.nblocks(DIMS, block)):
        A = np.stack([_block_rows(v, blk, b) for v in V], axis=1)
        q, r = np.linalg.qr(A)
        ph = np.diag(r) / np.abs(np.diag(r))  # make diag(R) real positive
        q, r = q * ph[None, :], r * ph.conj()[:, None]
        got = np.stack([_block_rows(v, blk, b) for v in Q], axis=1)
        assert np.max(np.abs(got - q)) < 1e-12
        assert np.max(np.abs(R[b] - r)) < 1e-12 * np.max(np.abs(r))
    # odd sites stay zero
    for q in Q:
        assert not np.any(L.on_parity(q, L.ODD))


def test_block_orthonormal_and_triangular_reconstruction():
    V = even_vectors(4, seed=13)
    Q, R = C.block_orthonormalize(V, DIMS, BLOCK)
    nb = C.nblocks(DIMS, BLOCK)
    for j in range(4):
        for k in range(4):
            g = C.block_inner(Q[j], Q[k], DIMS, BLOCK)
            assert np.max(np.abs(g - (1.0 if j == k else 0.0))) < 1e-13
    assert np.all(np.abs(np.tril(R, -1)) == 0)
    assert np.all(np.abs(np.imag(np.diagonal(R, axis1=1, axis2=2))) == 0)
    assert np.all(np.real(np.diagonal(R, axis1=1, axis2=2)) > 0)
    for k in range(4):
        rebuilt = C.prolong(Q, R[:, :, k], DIMS, BLOCK)
        assert np.max(np.abs(rebuilt - V[k])) < 1e-12
    assert R.shape == (nb, 4, 4)


def test_restrict_and_prolong_are_adjoint():
    basis = even_vectors(3, seed=14)  # not orthonormal: adjointness holds for any basis
    v = even_vectors(1, seed=15)[0]
    rng = np.random.default_rng(3)
    nb = C.nblocks(DIMS, BLOCK)
    c = rng.standard_normal((nb, 3)) + 1j * rng.standard_normal((nb, 3))
    lhs = np.vdot(c, C.restrict(basis, v, DIMS, BLOCK))
    rhs = L.inner(C.prolong(basis, c, DIMS, BLOCK), v)
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def test_subspace_projector():
    """With a block-orthonormal basis, restrict o prolong = 1 on the coarse space and
    P_S = prolong o restrict is a Hermitian projector that keeps every phi_k^b."""
    Q, _ = C.block_orthonormalize(even_vectors(4, seed=16), DIMS, BLOCK)
    rng = np.random.default_rng(4)
    nb = C.nblocks(DIMS, BLOCK)
    c = rng.standard_normal((nb, 4)) + 1j * rng.standard_normal((nb, 4))
    assert np.max(np.abs(C.restrict(Q, C.prolong(Q, c, DIMS, BLOCK), DIMS, BLOCK) - c)) < 1e-13

    def PS(v):
        return C.prolong(Q, C.restrict(Q, v, DIMS, BLOCK), DIMS, BLOCK)

    u, w = even_vectors(2, seed=17)
    assert np.max(np.abs(PS(PS(u)) - PS(u))) < 1e-12
    assert abs(L.inner(u, PS(w)) - L.inner(PS(u), w)) < 1e-12 * np.sqrt(L.norm2(u) * L.norm2(w))
    for q in Q:
        assert np.max(np.abs(PS(q) - q)) < 1e-13
    # a vector orthogonal to every block's span is annihilated
    r = u - PS(u)
    assert np.max(np.abs(C.restrict(Q, r, DIMS, BLOCK))) < 1e-12


def test_gamma5_commutes_with_restriction_for_a_chiral_basis():
    """Split basis [P+ phi_0, P- phi_0, P+ phi_1, ...] block-orthonormalised stays chiral,
    so restricting Gamma_5 v equals restricting v and flipping the sign of the P- rows."""
    raw = even_vectors(3, seed=18)
    split = [h for v in raw for h in C.chiral_split(v)]
    Q, _ = C.block_orthonormalize(split, DIMS, BLOCK)
    for k, q in enumerate(Q):
        assert np.max(np.abs(L.Gamma5(q) - (1 if k % 2 == 0 else -1) * q)) < 1e-13
    v = even_vectors(1, seed=19)[0]
    sign = np.array([1 if k % 2 == 0 else -1 for k in range(len(Q))])
    lhs = C.restrict(Q, L.Gamma5(v), DIMS, BLOCK)
    rhs = C.restrict(Q, v, DIMS, BLOCK) * sign[None, :]
    assert np.max(np.abs(lhs - rhs)) < 1e-12


def test_block_orthonormalize_stays_orthogonal_when_ill_conditioned():
    """kappa ~ 1e6 inside every block: one Gram-Schmidt pass would lose orthogonality at
    the kappa^2 eps ~ 1e-4 level; the second pass restores it to rounding."""
    V = even_vectors(4, seed=20)
    V[2] = V[0] + 1e-6 * V[2]
    Q, R = C.block_orthonormalize(V, DIMS, BLOCK)
    for j in range(4):
        for k in range(4):
            g = C.block_inner(Q[j], Q[k], DIMS, BLOCK)
            assert np.max(np.abs(g - (1.0 if j == k else 0.0))) < 1e-13
    for k in range(4):
        assert np.max(np.abs(C.prolong(Q, R[:, :, k], DIMS, BLOCK) - V[k])) < 1e-12
