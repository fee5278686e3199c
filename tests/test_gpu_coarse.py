"""GPU parity of the coarse-space transfer (chirality split, block orthonormalisation,
restriction, prolongation) against the oracle, through the C ABI.

The oracle runs on the values the GPU actually holds (the packed input unpacked
again), so restriction differs only by the order of FP64 summation whatever the
storage precision; prolongation and orthonormalisation round their outputs to
the storage precision.  At the paper's 16^3x32, Ls=16 size the checks are the
size-independent identities of an orthonormal blocked basis."""

import numpy as np
import pytest

import synth
from oracle import coarse as C
from oracle import lattice as L
from tests.gpu_util import make_operator, pack, unpack

pytestmark = pytest.mark.gpu

F64, F32, F16S = 0, 1, 2
EVEN = 0
C1 = ((4, 4, 4, 4), 8)


def even_fields(dims, Ls, n, seed):
    return np.stack([L.on_parity(f, L.EVEN) for f in synth.gaussian_fermion_batch(dims, Ls, n, seed)])


def coarse_host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


def relmax(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.mark.parametrize("prec,tol", [(F64, 0.0), (F32, 1e-7), (F16S, 2e-3)])
def test_chiral_split(prec, tol):
    dims, Ls = C1
    op, _ = make_operator(dims, Ls, prec=prec, max_nrhs=4)
    v = even_fields(dims, Ls, 2, seed=40)
    buf = pack(op, v, EVEN)
    held = unpack(op, buf, 2, EVEN)
    out = op.chiral_split(buf, 2)
    got = unpack(op, out, 4, EVEN)
    for k in range(2):
        p, m = C.chiral_split(held[k])
        if prec == F64:
            assert np.array_equal(got[2 * k], p) and np.array_equal(got[2 * k + 1], m)
        else:
            assert relmax(got[2 * k], p) <= tol and relmax(got[2 * k + 1], m) <= tol


@pytest.mark.parametrize("prec", [F64, F32, F16S])
@pytest.mark.parametrize("block", [(2, 2, 2, 2), (4, 2, 4, 2), (2, 4, 2, 1)])
def test_restrict_and_prolong(prec, block):
    import torch

    dims, Ls = C1
    op, _ = make_operator(dims, Ls, prec=prec, max_nrhs=8)
    nb = op.set_blocks(block)
    assert nb == C.nblocks(dims, block)
    nvec, nrhs = 5, 3
    basis = pack(op, even_fields(dims, Ls, nvec, seed=41), EVEN)
    v = pack(op, even_fields(dims, Ls, nrhs, seed=42), EVEN)
    B = unpack(op, basis, nvec, EVEN)
    V = unpack(op, v, nrhs, EVEN)
    c = coarse_host(op.restrict(basis, nvec, v, nrhs))
    assert c.shape == (nrhs, nb, nvec)
    for r in range(nrhs):
        assert relmax(c[r], C.restrict(list(B), V[r], dims, block)) < 1e-13
    rng = np.random.default_rng(5)
    cc = rng.standard_normal((nrhs, nb, nvec)) + 1j * rng.standard_normal((nrhs, nb, nvec))
    out = op.prolong(basis, nvec, torch.from_numpy(cc).cuda(), nrhs)
    got = unpack(op, out, nrhs, EVEN)
    tol = {F64: 1e-14, F32: 2e-7, F16S: 2e-3}[prec]
    for r in range(nrhs):
        assert relmax(got[r], C.prolong(list(B), cc[r], dims, block)) < tol


@pytest.mark.parametrize("block", [(2, 2, 2, 2), (4, 2, 4, 2)])
def test_block_orthonormalize_f64(block):
    dims, Ls = C1
    op, _ = make_operator(dims, Ls, prec=F64, max_nrhs=8)
    op.set_blocks(block)
    V = even_fields(dims, Ls, 6, seed=43)
    V[4] = V[4] + 25.0 * V[1]
    buf = pack(op, V, EVEN)
    op.block_orthonormalize(buf, 6)
    Q = unpack(op, buf, 6, EVEN)
    Qo, _ = C.block_orthonormalize(list(V), dims, block)
    for k in range(6):
        assert relmax(Q[k], Qo[k]) < 1e-12
        assert not np.any(L.on_parity(Q[k], L.ODD))


def test_block_orthonormalize_ill_conditioned_and_breakdown():
    import paper_2103_05034_amd as dwf

    dims, Ls = C1
    block = (2, 2, 2, 2)
    op, _ = make_operator(dims, Ls, prec=F64, max_nrhs=8)
    op.set_blocks(block)
    V = even_fields(dims, Ls, 4, seed=44)
    V[2] = V[0] + 1e-6 * V[2]  # kappa ~ 1e6 in every block
    buf = pack(op, V, EVEN)
    op.block_orthonormalize(buf, 4)
    Q = unpack(op, buf, 4, EVEN)
    for j in range(4):
        for k in range(4):
            g = C.block_inner(Q[j], Q[k], dims, block)
            assert np.max(np.abs(g - (1.0 if j == k else 0.0))) < 1e-13
    V[3] = V[1]  # dependent in every block
    buf = pack(op, V, EVEN)
    with pytest.raises(dwf.DWFError) as e:
        op.block_orthonormalize(buf, 4)
    assert e.value.code == dwf.DWF_EBREAKDOWN


@pytest.mark.parametrize("prec,tol", [(F32, 1e-5), (F16S, 3e-3)])
def test_block_orthonormalize_low_precision(prec, tol):
    dims, Ls = C1
    block = (2, 2, 2, 2)
    op, _ = make_operator(dims, Ls, prec=prec, max_nrhs=8)
    op.set_blocks(block)
    buf = pack(op, even_fields(dims, Ls, 5, seed=45), EVEN)
    held = unpack(op, buf, 5, EVEN)
    op.block_orthonormalize(buf, 5)
    Q = unpack(op, buf, 5, EVEN)
    Qo, _ = C.block_orthonormalize(list(held), dims, block)
    for k in range(5):
        assert relmax(Q[k], Qo[k]) < tol
    for j in range(5):
        for k in range(5):
            g = C.block_inner(Q[j], Q[k], dims, block)
            assert np.max(np.abs(g - (1.0 if j == k else 0.0))) < 4 * tol


def test_gamma5_commutes_with_gpu_restriction():
    """GPU chirality split + block orthonormalisation keeps each basis vector chiral, so
    restricting Gamma_5 v flips the sign of the (1 - Gamma_5) rows."""
    dims, Ls = C1
    block = (2, 2, 2, 2)
    op, _ = make_operator(dims, Ls, prec=F64, max_nrhs=8)
    op.set_blocks(block)
    raw = pack(op, even_fields(dims, Ls, 3, seed=46), EVEN)
    basis = op.chiral_split(raw, 3)
    op.block_orthonormalize(basis, 6)
    v = even_fields(dims, Ls, 1, seed=47)
    c = coarse_host(op.restrict(basis, 6, pack(op, v, EVEN), 1))[0]
    cg = coarse_host(op.restrict(basis, 6, pack(op, L.Gamma5(v[0])[None], EVEN), 1))[0]
    sign = np.array([1, -1] * 3)
    assert np.max(np.abs(cg - c * sign[None, :])) < 1e-12 * np.max(np.abs(c))


@pytest.mark.parametrize("block", [(2, 2, 2, 2), (4, 2, 4, 2)])
def test_fullsize_orthonormal_basis_identities(block):
    """16^3x32, Ls=16, FP32 (the Algorithm A / B blocks): after orthonormalisation
    restrict(Q, Q_k) is the k-th unit vector in every block, and restrict o prolong is
    the identity on random coarse vectors."""
    import torch

    dims, Ls = (16, 16, 16, 32), 16
    nvec = 8
    op, _ = make_operator(dims, Ls, eps=0.2, prec=F32, max_nrhs=nvec, max_cg_rhs=0)
    nb = op.set_blocks(block)
    basis = op.new_field(nvec)
    for k in range(nvec):
        op.pack(torch.from_numpy(synth.gaussian_fermion_batch(dims, Ls, 1, 100 + k)).cuda(), EVEN,
                out=basis[k * op.field_bytes(1) : (k + 1) * op.field_bytes(1)])
    op.block_orthonormalize(basis, nvec)
    G = coarse_host(op.restrict(basis, nvec, basis, nvec))  # [r][b][k] = <Q_k, Q_r>
    eye = np.eye(nvec)[:, None, :]
    assert np.max(np.abs(G - eye)) < 2e-6
    rng = np.random.default_rng(6)
    cc = rng.standard_normal((1, nb, nvec)) + 1j * rng.standard_normal((1, nb, nvec))
    back = coarse_host(op.restrict(basis, nvec, op.prolong(basis, nvec, torch.from_numpy(cc).cuda(), 1), 1))
    assert relmax(back, cc) < 1e-6


def test_block_orthonormalize_max_nvec():
    """nvec = 64, the largest basis: the Gram, Cholesky and update kernels hold a full
    64 x 64 complex matrix per block in LDS."""
    dims, Ls = C1
    block = (2, 2, 2, 2)
    op, _ = make_operator(dims, Ls, prec=F64, max_nrhs=64, max_cg_rhs=0)
    op.set_blocks(block)
    V = even_fields(dims, Ls, 64, seed=48)
    buf = pack(op, V, EVEN)
    op.block_orthonormalize(buf, 64)
    G = coarse_host(op.restrict(buf, 64, buf, 64))
    assert np.max(np.abs(G - np.eye(64)[:, None, :])) < 1e-12
    Q = unpack(op, buf, 64, EVEN)
    Qo, _ = C.block_orthonormalize(list(V), dims, block)
    assert max(relmax(Q[k], Qo[k]) for k in range(64)) < 1e-10


@pytest.mark.parametrize("both,block", [(False, (4, 4, 4, 2)), (True, (4, 2, 4, 2))])
def test_blocks_of_1024_5d_sites(both, block):
    """Ls = 16 with 64 sites per block (even sites of 4x4x4x2, or all sites of the
    Algorithm A block 4x2x4x2): 1024 5D sites, two per lane of the per-block kernels."""
    import torch

    dims, Ls = (8, 4, 8, 4), 16
    parity = 2 if both else EVEN
    op, _ = make_operator(dims, Ls, prec=F64, max_nrhs=8, max_cg_rhs=2)
    nb = op.set_blocks(block, both=both)
    assert nb == C.nblocks(dims, block)
    raw = synth.gaussian_fermion_batch(dims, Ls, 3, 50)
    if not both:
        raw = np.stack([L.on_parity(f, L.EVEN) for f in raw])
    split = unpack(op, op.chiral_split(pack(op, raw, parity), 3), 6, parity)
    basis = pack(op, split, parity)
    op.block_orthonormalize(basis, 6)
    Q = unpack(op, basis, 6, parity)
    Qo, _ = C.block_orthonormalize(list(split), dims, block)
    for k in range(6):
        assert relmax(Q[k], Qo[k]) < 1e-12
    W = synth.gaussian_fermion_batch(dims, Ls, 3, 51)
    if not both:
        W = np.stack([L.on_parity(f, L.EVEN) for f in W])
    c = coarse_host(op.restrict(basis, 6, pack(op, W, parity), 3))
    for r in range(3):
        assert relmax(c[r], C.restrict(list(Q), W[r], dims, block)) < 1e-13
    cc = np.random.default_rng(52).standard_normal((2, nb, 6)) + 0.5j
    got = unpack(op, op.prolong(basis, 6, torch.from_numpy(cc).cuda(), 2), 2, parity)
    for r in range(2):
        assert relmax(got[r], C.prolong(list(Q), cc[r], dims, block)) < 1e-14
