"""GPU parity of the pseudofermion force: the link-gradient kernel given
(X, Y) against the oracle's outer products, and the whole GPU chain
(CG + M_pc + force) against central differences of the action computed with
the resolvent identity S(U+) - S(U-) = X+^dag (A(U-) - A(U+)) X-."""

import numpy as np
import pytest

import synth
from oracle import force as F, lattice as L
from tests.gpu_util import M5, MF, dev_tensor, make_operator, pack, rel, unpack

pytestmark = pytest.mark.gpu

EVEN = 0


# Ls = 1, 2, 4, 8, 16, 32: every width of the in-register sum over s (the lanes of a site);
# Ls = 5, 12: the LDS sum; Ls = 72: one workgroup lane per (site, s) looping over directions
@pytest.mark.parametrize("dims,Ls", [((2, 2, 2, 2), 4), ((4, 4, 6, 8), 5), ((4, 4, 4, 4), 8), ((2, 2, 2, 2), 1),
                                     ((2, 2, 4, 2), 2), ((2, 2, 2, 4), 16), ((2, 4, 2, 2), 32), ((2, 2, 2, 2), 12),
                                     ((2, 2, 2, 2), 72)])
def test_force_kernel_given_X_Y(dims, Ls):
    op, U = make_operator(dims, Ls, eps=0.5, seed=30)
    X = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=31), EVEN)
    Y = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=32), EVEN)
    G = op.force(pack(op, X[None], EVEN), pack(op, Y[None], EVEN)).cpu().numpy()
    Go = F.link_gradient(U, X, Y, M5, MF)
    assert rel(G, Go) < 1e-13


@pytest.mark.parametrize("order", [1, 2, (1, 2, 4)])
@pytest.mark.parametrize("Ls", [4, 5])
def test_force_kernel_traversal_order(order, Ls):
    """The force kernel walks the sites in the handle's traversal order (XCD octants,
    XCD t-slabs); the order only permutes which workgroup forms a site's links, so
    the gradient is bitwise the lexicographic one (Ls = 4: in-register sums over s,
    Ls = 5: the LDS sums)."""
    import torch

    dims = (4, 4, 4, 8)
    op, U = make_operator(dims, Ls, eps=0.5, seed=33)
    X = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=34), EVEN)
    Y = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=35), EVEN)
    Xd, Yd = pack(op, X[None], EVEN), pack(op, Y[None], EVEN)
    G0 = op.force(Xd, Yd)
    if isinstance(order, tuple):
        op.set_order_box(*order)
    else:
        op.set_order(order)
    G1 = op.force(Xd, Yd)
    torch.cuda.synchronize()
    assert torch.equal(G0, G1)
    assert rel(G1.cpu().numpy(), F.link_gradient(U, X, Y, M5, MF)) < 1e-13


def _gpu_X(op, phi_dev, tol=1e-13):
    x = op.new_field(1)
    op.cg(phi_dev, x, 1, tol=tol, maxiter=20000, allow_noconv=True)
    return x


def test_force_vs_finite_differences_resolvent():
    """A small version of the 8^3 x 16, Ls = 12 force check: 16 random links, eps = 1e-5."""
    dims, Ls = (4, 4, 4, 4), 6
    U = synth.gauge_links(dims, eps=0.2, seed=0)
    phi = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=3), EVEN)
    op, _ = make_operator(dims, Ls, U=U)
    phi_d = pack(op, phi[None], EVEN)
    X = _gpu_X(op, phi_d)
    Y = op.new_field(1)
    op.mpc(X, Y, 1, False)
    G = op.force(X, Y).cpu().numpy()
    links = synth.random_link_sites(dims, 16, seed=4)
    rng = np.random.default_rng(5)
    eps = 1e-5
    for (t, z, y, x, mu) in links:
        E = np.zeros_like(U)
        E[t, z, y, x, mu] = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        ops = []
        Xs = []
        for sgn in (+1, -1):
            o, _ = make_operator(dims, Ls, U=U + sgn * eps * E)
            Xs.append(unpack(o, _gpu_X(o, pack(o, phi[None], EVEN)), 1, EVEN)[0])
            ops.append(o)
        Um = U - eps * E
        Up = U + eps * E
        diff = L.inner(Xs[0], L.mpcdagmpc(Um, Xs[1], M5, MF) - L.mpcdagmpc(Up, Xs[1], M5, MF)).real
        fd = diff / (2 * eps)
        an = float(np.sum(np.conj(G) * E).real)
        assert abs(fd - an) < 1e-6 * max(abs(an), 1e-2 * np.abs(G).max())


@pytest.mark.parametrize("dims,Ls", [((2, 2, 2, 2), 4), ((4, 4, 6, 8), 5)])
def test_lie_force(dims, Ls):
    """dwf_lie_force on the GPU gradient against the oracle's Lie-algebra force of the
    oracle gradient (the oracle's form is pinned by central differences along
    exp(i eps T^a) U), and the same map applied to the GPU gradient itself."""
    import torch

    op, U = make_operator(dims, Ls, eps=0.5, seed=36)
    X = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=37), EVEN)
    Y = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=38), EVEN)
    G = op.force(pack(op, X[None], EVEN), pack(op, Y[None], EVEN))
    Ud = torch.from_numpy(U).to(G.device)
    Fd = op.lie_force(Ud, G)
    torch.cuda.synchronize()
    Fg = Fd.cpu().numpy()
    assert Fg.shape == U.shape[:5] + (8,)
    assert rel(Fg, F.lie_force(U, G.cpu().numpy())) < 1e-14
    assert rel(Fg, F.lie_force(U, F.link_gradient(U, X, Y, M5, MF))) < 1e-13
