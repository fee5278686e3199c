"""The pseudofermion action S = phi^dag (M_pc^dag M_pc)^{-1} phi through
torch.autograd (PseudofermionAction: dwf_cg and dwf_dot forward, dwf_mpc and
the dwf_force adjoint kernel backward) against the oracle, and dwf_dot
against plain sums.

* S and U.grad against the oracle's action and gradient (a dense solve at
  2^4 x 4, CG to 1e-14 at 4^4 x 8), within 1e-10.  The GPU's CG stops at
  1e-13, so its X differs from the exact solve by at most kappa * 1e-13
  relative (kappa = lambda_max / lambda_min of M_pc^dag M_pc, about 1.4e3 on
  the 4^4 x 8 links), which bounds both differences below 1e-10.
* The same gradient given the GPU's own X (deterministic: a second solve is
  bitwise identical) against the oracle's outer-product formula, within 1e-12.
* Central finite differences of the oracle's dense action on 16 random links
  (eps = 1e-5) against Re sum conj(U.grad) E.
"""

import numpy as np
import pytest

import synth
from oracle import force as F, lattice as L
from tests.gpu_util import M5, MF, dev_tensor, make_operator, pack, rel, unpack

pytestmark = pytest.mark.gpu

EVEN = 0
F64, F32, F16S = 0, 1, 2


@pytest.mark.parametrize("prec", [F64, F32, F16S])
def test_dot_against_numpy(prec):
    import torch

    dims, Ls = (4, 4, 6, 4), 6
    # max_nrhs = max_cg_rhs = 1: the handle's reduction scratch holds one rhs, so
    # three rhs go through the chunked path
    op, _ = make_operator(dims, Ls, prec=prec, max_nrhs=1, max_cg_rhs=1)
    a = synth.gaussian_fermion_batch(dims, Ls, 3, seed=50)
    b = synth.gaussian_fermion_batch(dims, Ls, 3, seed=51)
    pa, pb = pack(op, a, EVEN), pack(op, b, EVEN)
    sa, sb = unpack(op, pa, 3, EVEN), unpack(op, pb, 3, EVEN)  # the stored values
    got = op.dot(pa, pb, 3).cpu().numpy()
    exp = np.array([np.vdot(sa[k].ravel(), sb[k].ravel()) for k in range(3)])
    assert np.max(np.abs(got - exp) / np.abs(exp)) < 1e-13
    again = op.dot(pa, pb, 3)
    torch.cuda.synchronize()
    assert np.array_equal(again.cpu().numpy(), got)


def _action(dims, Ls, seed_links=0, seed_phi=1, eps=0.3):
    import paper_2103_05034_amd as dwf

    U = synth.gauge_links(dims, eps=eps, seed=seed_links)
    phi = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=seed_phi), EVEN)
    op, _ = make_operator(dims, Ls, U=U, max_nrhs=1, max_cg_rhs=1)
    Ut = dev_tensor(U).requires_grad_(True)
    S = dwf.PseudofermionAction.apply(Ut, dev_tensor(phi), op, 1e-13, 100000)
    S.backward()
    return U, phi, op, float(S.item()), Ut.grad.cpu().numpy()


@pytest.mark.parametrize("dims,Ls,dense", [((2, 2, 2, 2), 4, True), ((4, 4, 4, 4), 8, False)])
def test_action_and_link_gradient_against_oracle(dims, Ls, dense):
    U, phi, op, S, G = _action(dims, Ls)
    So, _ = F.action(U, phi, M5, MF, tol=1e-14, dense=dense)
    Go, _ = F.force(U, phi, M5, MF, tol=1e-14, dense=dense)
    assert abs(S - So) / abs(So) < 1e-10
    assert rel(G, Go) < 1e-10
    # the chain given the GPU's own X
    x = op.new_field(1)
    op.cg(pack(op, phi[None], EVEN), x, 1, tol=1e-13, maxiter=100000)
    Xg = unpack(op, x, 1, EVEN)[0]
    assert abs(S - np.vdot(phi.ravel(), Xg.ravel()).real) / abs(S) < 1e-13
    Gx = F.link_gradient(U, Xg, L.mpc(U, Xg, M5, MF), M5, MF)
    assert rel(G, Gx) < 1e-12


def test_link_gradient_against_finite_differences():
    """16 random links of 2^4 x Ls 4; the finite differences use exact (dense) solves,
    so their error is O(eps^2) and rounding, far below the 1e-6 bar."""
    dims, Ls = (2, 2, 2, 2), 4
    U, phi, _, _, G = _action(dims, Ls)
    links = synth.random_link_sites(dims, 16, seed=52)
    rng = np.random.default_rng(53)
    eps = 1e-5
    for (t, z, y, x, mu) in links:
        E = np.zeros_like(U)
        E[t, z, y, x, mu] = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        Sp, _ = F.action(U + eps * E, phi, M5, MF, dense=True)
        Sm, _ = F.action(U - eps * E, phi, M5, MF, dense=True)
        fd = (Sp - Sm) / (2 * eps)
        an = float(np.sum(np.conj(G) * E).real)
        assert abs(fd - an) < 1e-6 * max(abs(an), 1e-2 * np.abs(G).max())


def test_gradient_scales_with_grad_output_and_phi_gradient():
    """d(c S)/dU = c dS/dU through the chain rule, and dS/dphi = 2 X on the even sites."""
    import torch

    import paper_2103_05034_amd as dwf

    dims, Ls = (2, 2, 2, 2), 4
    U = synth.gauge_links(dims, eps=0.3, seed=0)
    phi = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=1), EVEN)
    op, _ = make_operator(dims, Ls, U=U, max_nrhs=1, max_cg_rhs=1)
    Ut = dev_tensor(U).requires_grad_(True)
    pt = dev_tensor(phi).requires_grad_(True)
    S = dwf.PseudofermionAction.apply(Ut, pt, op, 1e-13, 100000)
    (3.0 * S).backward()
    Go, gphi = F.force(U, phi, M5, MF, dense=True)
    assert rel(Ut.grad.cpu().numpy(), 3.0 * Go) < 1e-10
    assert rel(pt.grad.cpu().numpy(), 3.0 * gphi) < 1e-10
    torch.cuda.synchronize()
