"""Parity at the workloads' full sizes and in the launch configurations the
benchmark times.  The oracle cannot process these lattices whole in a test,
so outputs are sampled: the value at a site depends only on inputs within a
fixed taxicab radius (1 for D_hop, 2 for M_pc, 4 for M_pc^dag M_pc), and the
oracle evaluated on a periodic patch that contains that radius reproduces it
exactly at the patch centre.  Hermiticity of the normal operator is checked
on the whole lattice.
"""

import numpy as np
import pytest

import synth
from oracle import force as F, lattice as L
from tests.gpu_util import (
    dev_tensor,
    make_operator,
    pack,
    patch_indices,
    rel,
    sample_sites,
    take_patch,
    unpack,
)

pytestmark = pytest.mark.gpu
F64, F32, F16S = 0, 1, 2
EVEN, ODD = 0, 1


def oracle_at_sites(fn, U, psi, dims, sites, radius):
    """fn(U_patch, psi_patch) evaluated by the oracle, read at each sampled site."""
    vals = []
    for c in sites:
        idx, (lx, ly, lz, lt) = patch_indices(dims, c, radius)
        Up = take_patch(U, idx, -4)  # links [T][Z][Y][X][mu][a][b]: x is 4th from the end
        pp = take_patch(psi, idx, -3)
        vals.append(fn(Up, pp)[:, lt, lz, ly, lx])
    return np.stack(vals)


def gpu_at_sites(field, sites):
    return np.stack([field[:, t, z, y, x] for (x, y, z, t) in sites])


def _workload(dims, Ls, eps, prec, nrhs=1, mf=0.01, seed_src=1, max_cg_rhs=0):
    op, U = make_operator(dims, Ls, eps=eps, seed=0, prec=prec, max_nrhs=nrhs, max_cg_rhs=max_cg_rhs, mf=mf)
    op.autotune(nrhs, 2)
    return op, U


@pytest.mark.parametrize("order", [0, 1, 2])
def test_rb_workload_fp64_sampled(order):
    """16^3 x 32, Ls = 16, FP64 (the red-black solve workload): D_hop, M_pc and
    M_pc^dag M_pc at sampled sites, in the autotuned launch shape."""
    dims, Ls, mf = (16, 16, 16, 32), 16, 0.01
    op, U = _workload(dims, Ls, 0.2, F64)
    op.set_order(order)
    psi = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=1), EVEN)
    v = pack(op, psi[None], EVEN)
    sites_e = sample_sites(dims, 3, seed=7, parity=EVEN)
    sites_o = sample_sites(dims, 3, seed=8, parity=ODD)
    w = op.new_field(1)
    op.dhop(v, w, ODD, 1, False)
    got = gpu_at_sites(unpack(op, w, 1, ODD)[0], sites_o)
    exp = oracle_at_sites(lambda u, p: L.dhop(u, p), U, psi, dims, sites_o, 1)
    assert rel(got, exp) < 1e-13
    op.mpc(v, w, 1, False)
    got = gpu_at_sites(unpack(op, w, 1, EVEN)[0], sites_e)
    exp = oracle_at_sites(lambda u, p: L.mpc(u, L.on_parity(p, EVEN), 1.8, mf), U, psi, dims, sites_e, 2)
    assert rel(got, exp) < 1e-13
    op.mpcdagmpc(v, w, 1)
    got = gpu_at_sites(unpack(op, w, 1, EVEN)[0], sites_e[:2])
    exp = oracle_at_sites(lambda u, p: L.mpcdagmpc(u, L.on_parity(p, EVEN), 1.8, mf), U, psi, dims, sites_e[:2], 4)
    assert rel(got, exp) < 1e-13


def test_rb_workload_hermiticity_whole_lattice():
    import torch

    dims, Ls = (16, 16, 16, 32), 16
    op, U = _workload(dims, Ls, 0.2, F64, nrhs=2)
    f = synth.gaussian_fermion_batch(dims, Ls, 2, seed=3)
    v = pack(op, np.stack([L.on_parity(x, EVEN) for x in f]), EVEN)
    w = op.new_field(2)
    op.mpcdagmpc(v, w, 2)
    torch.cuda.synchronize()
    fb = op.field_bytes(1)
    c = lambda t, k: t[k * fb : (k + 1) * fb].view(torch.complex128)
    # packed layouts hold the same entries in another order: inner products are layout-free
    a = torch.vdot(c(v, 0), c(w, 1)).item()
    b = torch.vdot(c(w, 0), c(v, 1)).item()
    assert abs(a - b) < 1e-12 * abs(a)
    n = torch.vdot(c(v, 0), c(w, 0)).item()
    assert abs(n.imag) < 1e-12 * abs(n.real) and n.real > 0


def test_batched_workload_fp32_40rhs_sampled():
    """The batched filter's launch: 40 complex64 rhs per launch at 16^3 x 32, Ls = 16."""
    dims, Ls, nrhs = (16, 16, 16, 32), 16, 40
    op, U = _workload(dims, Ls, 0.2, F32, nrhs=nrhs)
    fb = op.field_bytes(1)
    v = op.new_field(nrhs)  # zero fields except the three sampled rhs
    picks = {}
    for k in (0, 23, 39):
        picks[k] = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=100 + k), EVEN)
        op.pack(dev_tensor(picks[k][None]), EVEN, out=v[k * fb : (k + 1) * fb])
    w = op.new_field(nrhs)
    op.mpcdagmpc(v, w, nrhs)
    sites = sample_sites(dims, 2, seed=9, parity=EVEN)
    for k, nat in picks.items():
        src = unpack(op, v[k * fb : (k + 1) * fb], 1, EVEN)[0]  # the FP32 values the kernel read
        got = gpu_at_sites(unpack(op, w[k * fb : (k + 1) * fb], 1, EVEN)[0], sites)
        exp = oracle_at_sites(lambda u, p: L.mpcdagmpc(u, L.on_parity(p, EVEN), 1.8, 0.01), U, src, dims, sites, 4)
        assert rel(got, exp) < 1e-6


def test_mixed_workload_sampled():
    """24^3 x 48, Ls = 24, mf = 0.00078: FP64 and FP16 + scale M_pc^dag M_pc at sampled sites."""
    dims, Ls, mf = (24, 24, 24, 48), 24, 0.00078
    psi = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=5), EVEN)
    for prec, tol, nsites in ((F64, 1e-13, 2), (F16S, 3e-3, 1)):
        sites = sample_sites(dims, nsites, seed=10, parity=EVEN)
        op, U = _workload(dims, Ls, 0.15, prec, mf=mf)
        v = pack(op, psi[None], EVEN)
        src = unpack(op, v, 1, EVEN)[0]
        w = op.new_field(1)
        op.mpcdagmpc(v, w, 1)
        got = gpu_at_sites(unpack(op, w, 1, EVEN)[0], sites)
        exp = oracle_at_sites(lambda u, p: L.mpcdagmpc(u, L.on_parity(p, EVEN), 1.8, mf), U, src, dims, sites, 4)
        assert rel(got, exp) < tol
        op.close()
        del op, v, w
        import torch

        torch.cuda.empty_cache()


def test_force_workload_c4():
    """8^3 x 16, Ls = 12, FP64: the force kernel against the oracle's gradient on the
    whole lattice (given X, Y), and the full GPU chain (CG + M_pc + force) against
    central differences of the action on 64 random links via the resolvent identity."""
    import torch

    dims, Ls = (8, 8, 8, 16), 12
    U = synth.gauge_links(dims, eps=0.2, seed=0)
    op, _ = make_operator(dims, Ls, U=U, max_nrhs=1, max_cg_rhs=1)
    X = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=31), EVEN)
    Y = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=32), EVEN)
    G = op.force(pack(op, X[None], EVEN), pack(op, Y[None], EVEN)).cpu().numpy()
    assert rel(G, F.link_gradient(U, X, Y, 1.8, 0.01)) < 1e-13

    phi = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=3), EVEN)

    def solve(o):
        x = o.new_field(1)
        o.cg(pack(o, phi[None], EVEN), x, 1, tol=1e-13, maxiter=50000, allow_noconv=True)
        return x

    Xd = solve(op)
    Yd = op.new_field(1)
    op.mpc(Xd, Yd, 1, False)
    G = op.force(Xd, Yd).cpu().numpy()
    eps = 1e-5
    rng = np.random.default_rng(4)
    links = synth.random_link_sites(dims, 64, seed=4)
    fb = op.field_bytes(1)
    for (t, z, y, x, mu) in links:
        E = np.zeros_like(U)
        E[t, z, y, x, mu] = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        op_p, _ = make_operator(dims, Ls, U=U + eps * E, max_nrhs=1, max_cg_rhs=1)
        op_m, _ = make_operator(dims, Ls, U=U - eps * E, max_nrhs=1, max_cg_rhs=1)
        Xp, Xm = solve(op_p), solve(op_m)
        Am, Ap = op.new_field(1), op.new_field(1)
        op_m.mpcdagmpc(Xm, Am, 1)
        op_p.mpcdagmpc(Xm, Ap, 1)
        torch.cuda.synchronize()
        cv = lambda t_: t_.view(torch.complex128)
        diff = torch.vdot(cv(Xp), cv(Am) - cv(Ap)).real.item()
        fd = diff / (2 * eps)
        an = float(np.sum(np.conj(G) * E).real)
        assert abs(fd - an) < 1e-6 * max(abs(an), 1e-2 * np.abs(G).max()), (t, z, y, x, mu, fd, an)
        op_p.close()
        op_m.close()


@pytest.mark.parametrize("prec", [F32, F16S])
def test_mixed_workload_field_solve_sampled(prec):
    """24^3 x 48, Ls = 24, mf = 0.00078: the mixed workload's solve with the search direction
    stored in FP32 or in FP16 + per-site scale (FP32 operator intermediates, FP64 reliable
    updates) reaches an FP64 true residual of 1e-10: measured by the solver, by the FP64
    operator of the library over the whole lattice, and by the oracle's M_pc^dag M_pc applied
    to the GPU solution on patches around sampled sites, which reproduces b there."""
    import torch

    dims, Ls, mf = (24, 24, 24, 48), 24, 0.00078
    U = synth.gauge_links(dims, eps=0.15, seed=0)
    psi = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=5), EVEN)
    op64, _ = make_operator(dims, Ls, prec=F64, mf=mf, U=U, max_nrhs=1, max_cg_rhs=0)
    b = pack(op64, psi[None], EVEN)
    opl, _ = make_operator(dims, Ls, prec=prec, mf=mf, U=U, max_nrhs=1, max_cg_rhs=1)
    x = opl.new_field(1, prec=F64)
    code, iters, res = opl.cg(b, x, 1, tol=1e-10, maxiter=5000)
    print(f"prec {prec}: {iters[0]} iterations, true residual {res[0]:.3e}", flush=True)
    assert code == 0 and res[0] < 1.5e-10
    opl.close()
    del opl
    torch.cuda.empty_cache()
    Ax = op64.new_field(1)
    op64.mpcdagmpc(x, Ax, 1)
    torch.cuda.synchronize()
    cv = lambda t_: t_.view(torch.complex128)  # noqa: E731
    whole = (torch.linalg.vector_norm(cv(b) - cv(Ax)) / torch.linalg.vector_norm(cv(b))).item()
    assert whole < 1.5e-10
    X = unpack(op64, x, 1, EVEN)[0]
    sites = sample_sites(dims, 2, seed=11, parity=EVEN)
    Axs = oracle_at_sites(lambda u, p: L.mpcdagmpc(u, L.on_parity(p, EVEN), 1.8, mf), U, X, dims, sites, 4)
    bs = gpu_at_sites(psi, sites)
    assert rel(Axs, bs) < 1e-7


def test_rb_workload_every_bench_launch_shape():
    """16^3 x 32, Ls = 16, FP64: the launch shapes bench.py chooses from (4 / 8 / 16 sites per
    workgroup, pipeline depth 2 / 3, traversal orders 0 / 1 / 2) give bit-identical
    M_pc^dag M_pc (a site's arithmetic does not depend on the tile or the order), and the
    shape the bench usually picks (8 sites, depth 3, order 1) matches the oracle at a
    sampled site."""
    import torch

    dims, Ls, mf = (16, 16, 16, 32), 16, 0.01
    op, U = make_operator(dims, Ls, eps=0.2, seed=0, prec=F64, max_nrhs=1, max_cg_rhs=0, mf=mf)
    psi = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=11), EVEN)
    v = pack(op, psi[None], EVEN)
    ref = None
    for order in (0, 1, 2):
        op.set_order(order)
        for spb in (4, 8, 16):
            for depth in (2, 3):
                op.set_tile(spb, depth, 1)
                w = op.new_field(1)
                op.mpcdagmpc(v, w, 1)
                torch.cuda.synchronize()
                if ref is None:
                    ref = w.clone()
                else:
                    assert torch.equal(w, ref), (order, spb, depth)
    op.set_order(1)
    op.set_tile(8, 3, 1)
    w = op.new_field(1)
    op.mpcdagmpc(v, w, 1)
    sites = sample_sites(dims, 1, seed=12, parity=EVEN)
    got = gpu_at_sites(unpack(op, w, 1, EVEN)[0], sites)
    exp = oracle_at_sites(lambda u, p: L.mpcdagmpc(u, L.on_parity(p, EVEN), 1.8, mf), U, psi, dims, sites, 4)
    assert rel(got, exp) < 1e-13


def test_rb_workload_gauge_covariance():
    """16^3 x 32, Ls = 16, FP64: with U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag and psi -> g psi,
    M_pc^dag M_pc[U^g] (g psi) = g (M_pc^dag M_pc[U] psi) over the whole lattice."""
    dims, Ls = (16, 16, 16, 32), 16
    U = synth.gauge_links(dims, eps=0.2, seed=0)
    g = synth.gauge_transform(dims, seed=13)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ L.dagger(L.shift(g, mu, +1))
    gpsi = lambda f: f @ np.swapaxes(g, -1, -2)  # noqa: E731  colour rotation per site
    psi = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=14), EVEN)
    outs = []
    for links, field in ((U, psi), (Ug, gpsi(psi))):
        op, _ = make_operator(dims, Ls, prec=F64, max_nrhs=1, max_cg_rhs=0, U=links)
        w = op.new_field(1)
        op.mpcdagmpc(pack(op, field[None], EVEN), w, 1)
        outs.append(unpack(op, w, 1, EVEN)[0])
        op.close()
    assert rel(outs[1], gpsi(outs[0])) < 1e-13
