"""GPU parity at the method's edge cases, against the FP64 oracle.

* Ls = 1 and Ls = 2: the mass corners of the D_DW matrix (Chiral Fermion
  Actions section) land on the diagonal (Ls = 1: D_DW = D_W(1 + mf - M5)) or on
  the off-diagonal blocks (Ls = 2), which the kernel's wrapped s-couplings and
  the closed-form M5D^{-1} recursion must reproduce.
* Ls >= 32: few 4D sites per workgroup and long M5D^{-1} columns in LDS.
* FP16 + scale storage with several right-hand sides per workgroup.
Bars: FP64 relative 2-norm error <= 1e-13 (1e-14 for the site-local M5D).
"""

import numpy as np
import pytest

import synth
from oracle import lattice as L
from tests.gpu_util import M5, make_operator, pack, rel_per_rhs, unpack

pytestmark = pytest.mark.gpu

EVEN, ODD, BOTH = 0, 1, 2
F64, F16S = 0, 2
MF_EDGE = 0.05  # a mass large enough that a wrong corner term is far above the bar

EDGE_SHAPES = [((2, 2, 2, 2), 1), ((4, 4, 4, 4), 1), ((2, 2, 2, 2), 2), ((4, 4, 6, 4), 2), ((4, 4, 4, 4), 32),
               ((2, 2, 4, 2), 48)]


def _nat(dims, Ls, n, seed, parity=None):
    f = synth.gaussian_fermion_batch(dims, Ls, n, seed)
    if parity is None:
        return f
    return np.stack([L.on_parity(v, parity) for v in f])


@pytest.mark.parametrize("dims,Ls", EDGE_SHAPES)
def test_edge_dhop_and_m5d(dims, Ls):
    op, U = make_operator(dims, Ls, eps=0.4, seed=40, mf=MF_EDGE)
    nat = _nat(dims, Ls, 2, seed=41)
    for out_parity in (EVEN, ODD):
        inp = pack(op, nat, 1 - out_parity)
        out = op.new_field(2)
        for dagger in (False, True):
            op.dhop(inp, out, out_parity, 2, dagger)
            exp = np.stack([L.on_parity(L.dhop(U, L.on_parity(v, 1 - out_parity), dagger), out_parity) for v in nat])
            assert rel_per_rhs(unpack(op, out, 2, out_parity), exp) < 1e-13
    inp = pack(op, nat, EVEN)
    out = op.new_field(2)
    src = np.stack([L.on_parity(v, EVEN) for v in nat])
    for dagger in (False, True):
        op.m5d(inp, out, 2, dagger)
        exp = np.stack([L.m5d(v, M5, MF_EDGE, dag=dagger) for v in src])
        assert rel_per_rhs(unpack(op, out, 2, EVEN), exp) < 1e-14
        op.m5d_inv(inp, out, 2, dagger)
        exp = np.stack([L.m5d_inv(v, M5, MF_EDGE, dag=dagger) for v in src])
        assert rel_per_rhs(unpack(op, out, 2, EVEN), exp) < 1e-13


@pytest.mark.parametrize("dims,Ls", EDGE_SHAPES)
def test_edge_ddw_mpc_and_normal_operator(dims, Ls):
    op, U = make_operator(dims, Ls, eps=0.4, seed=42, mf=MF_EDGE)
    nat = _nat(dims, Ls, 1, seed=43)
    out = op.new_field(1, both=True)
    for dagger in (False, True):
        op.ddw(pack(op, nat, BOTH), out, 1, dagger)
        assert rel_per_rhs(unpack(op, out, 1, BOTH), L.ddw(U, nat[0], M5, MF_EDGE, dag=dagger)[None]) < 1e-13
    src = _nat(dims, Ls, 2, seed=44, parity=EVEN)
    inp = pack(op, src, EVEN)
    out = op.new_field(2)
    op.mpc(inp, out, 2, False)
    assert rel_per_rhs(unpack(op, out, 2, EVEN), np.stack([L.mpc(U, v, M5, MF_EDGE) for v in src])) < 1e-13
    op.mpc(inp, out, 2, True)
    assert rel_per_rhs(unpack(op, out, 2, EVEN), np.stack([L.mpc_dag(U, v, M5, MF_EDGE) for v in src])) < 1e-13
    op.mpcdagmpc(inp, out, 2)
    assert rel_per_rhs(unpack(op, out, 2, EVEN), np.stack([L.mpcdagmpc(U, v, M5, MF_EDGE) for v in src])) < 1e-13


def test_ls1_is_wilson():
    """At Ls = 1 the domain-wall operator is the Wilson operator with mass 1 + mf - M5:
    the GPU's D_DW against the oracle's plain Wilson D_W."""
    dims = (4, 4, 4, 4)
    op, U = make_operator(dims, 1, eps=0.4, seed=45, mf=MF_EDGE)
    nat = _nat(dims, 1, 1, seed=46)
    out = op.new_field(1, both=True)
    op.ddw(pack(op, nat, BOTH), out, 1, False)
    exp = L.wilson(U, nat[0], 1.0 + MF_EDGE - M5)
    assert rel_per_rhs(unpack(op, out, 1, BOTH), exp[None]) < 1e-13


def test_fp16s_rhs_per_block_identical():
    """FP16 + scale fields: workgroups looping over several rhs (links staged once)
    store exactly what one rhs per workgroup stores (5 rhs in groups of 2 and of 4)."""
    import torch

    dims, Ls = (4, 4, 6, 8), 5
    op, U = make_operator(dims, Ls, seed=47, prec=F16S, max_nrhs=5)
    inp = pack(op, _nat(dims, Ls, 5, seed=48, parity=EVEN), EVEN)
    ref = op.new_field(5)
    op.set_tile(0, 0, 1)
    op.mpcdagmpc(inp, ref, 5)
    for rpb in (2, 4):
        got = op.new_field(5)
        op.set_tile(0, 0, rpb)
        op.mpcdagmpc(inp, got, 5)
        torch.cuda.synchronize()
        assert torch.equal(ref, got), rpb
    fa, fb = inp.clone(), inp.clone()
    op.set_tile(0, 0, 1)
    op.chebyshev_filter(fa, 5, 3, 0.1, 40.0)
    op.set_tile(0, 0, 4)
    op.chebyshev_filter(fb, 5, 3, 0.1, 40.0)
    torch.cuda.synchronize()
    assert torch.equal(fa, fb)
