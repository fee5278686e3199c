"""Helpers of the GPU parity tests: build a libdwf operator from the seeded
synthetic inputs, move natural-layout NumPy fields through the C ABI, and
measure relative errors.  The oracle side of each comparison is computed by
the test itself from ``oracle``; nothing here does the method's arithmetic."""

import numpy as np

import synth

M5, MF = 1.8, 0.01


def torch_mod():
    import torch

    return torch


def dev_tensor(a):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def make_operator(dims, Ls, eps=0.3, seed=0, prec=0, max_nrhs=3, max_cg_rhs=2, M5_=M5, mf=MF, U=None):
    import paper_2103_05034_amd as dwf

    if U is None:
        U = synth.gauge_links(dims, eps=eps, seed=seed)
    op = dwf.Operator(dev_tensor(U), dims, Ls, M5_, mf, prec=prec, max_nrhs=max_nrhs, max_cg_rhs=max_cg_rhs)
    return op, U


def pack(op, nat, parity):
    """nat: [nrhs][Ls][T][Z][Y][X][4][3] complex128 numpy -> packed device buffer."""
    return op.pack(dev_tensor(nat), parity)


def unpack(op, packed, nrhs, parity):
    torch = torch_mod()
    torch.cuda.synchronize()
    out = op.unpack(packed, nrhs, parity)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def rel_per_rhs(a, b):
    return max(rel(a[k], b[k]) for k in range(a.shape[0]))
