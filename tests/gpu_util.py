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


def patch_indices(dims, centre, radius):
    """Index arrays (t, z, y, x order) of a periodic patch of side 2*radius+2
    around ``centre`` = (x, y, z, t), with the origin's coordinate sum even so
    the patch's own checkerboard parity equals the lattice's."""
    X, Y, Z, T = dims
    side = 2 * radius + 2
    origin = [c - radius for c in centre]
    if sum(origin) % 2:
        origin[0] -= 1  # keep parity; the centre stays >= radius from both ends
    idx = [np.arange(o, o + side) % L for o, L in zip(origin, (X, Y, Z, T))]
    local = tuple(c - o for c, o in zip(centre, origin))
    return idx, local


def take_patch(field, idx, lattice_axes_from_end):
    """Sub-array of a natural-layout field at the patch indices (periodic)."""
    ix, iy, iz, it = idx
    a = lattice_axes_from_end  # axis of x counted from the end (fermions: -3, links: -3)
    out = np.take(field, it, axis=a - 3)
    out = np.take(out, iz, axis=a - 2)
    out = np.take(out, iy, axis=a - 1)
    out = np.take(out, ix, axis=a)
    return out


def sample_sites(dims, n, seed, parity=0):
    """n distinct lattice sites (x, y, z, t) of one parity."""
    rng = np.random.default_rng(seed)
    X, Y, Z, T = dims
    out = []
    while len(out) < n:
        c = (int(rng.integers(X)), int(rng.integers(Y)), int(rng.integers(Z)), int(rng.integers(T)))
        if sum(c) % 2 == parity and c not in out:
            out.append(c)
    return out
