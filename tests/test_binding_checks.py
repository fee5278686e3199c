"""Host-only checks of the binding's argument validation: every Operator method
rejects a tensor on the wrong device, a non-contiguous one, a natural field or
link array of the wrong dtype or shape, and a packed buffer shorter than the
call needs -- before anything reaches the library, so no GPU is involved.

The operator is built without a handle (no device work); its device is the
CPU so that correctly placed CPU tensors reach the size checks."""

import pytest
import torch

import paper_2103_05034_amd as dwf


@pytest.fixture(scope="module")
def op():
    o = object.__new__(dwf.Operator)
    o.lib = dwf.load_library() if _have_lib() else None
    o.dims, o.Ls, o.prec = (4, 4, 4, 4), 4, dwf.DWF_F64
    o.device = torch.device("cpu")
    o.h = None
    o.max_nrhs = o.max_cg_rhs = 1
    o.nblocks = 8
    o.coarse_both = False
    return o


def _have_lib():
    import os

    if not os.path.exists(dwf.LIB_PATH):
        from paper_2103_05034_amd import build

        build.build()
    return True


FB = 192 * 4 * 128  # one FP64 half field of 4^4 x Ls 4


def _raises(fn, needle):
    with pytest.raises(dwf.DWFError) as e:
        fn()
    assert e.value.code == dwf.DWF_EINVAL
    assert needle in str(e.value), str(e.value)


def test_short_packed_buffers_are_rejected(op):
    good = torch.zeros(FB, dtype=torch.uint8)
    short = torch.zeros(FB - 1, dtype=torch.uint8)
    _raises(lambda: op.mpc(short, good), "bytes")
    _raises(lambda: op.mpc(good, short), "bytes")
    _raises(lambda: op.mpcdagmpc(good, good, nrhs=2), "bytes")
    _raises(lambda: op.dhop(good, short, 0), "bytes")
    _raises(lambda: op.ddw(good, good), "bytes")  # both parities need 2 FB
    _raises(lambda: op.cg(short, good), "bytes")
    _raises(lambda: op.solve_rb(good, good), "bytes")
    _raises(lambda: op.chebyshev_filter(good, 2, 4, 0.1, 60.0), "bytes")
    _raises(lambda: op.gram_schmidt(good, 2), "bytes")
    _raises(lambda: op.force(good, short), "bytes")
    _raises(lambda: op.dot(good, short), "bytes")
    _raises(lambda: op.unpack(short, 1, dwf.DWF_EVEN), "bytes")


def test_wrong_device_and_layout_are_rejected(op):
    meta = torch.empty(FB, dtype=torch.uint8, device="meta")
    good = torch.zeros(FB, dtype=torch.uint8)
    _raises(lambda: op.mpc(meta, good), "device")
    strided = torch.zeros(2 * FB, dtype=torch.uint8)[::2]
    _raises(lambda: op.mpc(strided, good), "contiguous")
    _raises(lambda: op.mpc(object(), good), "torch tensor")


def test_natural_fields_and_links_are_checked(op):
    nat = torch.zeros((1, 4, 4, 4, 4, 4, 4, 3), dtype=torch.complex64)
    _raises(lambda: op.pack(nat, dwf.DWF_EVEN), "dtype")
    nat = torch.zeros((1, 4, 4, 4, 4, 4, 4, 2), dtype=torch.complex128)
    _raises(lambda: op.pack(nat, dwf.DWF_EVEN), "shape")
    _raises(lambda: op.pack(torch.zeros(3, dtype=torch.complex128), dwf.DWF_EVEN), "natural field")
    U = torch.zeros((4, 4, 4, 4, 4, 3, 3), dtype=torch.complex64)
    _raises(lambda: op.update_links(U), "dtype")
    U = torch.zeros((4, 4, 4, 4, 3, 3, 3), dtype=torch.complex128)
    _raises(lambda: op.update_links(U), "shape")
    good = torch.zeros(FB, dtype=torch.uint8)
    grad = torch.zeros((4, 4, 4, 4, 4, 3, 3), dtype=torch.float64)
    _raises(lambda: op.force(good, good, grad), "dtype")


def test_coarse_vectors_are_checked(op):
    good = torch.zeros(FB * 4, dtype=torch.uint8)
    coarse = torch.zeros((1, 8, 3), dtype=torch.complex128)
    _raises(lambda: op.restrict(good, 4, good, 1, coarse=coarse), "shape")
    _raises(lambda: op.prolong(good, 4, coarse.to(torch.complex64), 1, out=good), "dtype")


def test_operator_refuses_links_off_the_device():
    U = torch.zeros((4, 4, 4, 4, 4, 3, 3), dtype=torch.complex128)
    _raises(lambda: dwf.Operator(U, (4, 4, 4, 4), 4, 1.8, 0.01), "HIP device")
