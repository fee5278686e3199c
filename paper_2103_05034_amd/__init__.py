"""Python binding of libdwf: the red-black Shamir domain-wall operator on gfx950.

The binding only marshals arguments: every step runs in the HIP kernels of
``libdwf.so``.  PyTorch provides device memory (the workspace and the field
buffers are torch tensors) and the stream (torch's current stream).  If the
library has not been built this module raises at import-free call time --
there is no CPU fallback.

Two levels:

* module functions with the C ABI's names (``dwf_create``, ``dwf_mpc``, ...)
  taking raw integers / pointers, for callers who manage memory themselves;
* :class:`Operator`, which owns a workspace tensor and a handle and accepts
  torch tensors.

Packed fields are 1-D ``torch.uint8`` tensors of ``field_bytes(nrhs)`` bytes
(layout documented in ``include/dwf.h``); natural fields are complex128
tensors ``[nrhs][Ls][T][Z][Y][X][4][3]``; links are complex128
``[T][Z][Y][X][4][3][3]``.
"""

from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdwf.so")

DWF_OK, DWF_EINVAL, DWF_ENOMEM, DWF_EHIP, DWF_ENOCONV, DWF_EBREAKDOWN, DWF_WLAMBDA = 0, -1, -2, -3, -4, -5, 1
DWF_F64, DWF_F32, DWF_F16S = 0, 1, 2
DWF_EVEN, DWF_ODD, DWF_BOTH = 0, 1, 2
DWF_DOT_NOALLOC_MAX_RHS = 64  # as in include/dwf.h

_STATUS = {
    DWF_EINVAL: "DWF_EINVAL",
    DWF_ENOMEM: "DWF_ENOMEM",
    DWF_EHIP: "DWF_EHIP",
    DWF_ENOCONV: "DWF_ENOCONV",
    DWF_EBREAKDOWN: "DWF_EBREAKDOWN",
}


class DWFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_dbl_p = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
# int (*)(void* user, int iteration, int nrhs, const double* rel_resid)
class HDCRParams(ctypes.Structure):
    """dwf_hdcr_params of include/dwf.h."""

    _fields_ = [
        ("smoother_order", ctypes.c_int),
        ("smoother_lo", ctypes.c_double),
        ("smoother_hi", ctypes.c_double),
        ("coarse_tol", ctypes.c_double),
        ("coarse_maxiter", ctypes.c_int),
        ("nkrylov", ctypes.c_int),
        ("coarse_prec", ctypes.c_int),
    ]


PROGRESS_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double))

# name -> (restype, argtypes); mirrors include/dwf.h
_PROTOS = {
    "dwf_workspace_bytes": (ctypes.c_size_t, [_c_int_p, _i, _i, _i, _i]),
    "dwf_field_bytes": (ctypes.c_size_t, [_c_int_p, _i, _i, _i]),
    "dwf_create": (_i, [ctypes.POINTER(_vp), _vp, _c_int_p, _i, _d, _d, _i, _i, _i, _vp, ctypes.c_size_t, _vp]),
    "dwf_update_links": (_i, [_vp, _vp]),
    "dwf_set_stream": (_i, [_vp, _vp]),
    "dwf_destroy": (_i, [_vp]),
    "dwf_last_error": (ctypes.c_char_p, []),
    "dwf_pack": (_i, [_vp, _vp, _vp, _i, _i]),
    "dwf_unpack": (_i, [_vp, _vp, _vp, _i, _i]),
    "dwf_dhop": (_i, [_vp, _vp, _vp, _i, _i, _i]),
    "dwf_m5d": (_i, [_vp, _vp, _vp, _i, _i]),
    "dwf_m5d_inv": (_i, [_vp, _vp, _vp, _i, _i]),
    "dwf_ddw": (_i, [_vp, _vp, _vp, _i, _i]),
    "dwf_mpc": (_i, [_vp, _vp, _vp, _i, _i]),
    "dwf_mpcdagmpc": (_i, [_vp, _vp, _vp, _i]),
    "dwf_cg": (_i, [_vp, _vp, _vp, _i, _d, _i, _c_int_p, _c_dbl_p]),
    "dwf_solve_rb": (_i, [_vp, _vp, _vp, _d, _i, _c_int_p, _c_dbl_p]),
    "dwf_power": (_i, [_vp, _vp, _i, _d, _c_dbl_p, _c_int_p]),
    "dwf_chebyshev_filter": (_i, [_vp, _i, _d, _d, _vp, _i]),
    "dwf_chebyshev_series": (_i, [_vp, _i, _d, _d, _i, _i, _vp, _vp]),
    "dwf_chebyshev_smoother": (_i, [_vp, _i, _d, _d, _vp, _vp, _i]),
    "dwf_gram_schmidt": (_i, [_vp, _vp, _i, _c_dbl_p]),
    "dwf_dot": (_i, [_vp, _i, _vp, _vp, _i, _vp]),
    "dwf_dot_noalloc": (_i, [_c_int_p, _i, _i, _vp, _vp, _i, _vp, _vp]),
    "dwf_force": (_i, [_vp, _vp, _vp, _vp]),
    "dwf_lie_force": (_i, [_vp, _vp, _vp, _vp]),
    "dwf_set_schur_form": (_i, [_vp, _i]),
    "dwf_solve_unprec": (_i, [_vp, _vp, _vp, _d, _i, _c_int_p, _c_dbl_p]),
    "dwf_set_blocks": (_i, [_vp, _c_int_p, _c_int_p]),
    "dwf_set_blocks_ex": (_i, [_vp, _c_int_p, _i, _c_int_p]),
    "dwf_hdw": (_i, [_vp, _vp, _vp, _i]),
    "dwf_hdcr_workspace_bytes": (ctypes.c_size_t, [_vp, _i, _i]),
    "dwf_hdcr_create": (_i, [_vp, _i, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp)]),
    "dwf_hdcr_destroy": (_i, [_vp]),
    "dwf_hdcr_filter": (_i, [_vp, _i, _d, _d, _vp, _i]),
    "dwf_hdcr_series": (_i, [_vp, _i, _d, _d, _i, _i, _vp, _vp]),
    "dwf_hdcr_set_basis": (_i, [_vp, _vp]),
    "dwf_hdcr_coarse_data": (_vp, [_vp]),
    "dwf_hdcr_coarse_apply": (_i, [_vp, _vp, _vp]),
    "dwf_hdcr_coarse_solve": (_i, [_vp, _vp, _vp, _d, _i, _c_int_p]),
    "dwf_hdcr_smoother": (_i, [_vp, _vp, _vp]),
    "dwf_hdcr_vcycle": (_i, [_vp, _vp, _vp, _c_int_p]),
    "dwf_hdcr_solve": (_i, [_vp, _vp, _vp, _d, _i, _c_int_p, _c_dbl_p, _c_int_p]),
    "dwf_chiral_split": (_i, [_vp, _vp, _vp, _i]),
    "dwf_block_scratch_bytes": (ctypes.c_size_t, [_vp, _i]),
    "dwf_block_orthonormalize": (_i, [_vp, _vp, _i, _vp, ctypes.c_size_t]),
    "dwf_restrict": (_i, [_vp, _vp, _i, _vp, _i, _vp]),
    "dwf_prolong": (_i, [_vp, _vp, _i, _vp, _i, _vp]),
    "dwf_set_tile": (_i, [_vp, _i, _i, _i]),
    "dwf_set_order": (_i, [_vp, _i]),
    "dwf_set_order_box": (_i, [_vp, _i, _i, _i]),
    "dwf_get_order": (_i, [_vp, _c_int_p, _c_int_p]),
    "dwf_set_occupancy": (_i, [_vp, _i]),
    "dwf_set_progress": (_i, [_vp, PROGRESS_FN, _vp, _i]),
    "dwf_autotune": (_i, [_vp, _i, _i, _c_int_p, _c_int_p, _c_int_p, _c_dbl_p]),
    "dwf_tune_cache_clear": (_i, []),
    "dwf_enable_timing": (_i, [_vp, _i]),
    "dwf_kernel_time": (_i, [_vp, _c_dbl_p, ctypes.POINTER(ctypes.c_longlong)]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libdwf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2103_05034_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _PROTOS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load_library().dwf_last_error().decode()


def _check(code, allow=()):
    if code != DWF_OK and code not in allow:
        raise DWFError(code, last_error())
    return code


def _dims(dims):
    return (ctypes.c_int * 4)(*[int(d) for d in dims])


# ---- thin functions with the C names -------------------------------------------------
def dwf_workspace_bytes(dims, Ls, prec, max_nrhs, max_cg_rhs):
    return load_library().dwf_workspace_bytes(_dims(dims), Ls, prec, max_nrhs, max_cg_rhs)


def dwf_field_bytes(dims, Ls, prec, nrhs):
    return load_library().dwf_field_bytes(_dims(dims), Ls, prec, nrhs)


def tune_cache_clear():
    """Forget the launch shapes dwf_autotune cached in this process (the DWF_TUNE_CACHE
    file, if any, is kept and read again on the next tuning)."""
    _check(load_library().dwf_tune_cache_clear())


def dwf_dot_noalloc(dims, Ls, prec, a, b, nrhs, result, stream=None):
    """The allocation-free inner products (include/dwf.h): a and b packed one-parity fields
    (torch tensors on one HIP device), result a float64 tensor of 2 nrhs values on that device,
    stream a hipStream_t (default: torch's current stream).  The tensors are checked here; the
    lattice, precision and nrhs are checked by the library, whose status code is returned."""
    import torch

    dev = a.device if isinstance(a, torch.Tensor) else None
    if dev is None or dev.type != "cuda":
        raise DWFError(DWF_EINVAL, "dwf_dot_noalloc: a must be a tensor on a HIP device")
    need = dwf_field_bytes(dims, Ls, prec, nrhs) if 0 < nrhs <= DWF_DOT_NOALLOC_MAX_RHS else 0
    pa = _tensor_ptr(a, dev, "a", nbytes=need or None)
    pb = _tensor_ptr(b, dev, "b", nbytes=need or None)
    pr = _tensor_ptr(result, dev, "result", dtype=torch.float64,
                     nbytes=16 * nrhs if 0 < nrhs <= DWF_DOT_NOALLOC_MAX_RHS else None)
    if stream is None:
        stream = _stream()
    return load_library().dwf_dot_noalloc(_dims(dims), int(Ls), int(prec), pa, pb, int(nrhs), pr, stream)


def _thin(name):
    def call(*args):
        return getattr(load_library(), name)(*args)

    call.__name__ = name
    call.__doc__ = f"Direct call of {name} from libdwf.so (ctypes arguments, see include/dwf.h)."
    return call


for _name in _PROTOS:
    if _name not in globals():
        globals()[_name] = _thin(_name)


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr() if hasattr(t, "data_ptr") else int(t))


def _tensor_ptr(t, device, what, nbytes=None, dtype=None, shape=None):
    """Device pointer of tensor t after checking what the C call will assume of it:
    a torch tensor on the operator's device, contiguous, of the given dtype and
    shape, and holding at least nbytes bytes.  Raises DWFError(DWF_EINVAL) otherwise,
    before anything reaches the library (a kernel would read or write past a short
    buffer)."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise DWFError(DWF_EINVAL, f"{what}: expected a torch tensor, got {type(t).__name__}")
    if t.device != device:
        raise DWFError(DWF_EINVAL, f"{what}: tensor on {t.device}, the operator's device is {device}")
    if not t.is_contiguous():
        raise DWFError(DWF_EINVAL, f"{what}: tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise DWFError(DWF_EINVAL, f"{what}: dtype {t.dtype}, expected {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise DWFError(DWF_EINVAL, f"{what}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if nbytes is not None and t.numel() * t.element_size() < nbytes:
        raise DWFError(DWF_EINVAL, f"{what}: {t.numel() * t.element_size()} bytes, at least {nbytes} needed")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Operator:
    """A libdwf handle with its torch-allocated workspace.

    ``U`` is a complex128 CUDA tensor ``[T][Z][Y][X][4][3][3]``; ``dims`` =
    (X, Y, Z, T).  ``prec`` selects the storage precision of the handle's
    packed fields; ``max_nrhs`` the batch held by the operator temporaries;
    ``max_cg_rhs`` the number of simultaneous CG right-hand sides.

    Every method checks its tensors (device, contiguity, dtype and shape of
    natural fields and links, byte size of packed fields) before calling the
    library, and raises :class:`DWFError` if one does not fit.
    """

    def __init__(self, U, dims, Ls, M5, mf, prec=DWF_F64, max_nrhs=1, max_cg_rhs=1):
        import torch

        lib = load_library()
        self.lib = lib
        self.dims = tuple(int(d) for d in dims)
        self.Ls, self.M5, self.mf, self.prec = int(Ls), float(M5), float(mf), int(prec)
        self.max_nrhs, self.max_cg_rhs = int(max_nrhs), int(max_cg_rhs)
        if not isinstance(U, torch.Tensor) or not U.is_cuda:
            raise DWFError(DWF_EINVAL, "U must be a complex128 tensor on a HIP device")
        self.device = U.device
        X, Y, Z, T = self.dims
        self.V4 = X * Y * Z * T
        self.V4h = self.V4 // 2
        self.U = U.contiguous()
        u_ptr = self._links(self.U)
        nbytes = lib.dwf_workspace_bytes(_dims(self.dims), self.Ls, self.prec, self.max_nrhs, self.max_cg_rhs)
        if nbytes == 0:
            raise DWFError(DWF_EINVAL, last_error())
        # 256-byte alignment: torch's caching allocator returns >= 512-byte aligned blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=U.device)
        h = ctypes.c_void_p()
        _check(
            lib.dwf_create(
                ctypes.byref(h), u_ptr, _dims(self.dims), self.Ls, self.M5, self.mf, self.prec,
                self.max_nrhs, self.max_cg_rhs, _ptr(self.workspace), nbytes, _stream(),
            )
        )
        self.h = h

    # -- memory helpers -------------------------------------------------------
    def field_bytes(self, nrhs=1, prec=None):
        p = self.prec if prec is None else prec
        return self.lib.dwf_field_bytes(_dims(self.dims), self.Ls, p, int(nrhs))

    def new_field(self, nrhs=1, both=False, prec=None):
        import torch

        n = self.field_bytes(nrhs, prec) * (2 if both else 1)
        return torch.zeros(n, dtype=torch.uint8, device=self.device)

    def natural_shape(self, nrhs=1):
        X, Y, Z, T = self.dims
        return (nrhs, self.Ls, T, Z, Y, X, 4, 3)

    def link_shape(self):
        X, Y, Z, T = self.dims
        return (T, Z, Y, X, 4, 3, 3)

    def _sync_stream(self):
        self.lib.dwf_set_stream(self.h, _stream())

    # -- argument checks (no library call) -------------------------------------
    def _f(self, t, nrhs=1, prec=None, both=False, what="field"):
        """Pointer of a packed field of nrhs right-hand sides (both parities if both)."""
        if int(nrhs) < 1:
            raise DWFError(DWF_EINVAL, f"{what}: nrhs must be >= 1")
        need = self.field_bytes(nrhs, prec) * (2 if both else 1)
        return _tensor_ptr(t, self.device, what, nbytes=need)

    def _natural(self, t, nrhs, what="natural field"):
        import torch

        return _tensor_ptr(t, self.device, what, dtype=torch.complex128, shape=self.natural_shape(nrhs))

    def _links(self, t, what="U"):
        import torch

        return _tensor_ptr(t, self.device, what, dtype=torch.complex128, shape=self.link_shape())

    def _coarse(self, t, shape, what="coarse vector"):
        import torch

        return _tensor_ptr(t, self.device, what, dtype=torch.complex128, shape=shape)

    # -- ABI calls ------------------------------------------------------------
    def update_links(self, U):
        U = U.contiguous() if hasattr(U, "contiguous") else U
        ptr = self._links(U)
        self.U = U
        self._sync_stream()
        _check(self.lib.dwf_update_links(self.h, ptr))

    def pack(self, natural, parity, out=None):
        if getattr(natural, "dim", lambda: 0)() != 8:
            raise DWFError(DWF_EINVAL, "natural field must be [nrhs][Ls][T][Z][Y][X][4][3]")
        nrhs = natural.shape[0]
        natural = natural.contiguous()
        src = self._natural(natural, nrhs)
        if out is None:
            out = self.new_field(nrhs, both=(parity == DWF_BOTH))
        dst = self._f(out, nrhs, both=(parity == DWF_BOTH), what="packed output")
        self._sync_stream()
        _check(self.lib.dwf_pack(self.h, src, dst, nrhs, parity))
        return out

    def unpack(self, packed, nrhs, parity, out=None):
        import torch

        src = self._f(packed, nrhs, both=(parity == DWF_BOTH), what="packed input")
        if out is None:
            out = torch.zeros(self.natural_shape(nrhs), dtype=torch.complex128, device=self.device)
        dst = self._natural(out, nrhs, what="natural output")
        self._sync_stream()
        _check(self.lib.dwf_unpack(self.h, src, dst, nrhs, parity))
        return out

    def dhop(self, inp, out, out_parity, nrhs=1, dagger=False):
        a, b = self._f(inp, nrhs, what="in"), self._f(out, nrhs, what="out")
        self._sync_stream()
        _check(self.lib.dwf_dhop(self.h, a, b, out_parity, nrhs, int(dagger)))
        return out

    def m5d(self, inp, out, nrhs=1, dagger=False):
        a, b = self._f(inp, nrhs, what="in"), self._f(out, nrhs, what="out")
        self._sync_stream()
        _check(self.lib.dwf_m5d(self.h, a, b, nrhs, int(dagger)))
        return out

    def m5d_inv(self, inp, out, nrhs=1, dagger=False):
        a, b = self._f(inp, nrhs, what="in"), self._f(out, nrhs, what="out")
        self._sync_stream()
        _check(self.lib.dwf_m5d_inv(self.h, a, b, nrhs, int(dagger)))
        return out

    def ddw(self, inp, out, nrhs=1, dagger=False):
        a, b = self._f(inp, nrhs, both=True, what="in"), self._f(out, nrhs, both=True, what="out")
        self._sync_stream()
        _check(self.lib.dwf_ddw(self.h, a, b, nrhs, int(dagger)))
        return out

    def mpc(self, inp, out, nrhs=1, dagger=False):
        a, b = self._f(inp, nrhs, what="in"), self._f(out, nrhs, what="out")
        self._sync_stream()
        _check(self.lib.dwf_mpc(self.h, a, b, nrhs, int(dagger)))
        return out

    def mpcdagmpc(self, inp, out, nrhs=1):
        a, b = self._f(inp, nrhs, what="in"), self._f(out, nrhs, what="out")
        self._sync_stream()
        _check(self.lib.dwf_mpcdagmpc(self.h, a, b, nrhs))
        return out

    def dot(self, a, b, nrhs=1, prec=None, out=None):
        """<a_r, b_r> for nrhs packed one-parity fields (FP64 sums in the library):
        a complex128 device tensor [nrhs] viewing ``out`` (float64 [nrhs, 2])."""
        import torch

        p = self.prec if prec is None else int(prec)
        pa, pb = self._f(a, nrhs, p, what="a"), self._f(b, nrhs, p, what="b")
        if out is None:
            out = torch.empty((nrhs, 2), dtype=torch.float64, device=self.device)
        po = _tensor_ptr(out, self.device, "out", dtype=torch.float64, shape=(nrhs, 2))
        self._sync_stream()
        _check(self.lib.dwf_dot(self.h, p, pa, pb, nrhs, po))
        return torch.view_as_complex(out)

    def cg(self, b, x, nrhs=1, tol=1e-10, maxiter=10000, allow_noconv=False):
        """Synchronous CG on M_pc^dag M_pc (b, x FP64 packed); returns (status, iters, true_rel_resid)."""
        pb, px = self._f(b, nrhs, DWF_F64, what="b"), self._f(x, nrhs, DWF_F64, what="x")
        it = (ctypes.c_int * nrhs)()
        res = (ctypes.c_double * nrhs)()
        self._sync_stream()
        code = self.lib.dwf_cg(self.h, pb, px, nrhs, tol, maxiter, it, res)
        _check(code, allow=(DWF_ENOCONV,) if allow_noconv else ())
        return code, list(it), list(res)

    def solve_rb(self, eta, psi, tol=1e-10, maxiter=10000):
        pe, pp = self._f(eta, 1, DWF_F64, both=True, what="eta"), self._f(psi, 1, DWF_F64, both=True, what="psi")
        it = ctypes.c_int()
        res = ctypes.c_double()
        self._sync_stream()
        code = self.lib.dwf_solve_rb(self.h, pe, pp, tol, maxiter, ctypes.byref(it), ctypes.byref(res))
        _check(code)
        return it.value, res.value

    def set_schur_form(self, form):
        """1: M_ee - M_eo M_oo^-1 M_oe (default); 2: 1 - M_ee^-1 M_eo M_oo^-1 M_oe."""
        _check(self.lib.dwf_set_schur_form(self.h, int(form)))

    def solve_unprec(self, eta, psi, tol=1e-10, maxiter=100000):
        """CGNR on D_DW^dag D_DW over both parities; returns (iterations, true residual)."""
        pe, pp = self._f(eta, 1, DWF_F64, both=True, what="eta"), self._f(psi, 1, DWF_F64, both=True, what="psi")
        it = ctypes.c_int()
        res = ctypes.c_double()
        self._sync_stream()
        code = self.lib.dwf_solve_unprec(self.h, pe, pp, tol, maxiter, ctypes.byref(it), ctypes.byref(res))
        _check(code)
        return it.value, res.value

    def power(self, v, iters=100, rtol=1e-6):
        pv = self._f(v, 1, what="v")
        lam = ctypes.c_double()
        done = ctypes.c_int()
        self._sync_stream()
        _check(self.lib.dwf_power(self.h, pv, iters, rtol, ctypes.byref(lam), ctypes.byref(done)))
        return lam.value, done.value

    @staticmethod
    def _warn_lambda(code):
        """DWF_WLAMBDA (the filter's top is below the measured lambda_max) becomes a Python warning."""
        if _check(code, allow=(DWF_WLAMBDA,)) == DWF_WLAMBDA:
            import warnings

            warnings.warn(last_error(), RuntimeWarning, stacklevel=3)

    def chebyshev_filter(self, vecs, nvecs, order, lo, hi):
        pv = self._f(vecs, nvecs, what="vecs")
        self._sync_stream()
        self._warn_lambda(self.lib.dwf_chebyshev_filter(self.h, order, lo, hi, pv, nvecs))
        return vecs

    def chebyshev_series(self, eta, out_series, m, lam_lo, lam_max, delta, nvec):
        pe, po = self._f(eta, 1, what="eta"), self._f(out_series, nvec, what="out_series")
        self._sync_stream()
        self._warn_lambda(self.lib.dwf_chebyshev_series(self.h, m, lam_lo, lam_max, delta, nvec, pe, po))
        return out_series

    def chebyshev_smoother(self, inp, out, order, lo, hi, nrhs=1):
        a, b = self._f(inp, nrhs, what="in"), self._f(out, nrhs, what="out")
        self._sync_stream()
        self._warn_lambda(self.lib.dwf_chebyshev_smoother(self.h, order, lo, hi, a, b, nrhs))
        return out

    def gram_schmidt(self, vecs, nvecs):
        import numpy as np

        pv = self._f(vecs, nvecs, what="vecs")
        R = (ctypes.c_double * (2 * nvecs * nvecs))()
        self._sync_stream()
        _check(self.lib.dwf_gram_schmidt(self.h, pv, nvecs, R))
        r = np.frombuffer(R, dtype=np.float64).reshape(nvecs, nvecs, 2)
        return r[..., 0] + 1j * r[..., 1]

    # ---- coarse-space transfer -----------------------------------------------------
    def set_blocks(self, block, both=False):
        """Blocks of bx, by, bz, bt 4D sites (all Ls slices); returns the number of blocks.
        both=True makes the coarse-space calls take fields of both parities."""
        nb = ctypes.c_int()
        par = DWF_BOTH if both else DWF_EVEN
        _check(self.lib.dwf_set_blocks_ex(self.h, (ctypes.c_int * 4)(*[int(b) for b in block]), par, ctypes.byref(nb)))
        self.nblocks = nb.value
        self.coarse_both = bool(both)
        return nb.value

    def _cf(self, t, n, what):
        """A field of the coarse-space calls: n fields, both parities if the blocks cover both."""
        return self._f(t, n, both=getattr(self, "coarse_both", False), what=what)

    def hdw(self, inp, out, nrhs=1):
        """out = H_DW inp = Gamma_5 D_DW inp (packed fields of both parities)."""
        a, b = self._f(inp, nrhs, both=True, what="in"), self._f(out, nrhs, both=True, what="out")
        self._sync_stream()
        _check(self.lib.dwf_hdw(self.h, a, b, nrhs))

    def chiral_split(self, vecs, nvec, out=None):
        """out[2k], out[2k+1] = (1 +- Gamma_5) vecs[k] / 2."""
        if out is None:
            out = self.new_field(2 * nvec, both=getattr(self, "coarse_both", False))
        a, b = self._cf(vecs, nvec, "vecs"), self._cf(out, 2 * nvec, "out")
        self._sync_stream()
        _check(self.lib.dwf_chiral_split(self.h, a, b, nvec))
        return out

    def block_orthonormalize(self, basis, nvec):
        import torch

        pb = self._cf(basis, nvec, "basis")
        nbytes = self.lib.dwf_block_scratch_bytes(self.h, nvec)
        if nbytes == 0:
            raise DWFError(DWF_EINVAL, "set blocks first; nvec must be in [1, 64]")
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._sync_stream()
        _check(self.lib.dwf_block_orthonormalize(self.h, pb, nvec, _ptr(scratch), nbytes))
        return basis

    def restrict(self, basis, nvec, v, nrhs=1, coarse=None):
        """coarse[r][b][k] = <phi_k^b, v_r> (complex128 device tensor [nrhs, nblocks, nvec])."""
        import torch

        if not hasattr(self, "nblocks"):
            raise DWFError(DWF_EINVAL, "set blocks first")
        pb, pv = self._cf(basis, nvec, "basis"), self._cf(v, nrhs, "v")
        if coarse is None:
            coarse = torch.empty((nrhs, self.nblocks, nvec), dtype=torch.complex128, device=self.device)
        pc = self._coarse(coarse, (nrhs, self.nblocks, nvec), "coarse")
        self._sync_stream()
        _check(self.lib.dwf_restrict(self.h, pb, nvec, pv, nrhs, pc))
        return coarse

    def prolong(self, basis, nvec, coarse, nrhs=1, out=None):
        """out_r = sum_{b,k} coarse[r][b][k] phi_k^b."""
        if not hasattr(self, "nblocks"):
            raise DWFError(DWF_EINVAL, "set blocks first")
        if out is None:
            out = self.new_field(nrhs, both=getattr(self, "coarse_both", False))
        coarse = coarse.contiguous()
        pb, po = self._cf(basis, nvec, "basis"), self._cf(out, nrhs, "out")
        pc = self._coarse(coarse, (nrhs, self.nblocks, nvec), "coarse")
        self._sync_stream()
        _check(self.lib.dwf_prolong(self.h, pb, nvec, pc, nrhs, po))
        return out

    def force(self, X_e, Y_e, grad=None):
        import torch

        px, py = self._f(X_e, 1, DWF_F64, what="X"), self._f(Y_e, 1, DWF_F64, what="Y")
        if grad is None:
            grad = torch.zeros(self.link_shape(), dtype=torch.complex128, device=self.device)
        pg = self._links(grad, what="grad")
        self._sync_stream()
        _check(self.lib.dwf_force(self.h, px, py, pg))
        return grad

    def lie_force(self, U, grad, F=None):
        """F[t, z, y, x, mu, a] = -Im tr(T^a U_mu(x) grad_mu(x)^dag), T^a = lambda^a / 2: the
        derivative of the action along exp(i omega T^a) U_mu(x), from dwf_force's gradient."""
        import torch

        pu, pg = self._links(U, what="U"), self._links(grad, what="grad")
        shape = self.link_shape()[:5] + (8,)
        if F is None:
            F = torch.empty(shape, dtype=torch.float64, device=self.device)
        pf = _tensor_ptr(F, self.device, "F", dtype=torch.float64, shape=shape)
        self._sync_stream()
        _check(self.lib.dwf_lie_force(self.h, pu, pg, pf))
        return F

    def set_tile(self, sites_per_block, pipeline_depth=0, rhs_per_block=0):
        _check(self.lib.dwf_set_tile(self.h, sites_per_block, pipeline_depth, rhs_per_block))

    def set_order(self, mode):
        _check(self.lib.dwf_set_order(self.h, int(mode)))

    def set_order_box(self, nx, ny, nz):
        """Traversal order 3: the (x, y, z) volume cut into nx x ny x nz boxes, one group per XCD."""
        _check(self.lib.dwf_set_order_box(self.h, int(nx), int(ny), int(nz)))

    def get_order(self):
        """(mode, (nx, ny, nz)) of the traversal order in use; the cut is (0, 0, 0) unless mode is 3."""
        mode = ctypes.c_int()
        box = (ctypes.c_int * 3)()
        _check(self.lib.dwf_get_order(self.h, ctypes.byref(mode), box))
        return mode.value, tuple(box)

    def set_occupancy(self, workgroups_per_cu):
        _check(self.lib.dwf_set_occupancy(self.h, int(workgroups_per_cu)))

    def autotune(self, nrhs=1, reps=10):
        """Pick the fastest hop launch shape by timing M_pc^dag M_pc; returns (spb, depth, ms)."""
        spb, depth, rpb, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self._sync_stream()
        _check(
            self.lib.dwf_autotune(
                self.h, nrhs, reps, ctypes.byref(spb), ctypes.byref(depth), ctypes.byref(rpb), ctypes.byref(ms)
            )
        )
        self.tile = (spb.value, depth.value, rpb.value)
        return spb.value, depth.value, ms.value

    def set_progress(self, fn=None, every=100):
        """Report solver progress: fn(iteration, [rel_resid per rhs]) is called from dwf_cg /
        dwf_solve_rb at least `every` iterations apart; a truthy return stops the solve
        (the solver then returns DWF_ENOCONV).  fn=None turns reporting off."""
        if fn is None:
            self._progress_cb = None
            _check(self.lib.dwf_set_progress(self.h, PROGRESS_FN(), None, 0))
            return

        def tramp(_user, it, n, rel):
            try:
                return 1 if fn(int(it), [rel[k] for k in range(n)]) else 0
            except Exception:  # an exception cannot cross the C frame: stop the solve instead
                return 1

        self._progress_cb = PROGRESS_FN(tramp)  # kept alive while registered
        _check(self.lib.dwf_set_progress(self.h, self._progress_cb, None, int(every)))

    def enable_timing(self, on=True, stride=1):
        """Time hop launches with HIP events (every `stride`-th one when stride > 1)."""
        _check(self.lib.dwf_enable_timing(self.h, (int(stride) if stride > 1 else 1) if on else 0))

    def kernel_time(self):
        ms = ctypes.c_double()
        n = ctypes.c_longlong()
        _check(self.lib.dwf_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.dwf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HDCR:
    """Two-level HDCR solver (pGCR(H_DW) with the V(1,1) preconditioner) on an
    FP64 :class:`Operator` whose blocks were set with ``set_blocks(block, both=True)``."""

    def __init__(self, op, nvec, smoother_order=12, smoother_lo=0.5, smoother_hi=60.0, coarse_tol=0.02,
                 coarse_maxiter=1000, nkrylov=8, coarse_prec=DWF_F64):
        import torch

        self.op, self.lib, self.nvec = op, op.lib, nvec
        self.params = HDCRParams(smoother_order, smoother_lo, smoother_hi, coarse_tol, coarse_maxiter, nkrylov,
                                 coarse_prec)
        nbytes = self.lib.dwf_hdcr_workspace_bytes(op.h, nvec, nkrylov)
        if nbytes == 0:
            raise DWFError(DWF_EINVAL, "set DWF_BOTH blocks first; nvec and nkrylov must be in [1, 64]")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=op.device)
        hd = _vp()
        op._sync_stream()
        _check(self.lib.dwf_hdcr_create(op.h, nvec, ctypes.byref(self.params), _ptr(self.ws), nbytes, ctypes.byref(hd)))
        self.hd = hd
        self.basis = None

    def coarse_vector(self):
        import torch

        return torch.zeros((self.op.nblocks, self.nvec), dtype=torch.complex128, device=self.op.device)

    def _cv(self, t, what):
        return self.op._coarse(t, (self.op.nblocks, self.nvec), what)

    def _both(self, t, n, what):
        return self.op._f(t, n, DWF_F64, both=True, what=what)

    def filter(self, vecs, nvecs, order, lo, hi):
        """vecs <- T_order(x(D^dag D)) vecs for nvecs fields of both parities."""
        pv = self._both(vecs, nvecs, "vecs")
        self.op._sync_stream()
        _check(self.lib.dwf_hdcr_filter(self.hd, order, lo, hi, pv, nvecs))

    def series(self, eta, m, lam_lo, lam_max, delta, nvec, out=None):
        """The setup series from one field eta: out[0] = T_m(x_[lam_lo, lam_max](D^dag D)) eta,
        out[k] = T_{k delta}(2 D^dag D / lam_max - 1) out[0] (nvec fields of both parities)."""
        if out is None:
            out = self.op.new_field(nvec, both=True)
        pe, po = self._both(eta, 1, "eta"), self._both(out, nvec, "out")
        self.op._sync_stream()
        _check(self.lib.dwf_hdcr_series(self.hd, m, lam_lo, lam_max, delta, nvec, pe, po))
        return out

    def set_basis(self, basis):
        """Build the little Dirac operator of H_DW on ``basis`` (kept referenced)."""
        pb = self._both(basis, self.nvec, "basis")
        self.op._sync_stream()
        self.basis = basis
        _check(self.lib.dwf_hdcr_set_basis(self.hd, pb))

    def coarse_operator(self):
        """The stencil as a complex128 (complex64 with coarse_prec=DWF_F32) tensor
        [nblocks, 9, nvec(k), nvec(j)] viewing the workspace."""
        import torch

        n, nb = self.nvec, self.op.nblocks
        f32 = self.params.coarse_prec == DWF_F32
        off = self.lib.dwf_hdcr_coarse_data(self.hd) - self.ws.data_ptr()
        raw = self.ws[off : off + nb * 9 * n * n * (8 if f32 else 16)]
        return raw.view(torch.complex64 if f32 else torch.complex128).view(nb, 9, n, n)

    def coarse_apply(self, x, y=None):
        if y is None:
            y = self.coarse_vector()
        px, py = self._cv(x, "x"), self._cv(y, "y")
        self.op._sync_stream()
        _check(self.lib.dwf_hdcr_coarse_apply(self.hd, px, py))
        return y

    def coarse_solve(self, d, c=None, tol=1e-10, maxiter=10000):
        if c is None:
            c = self.coarse_vector()
        pd, pc = self._cv(d, "d"), self._cv(c, "c")
        it = ctypes.c_int()
        self.op._sync_stream()
        _check(self.lib.dwf_hdcr_coarse_solve(self.hd, pd, pc, tol, maxiter, ctypes.byref(it)))
        return c, it.value

    def smoother(self, r, out=None):
        if out is None:
            out = self.op.new_field(1, both=True)
        pr, po = self._both(r, 1, "r"), self._both(out, 1, "out")
        self.op._sync_stream()
        _check(self.lib.dwf_hdcr_smoother(self.hd, pr, po))
        return out

    def vcycle(self, r, x=None):
        if x is None:
            x = self.op.new_field(1, both=True)
        pr, px = self._both(r, 1, "r"), self._both(x, 1, "x")
        ci = ctypes.c_int()
        self.op._sync_stream()
        _check(self.lib.dwf_hdcr_vcycle(self.hd, pr, px, ctypes.byref(ci)))
        return x, ci.value

    def solve(self, eta, psi, tol=1e-10, maxiter=1000, allow_noconv=False):
        """D_DW psi = eta; returns (outer iterations, true relative residual, coarse iterations)."""
        pe, pp = self._both(eta, 1, "eta"), self._both(psi, 1, "psi")
        it, ci = ctypes.c_int(), ctypes.c_int()
        res = ctypes.c_double()
        self.op._sync_stream()
        _check(
            self.lib.dwf_hdcr_solve(self.hd, pe, pp, tol, maxiter, ctypes.byref(it), ctypes.byref(res),
                                    ctypes.byref(ci)),
            allow=(DWF_ENOCONV,) if allow_noconv else (),
        )
        return it.value, res.value, ci.value

    def close(self):
        if getattr(self, "hd", None):
            self.lib.dwf_hdcr_destroy(self.hd)
            self.hd = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def __getattr__(name):
    """PseudofermionAction lives in the autograd module, which imports torch."""
    if name == "PseudofermionAction":
        from .autograd import PseudofermionAction

        return PseudofermionAction
    raise AttributeError(name)
