"""FP16 + per-site FP32 scale storage of a 5D fermion (oracle; test infrastructure).

The paper only reports that mixed-precision solves were also run (Results
section), with no storage format.  The reading used here: each (5D site,
right-hand side) spinor -- 24 real numbers, taken in FP32 -- is stored as one
FP32 scale s = max |v| and 24 IEEE half values h = round_to_nearest_even(v * r)
with r = 1 / s rounded to FP32 (s = 0 stores zeros).  Decoding is
v' = float32(h) * s.
"""

from __future__ import annotations

import numpy as np


def encode(psi: np.ndarray):
    """Natural-layout complex field -> (half reals [..., 4, 3, 2], scale [...])."""
    re = np.stack([psi.real, psi.imag], axis=-1).astype(np.float64)
    flat = re.reshape(re.shape[:-3] + (24,))
    scale = np.max(np.abs(flat), axis=-1).astype(np.float32)
    safe = np.where(scale > 0, scale, 1.0).astype(np.float32)
    inv = (np.float32(1.0) / safe).astype(np.float32)
    q = (flat.astype(np.float32) * inv[..., None]).astype(np.float16)
    q = np.where(scale[..., None] > 0, q, np.float16(0))
    return q.reshape(re.shape), scale


def decode(q: np.ndarray, scale: np.ndarray) -> np.ndarray:
    v = q.astype(np.float32) * scale[..., None, None, None]
    return (v[..., 0] + 1j * v[..., 1]).astype(np.complex128)
