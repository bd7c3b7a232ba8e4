"""Upload helpers: numpy problem arrays -> torch device tensors (marshalling only)."""
from __future__ import annotations

import numpy as np


def design_to_device(AT: np.ndarray, store: str, device="cuda", lda: int | None = None):
    """(n, m) design array in its storage type -> (n, lda) device tensor.
    store: 'f64' | 'f32' | 'bf16' (AT holds uint16 bit patterns for bf16).
    With lda > m the padding rows are filled with NaN, which the kernels must
    never read into a result."""
    import torch
    n, m = AT.shape
    lda = m if lda is None else lda
    if store == "bf16":
        t = torch.from_numpy(np.ascontiguousarray(AT).view(np.int16)).view(torch.bfloat16)
    else:
        t = torch.from_numpy(np.ascontiguousarray(AT))
    if lda != m:
        pad = torch.full((n, lda), float("nan"), dtype=t.dtype)
        pad[:, :m] = t
        t = pad
    return t.to(device)


def vec_to_device(v: np.ndarray, device="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).to(device)
