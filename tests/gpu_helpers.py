"""Helpers shared by the GPU parity tests (host-side marshalling only)."""
import numpy as np
import pytest


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1608_06356_amd as q
    q.lib()   # raises if the library is missing: no silent fallback
    return torch, q


def u64(a):
    return np.asarray(a).astype(np.uint64)
