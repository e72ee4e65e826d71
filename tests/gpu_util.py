"""Helpers shared by the GPU parity tests (no GPU work at import)."""
import numpy as np
import pytest
import torch


def rel_err(x, y):
    """|x - y| / max(|y|, 1), elementwise."""
    x = torch.as_tensor(x, dtype=torch.float64).cpu()
    y = torch.as_tensor(y, dtype=torch.float64).cpu()
    return (x - y).abs() / torch.clamp(y.abs(), min=1.0)


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2002_07401_amd as P
    P.load()   # raises if the HIP library is missing: no fallback
    return P
