"""Shared helpers for the GPU tests (not collected: no test_ prefix)."""

import sys

import numpy as np
import torch

DEV = "cuda:0"


def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1604_07893_amd import hyperpower as hpw
    hpw.load_library()  # raises if the library is missing: no fallback
    return hpw


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel(a, b) -> float:
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
