"""Helpers for the GPU tests: device transfers and error measures (no solver arithmetic)."""
import sys

import numpy as np
import torch

INTERIOR = (slice(None), slice(1, -1), slice(1, -1))


def say(*msg):
    """Name the case before a GPU step, so a failing run says what it was doing."""
    print("[case]", *msg, flush=True)
    sys.stdout.flush()


def dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda:0")


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_l2(a, b, where=INTERIOR) -> float:
    a, b = np.asarray(a)[where], np.asarray(b)[where]
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
