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


def rel_linf(a, b, where=INTERIOR) -> float:
    """max |a - b| / max |b| over the selected nodes (Sec. 5.1's epsilon_inf)."""
    a, b = np.asarray(a)[where], np.asarray(b)[where]
    return float(np.abs(a - b).max() / np.abs(b).max())


def eps2(a, b, r, where=INTERIOR) -> float:
    """Sec. 5.1's cylindrically weighted epsilon_2 of a against b: weights
    r_i dr dz per node (uniform dr, dz cancel), r the radial node coordinates."""
    a, b = np.asarray(a)[where], np.asarray(b)[where]
    w = np.broadcast_to(np.asarray(r)[where[2]], a.shape)
    return float(np.sqrt(np.sum(w * (a - b) ** 2) / np.sum(w * b * b)))


def histories_agree(ha, hb) -> bool:
    """Residual histories of two solves agree at every cycle both evaluated
    (a cycle that ends in a merged finest pass has no norm: None) and in length."""
    return len(ha) == len(hb) and all(a == b for a, b in zip(ha, hb) if a is not None and b is not None)
