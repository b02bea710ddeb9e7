"""Helpers shared by the GPU tests (no method arithmetic here)."""
import sys

import numpy as np


def dev():
    import torch
    return torch.device("cuda:0")


def to_gpu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def to_cpu(t):
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def announce(*what):
    """Print (and flush) which case is about to run on the GPU."""
    print("[gpu case]", *what, flush=True)
    sys.stdout.flush()
