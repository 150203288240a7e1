"""Helpers shared by the GPU tests (inputs from synth, references from oracle)."""
import sys

import numpy as np


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_rows(a, b):
    """max over rows of the relative 2-norm error."""
    return float(max(np.linalg.norm(x - y) / np.linalg.norm(y) for x, y in zip(a, b)))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
