"""Helpers for the GPU parity tests (inputs from synth, references from the
oracle only)."""

import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x):
    import torch
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda:0")


def host(t):
    return t.detach().cpu().numpy()


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
