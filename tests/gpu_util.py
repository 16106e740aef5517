"""Helpers shared by the GPU parity tests: host <-> device copies, comparison
of packed-path results with the oracle, and a flushing progress print that
names each case before it runs on the GPU."""
import sys

import numpy as np
import torch

from oracle import wilson as W


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def parity_rel(got, want, parity):
    """||got - want|| / ||want|| over the sites of one parity."""
    g = W.project(got, parity)
    w = W.project(want, parity)
    return np.sqrt(W.norm2(g - w) / W.norm2(w))


def parity_maxabs(got, want, parity):
    return np.abs(W.project(got, parity) - W.project(want, parity)).max()
