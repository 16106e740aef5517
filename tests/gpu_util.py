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


class DevSites:
    """A canonical device field read one site at a time (for the oracle's
    single-site hop on lattices too large to copy), optionally rounded as a
    storage class holds it."""

    def __init__(self, f, rnd=None):
        self.f, self.shape, self.rnd = f, tuple(f.shape), rnd

    def __getitem__(self, i):
        v = self.f[i].cpu().numpy()
        return self.rnd(v) if self.rnd else v


class RoundedLinks:
    """Links as a reduced-precision reconstruct-12 store holds them, rounded on
    access (the oracle's single-site hop reads 8 of them)."""

    def __init__(self, U, dtype):
        from oracle import storage
        self.U, self.dtype, self.shape, self._r = U, dtype, U.shape, storage.round_links_r12

    def __getitem__(self, i):
        return self._r(self.U[i], self.dtype)


def sampled_sites(rng, dims, parity, n):
    """n random sites (x, y, z, t) of the given parity."""
    out = []
    for _ in range(n):
        x = [int(rng.integers(0, L)) for L in dims]
        x[0] = (x[0] & ~1) | ((parity + x[1] + x[2] + x[3]) & 1)
        out.append(tuple(x))
    return out
