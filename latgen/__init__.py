"""Seeded synthetic inputs for the Wilson-Dirac solves: gauge links and sources.

This module is the only code shared by the CPU oracle (``oracle/``) and the
GPU path (``paper_1401_2039_amd``).  It draws random numbers and builds the
input arrays in the canonical layout; it holds none of the operator or solver
arithmetic.

Canonical layouts (the paper leaves layout open at the DSL level, Sec. 2; the
index-set product L x C x S of the goal statement fixes the order used here):

* gauge links ``U[t][z][y][x][mu][a][b]``, complex128, ``mu = 0..3 = x, y, z, t``;
  ``U[..., mu, :, :]`` is the SU(3) link from site x to x + mu_hat.
* spinors ``psi[rhs][t][z][y][x][colour][spin]``, complex128, spin fastest
  (a site's 12 components form a 3 x 4 colour-by-spin matrix, the form used by
  the Kronecker identity of Sec. 4.2).

Random streams: ``numpy.random.default_rng(SeedSequence([1401, 2039, cid, sys,
stream]))`` with stream 0 = gauge, 1 = source, 2 = point-source site,
3 = per-system (eps, kappa), 4 = training keys.  Draws fill arrays in canonical
order; a complex Gaussian number is ``re + 1j * im`` with re, im ~ N(0, 1).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = (1401, 2039)
STREAM_GAUGE, STREAM_SOURCE, STREAM_POINT, STREAM_SYSPARAM, STREAM_TRAIN = 0, 1, 2, 3, 4

# Lattice dims are (Lx, Ly, Lz, Lt); a "24^3 x 48" lattice has Lt = 48.
CONFIG_DIMS = {
    0: [(4, 4, 4, 4)],
    1: [(16, 16, 16, 32)],
    2: [(24, 24, 24, 48)],
    3: [(8, 8, 8, 8)] * 8 + [(12, 12, 12, 24)] * 8 + [(16, 16, 16, 32)] * 8 + [(20, 20, 20, 40)] * 8,
    4: [(24, 24, 24, 48)],
    99: [(32, 32, 32, 64)],
    100: [(64, 64, 64, 128)],
}


def rng(cid: int, sys: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([*SEED_BASE, cid, sys, stream]))


def site_shape(dims) -> tuple:
    lx, ly, lz, lt = dims
    return (lt, lz, ly, lx)


def complex_gaussian(g: np.random.Generator, shape) -> np.ndarray:
    r = g.standard_normal(tuple(shape) + (2,))
    return r[..., 0] + 1j * r[..., 1]


def haar_su3(g: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-random SU(3) matrices (Mezzadri 2007: QR of a complex Gaussian,
    phases of R's diagonal moved into Q, then division by the principal cube
    root of det Q)."""
    z = complex_gaussian(g, (n, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[:, None, None]


def _expih_chunk(a, eps):
    h = 0.5 * (a + np.conj(np.swapaxes(a, 1, 2)))
    tr = np.trace(h, axis1=1, axis2=2).real / 3.0
    h = h - tr[:, None, None] * np.eye(3)
    w, v = np.linalg.eigh(h)
    return (v * np.exp(1j * eps * w)[:, None, :]) @ np.conj(np.swapaxes(v, 1, 2))


def expih_su3(g: np.random.Generator, n: int, eps, chunk: int = 1 << 16) -> np.ndarray:
    """n links U = exp(i eps H), H a traceless Hermitian 3x3 built from a complex
    Gaussian A as H = (A + A^dagger)/2 - tr/3; the exponential is taken through
    the eigen-decomposition of H.  ``eps`` is a scalar.  The random numbers are
    drawn in one stream; the per-matrix decompositions run on a thread pool
    (NumPy's linalg releases the GIL), which does not change any value."""
    import concurrent.futures
    import os
    a = complex_gaussian(g, (n, 3, 3))
    out = np.empty_like(a)
    starts = list(range(0, n, chunk))

    def work(s0):
        out[s0:s0 + chunk] = _expih_chunk(a[s0:s0 + chunk], eps)

    nthr = max(1, min(16, len(os.sched_getaffinity(0)), len(starts)))
    if nthr == 1:
        for s0 in starts:
            work(s0)
    else:
        with concurrent.futures.ThreadPoolExecutor(nthr) as ex:
            list(ex.map(work, starts))
    return out


def gauge_field(cid: int, sys: int, dims, kind: str, eps: float | None = None) -> np.ndarray:
    shp = site_shape(dims) + (4,)
    n = int(np.prod(shp))
    g = rng(cid, sys, STREAM_GAUGE)
    if kind == "haar":
        u = haar_su3(g, n)
    elif kind == "expih":
        u = expih_su3(g, n, eps)
    elif kind == "unit":
        u = np.broadcast_to(np.eye(3, dtype=np.complex128), (n, 3, 3)).copy()
    else:
        raise ValueError(kind)
    return u.reshape(shp + (3, 3))


def gaussian_source(cid: int, sys: int, dims, nrhs: int = 1) -> np.ndarray:
    g = rng(cid, sys, STREAM_SOURCE)
    return complex_gaussian(g, (nrhs,) + site_shape(dims) + (3, 4))


def point_site(cid: int, sys: int, dims) -> tuple:
    """Seeded site (x, y, z, t), one uniform integer per axis in x, y, z, t order."""
    g = rng(cid, sys, STREAM_POINT)
    return tuple(int(g.integers(0, L)) for L in dims)


def point_sources(cid: int, sys: int, dims) -> np.ndarray:
    """12 point sources at one seeded site, b_k = delta_{x,x0} e_(c,s), k = 4c + s."""
    x, y, z, t = point_site(cid, sys, dims)
    b = np.zeros((12,) + site_shape(dims) + (3, 4), dtype=np.complex128)
    for c in range(3):
        for s in range(4):
            b[4 * c + s, t, z, y, x, c, s] = 1.0
    return b


def system_params(cid: int, sys: int) -> tuple:
    """(eps, kappa) of one system of the uneven batch: eps ~ U[0.2, 0.5],
    kappa ~ U[0.10, 0.12]."""
    g = rng(cid, sys, STREAM_SYSPARAM)
    eps = float(g.uniform(0.2, 0.5))
    kappa = float(g.uniform(0.10, 0.12))
    return eps, kappa


def make_config(cid: int, sys: int = 0, with_source: bool = True) -> dict:
    """Inputs of one synthetic workload.

    0: 4^4 Haar links, kappa 0.12, 1 Gaussian source.
    1: 16^3x32, exp(0.3 i H), kappa 0.12, 1 Gaussian source.
    2: 24^3x48, exp(0.4 i H), kappa 0.12, 12 point sources at one site.
    3: one of 32 systems (8 each of 8^4, 12^3x24, 16^3x32, 20^3x40), per-system
       eps ~ U[0.2,0.5], kappa ~ U[0.10,0.12], 1 Gaussian source.
    4: 24^3x48, exp(0.5 i H), kappa 0.125, 12 Gaussian sources.
    99: 32^3x64, exp(0.3 i H), kappa 0.12, 1 Gaussian source (a lattice whose
        working set exceeds the 256 MB last-level cache).
    """
    dims = CONFIG_DIMS[cid][sys if cid == 3 else 0]
    if cid == 0:
        kind, eps, kappa, nrhs = "haar", None, 0.12, 1
    elif cid in (1, 99):
        kind, eps, kappa, nrhs = "expih", 0.3, 0.12, 1
    elif cid == 2:
        kind, eps, kappa, nrhs = "expih", 0.4, 0.12, 12
    elif cid == 3:
        kind = "expih"
        eps, kappa = system_params(cid, sys)
        nrhs = 1
    elif cid == 4:
        kind, eps, kappa, nrhs = "expih", 0.5, 0.125, 12
    else:
        raise ValueError(cid)
    cfg = dict(cid=cid, sys=sys, dims=tuple(dims), kappa=kappa, mu=0.0, eps=eps, kind=kind, nrhs=nrhs)
    cfg["U"] = gauge_field(cid, sys, dims, kind, eps)
    if with_source:
        cfg["b"] = point_sources(cid, sys, dims) if cid == 2 else gaussian_source(cid, sys, dims, nrhs)
    return cfg


def tiled_config() -> dict:
    """Config 100 (measurement only): the 64^3x128 lattice of the paper's largest
    run.  Its links repeat the 32^3x64 links of config 99 twice along every axis
    (a periodic tiling of that cell, so every link is the same exp(0.3 i H) draw
    as there); kappa 0.12; one Gaussian source drawn on the whole lattice.
    Returns the cell links, the tiling and the source; the caller tiles the links
    where they are needed (19.3 GB in complex128)."""
    cell = make_config(99, with_source=False)
    dims = CONFIG_DIMS[100][0]
    reps = tuple(d // c for d, c in zip(dims, cell["dims"]))
    return dict(cid=100, sys=0, dims=dims, kappa=cell["kappa"], mu=0.0, eps=cell["eps"], kind="tiled " + cell["kind"],
                nrhs=1, U_cell=cell["U"], cell_dims=cell["dims"], reps=reps)


def device_gaussian_source(cid: int, sys: int, dims, nrhs: int = 1, device: str = "cuda"):
    """A complex Gaussian source (Re, Im ~ N(0, 1)) drawn directly in device
    memory by torch's counter-based generator, seeded from the same seed
    sequence as gaussian_source (stream 1).  For lattices whose host-side draw
    would take minutes; the values differ from gaussian_source's."""
    import torch
    seed = int(np.random.SeedSequence([*SEED_BASE, cid, sys, STREAM_SOURCE]).generate_state(1, dtype=np.uint64)[0])
    g = torch.Generator(device=device)
    g.manual_seed(seed & ((1 << 63) - 1))
    shape = (nrhs,) + site_shape(dims) + (3, 4)
    re = torch.randn(shape, generator=g, device=device, dtype=torch.float64)
    im = torch.randn(shape, generator=g, device=device, dtype=torch.float64)
    return torch.complex(re, im)


def small_config(dims, seed: int = 0, kind: str = "haar", eps: float = 0.3, kappa: float = 0.12,
                 nrhs: int = 1) -> dict:
    """A seeded test lattice of arbitrary (even) dims, drawn with cid = 1000 + seed."""
    cid = 1000 + seed
    U = gauge_field(cid, 0, dims, kind, eps)
    b = gaussian_source(cid, 0, dims, nrhs)
    return dict(cid=cid, sys=0, dims=tuple(dims), kappa=kappa, mu=0.0, eps=eps, kind=kind, nrhs=nrhs, U=U, b=b)


def random_su3_field(seed: int, dims) -> np.ndarray:
    """A Haar SU(3) matrix per site, shape [t][z][y][x][3][3] (gauge transforms in tests)."""
    g = np.random.default_rng(np.random.SeedSequence([*SEED_BASE, 7777, seed]))
    n = int(np.prod(site_shape(dims)))
    return haar_su3(g, n).reshape(site_shape(dims) + (3, 3))
