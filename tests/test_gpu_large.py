"""The paper's largest lattice, 64^3x128 (33.5 M sites, 19.3 GB of FP64 links),
on one GPU, in the launch configuration the benchmarks time at that size
(streaming accesses, z-tiled block order, XCD remap).

The links are the 32^3x64 exp(0.3 i H) links tiled 2x2x2x2 (a periodic tiling,
so every link is still an exp(0.3 i H) draw); the source is drawn on the device.
The oracle cannot apply D to the whole lattice in seconds, so outputs are
checked on sampled sites against its single-site hop, with the bars of the
small-lattice tests: FP64 within 1e-12 of the site's largest element; FP32 with
reconstruct-12 links against the oracle applied to the same rounded inputs
within 2e-6 of it; F16S within the FP16 quantisation of the output (2^-11 of
the site's scale) plus FP32 rounding.  A mixed-precision solve is judged by
the oracle's full residual b - D x on two whole time slices, each held to a
few times its share of the residual budget."""
import numpy as np
import pytest
import torch

import latgen
from oracle import storage, wilson as W
import paper_1401_2039_amd as q
from gpu_util import say

pytestmark = pytest.mark.gpu

NSAMPLE = 16


class Tiled:
    """Read-only view of the periodic tiling of a cell of links."""

    def __init__(self, u, cell_dims):
        self.u, self.c = u, cell_dims

    def __getitem__(self, i):
        t, z, y, x = i[0] % self.c[3], i[1] % self.c[2], i[2] % self.c[1], i[3] % self.c[0]
        return self.u[(t, z, y, x) + tuple(i[4:])]


class DevSites:
    """A canonical device field read one site at a time, optionally rounded as
    a storage class holds it."""

    def __init__(self, f, rnd=None):
        self.f, self.shape, self.rnd = f, tuple(f.shape), rnd

    def __getitem__(self, i):
        v = self.f[i].cpu().numpy()
        return self.rnd(v) if self.rnd else v


@pytest.fixture(scope="module")
def big():
    say("64^3x128 setup")
    cfg = latgen.tiled_config()
    dims, reps = cfg["dims"], cfg["reps"]
    cell = torch.from_numpy(cfg["U_cell"]).cuda()
    U = cell.repeat(reps[3], reps[2], reps[1], reps[0], 1, 1, 1)
    del cell
    lat = q.Lattice(dims, cfg["kappa"], U)
    del U
    b = latgen.device_gaussian_source(100, 0, dims, 1)
    torch.cuda.synchronize()
    yield cfg, lat, b
    lat.close()


def _sites(rng, dims, p, n):
    out = []
    for _ in range(n):
        x = [int(rng.integers(0, L)) for L in dims]
        x[0] = (x[0] & ~1) | ((p + x[1] + x[2] + x[3]) & 1)
        out.append(tuple(x))
    return out


@pytest.mark.parametrize("prec", [q.F64, q.F32, q.F16S], ids=["f64", "f32", "f16s"])
def test_hop_64x128_sampled(big, prec):
    cfg, lat, b = big
    dims = cfg["dims"]
    say("hop 64^3x128 sampled", prec)
    if prec == q.F64:
        Uo, rnd = Tiled(cfg["U_cell"], cfg["cell_dims"]), None
    elif prec == q.F32:
        Uo, rnd = Tiled(storage.round_links_r12(cfg["U_cell"], np.complex64), cfg["cell_dims"]), storage.round_f32
    else:
        Uo, rnd = Tiled(storage.round_links_r12(cfg["U_cell"], "f16"), cfg["cell_dims"]), storage.round_f16s
    src_all = lat.import_field(b, q.FULL, prec)
    hb = q.qiral_field_bytes(dims, q.EVEN, prec)
    rng = np.random.default_rng(128 + prec)
    for p, dag in ((0, 0), (1, 1)):
        out = lat.field(q.EVEN, prec)
        lat.dslash_eo(out, src_all[(1 - p) * hb:(2 - p) * hb], p, dag, prec)
        got = lat.export_field(out, p, prec)
        del out
        # the 8 neighbours of a site of parity p have parity 1 - p, so the
        # whole source stands for its (1 - p) half
        psi = DevSites(b[0], rnd)
        for x in _sites(rng, dims, p, NSAMPLE):
            want = W.hop_site(Uo, psi, x, dagger=bool(dag))
            g = got[0, x[3], x[2], x[1], x[0]].cpu().numpy()
            err = np.abs(g - want).max()
            if prec == q.F64:
                assert err <= 1e-12 * np.abs(want).max(), (x, err)
            elif prec == q.F32:
                assert err <= 2e-6 * np.abs(want).max(), (x, err)
            else:
                scale = np.abs(np.stack([want.real, want.imag])).max()
                assert err <= (2.0 ** -11) * scale * 1.01 + 1e-6 * scale, (x, err, scale)
        del got
    del src_all


def _slab_links(cfg, t0):
    """Links of the t-slices t0 - 1, t0, t0 + 1 of the tiled lattice, as a
    lattice of 3 time slices [3][Lz][Ly][Lx][4][3][3]."""
    cell, cd, reps = cfg["U_cell"], cfg["cell_dims"], cfg["reps"]
    lt = cfg["dims"][3]
    return np.stack([np.tile(cell[(t % lt) % cd[3]], (reps[2], reps[1], reps[0], 1, 1, 1))
                     for t in (t0 - 1, t0, t0 + 1)])


def test_solve_64x128_f16s_slab_residual(big):
    """F16S mixed-precision even-odd CGNR to 1e-10 on the whole lattice; the
    oracle recomputes b - D x on two whole time slices (both parities).  On a
    periodic lattice of the 3 slices t0 - 1, t0, t0 + 1 the hop at slice t0 is
    exactly the full lattice's, so the residual there is exact.  A Gaussian
    source spreads the residual over the lattice, so each slice's share of
    ||b - D x||^2 is about 1/Lt of it: the bar is 16/Lt of the whole budget
    (tol ||b||)^2 per slice, 4x the fair share in norm."""
    cfg, lat, b = big
    dims, kappa, tol = cfg["dims"], cfg["kappa"], 1e-10
    say("solve 64^3x128 f16s")
    x, st, info = lat.solve(b, tol=tol, inner_prec=q.F16S)
    torch.cuda.synchronize()
    assert st == 0 and info[0]["converged"] and info[0]["true_rel_resid"] <= tol, info[0]
    bnorm = float(torch.linalg.vector_norm(b).item())
    lt = dims[3]
    for t0 in (0, 77):
        say("oracle residual on slice", t0)
        idx = [(t0 - 1) % lt, t0, (t0 + 1) % lt]
        xs = x[0, idx].cpu().numpy()
        bs = b[0, t0].cpu().numpy()
        Hx = W.hop(_slab_links(cfg, t0), xs)[1]
        r = bs - (xs[1] - kappa * Hx)
        share = np.sqrt(np.sum(np.abs(r) ** 2)) / (tol * bnorm)
        assert share <= np.sqrt(16.0 / lt), (t0, share)
        # and not vacuous: the slice holds a real part of the residual budget
        assert share > 0
