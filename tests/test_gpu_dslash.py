"""GPU parity of the packed layouts, the hopping term H_{p,1-p} and the operators
D, D^dagger, S, S^dagger against the complex128 oracle, element by element.

Bars: FP64 within 1e-12 relative (and 1e-12 of the largest element); FP32 with
reconstruct-12 links against the oracle applied to the same rounded inputs
within 2e-6 relative and 5e-6 of the largest element, element by element; F16S against the oracle on the same rounded inputs within the FP16
quantisation of the output (2^-11 of each site's scale, plus FP32 rounding).
Sizes: 4^4 (two blocks), 2^4 and 4x2x2x4 (a block only partly filled), 6x4x2x4
(a ragged last block), and 16^3x32; 24^3x48 on sampled sites."""
import numpy as np
import pytest
import torch

import latgen
from oracle import solvers as S, storage, wilson as W
import paper_1401_2039_amd as q
from gpu_util import say, dev, host, parity_rel, parity_maxabs

pytestmark = pytest.mark.gpu

DIMS = [(4, 4, 4, 4), (2, 2, 2, 2), (4, 2, 2, 4), (6, 4, 2, 4), (16, 16, 16, 32)]


def _cfg(dims, seed=0, kind="haar"):
    return latgen.small_config(dims, seed=seed, kind=kind, eps=0.4, nrhs=2)


@pytest.fixture(scope="module", params=DIMS, ids=lambda d: "x".join(map(str, d)))
def setup(request):
    dims = request.param
    say("dslash setup", dims)
    cfg = _cfg(dims, kind="expih" if dims[0] >= 16 else "haar")
    lat = q.Lattice(dims, 0.12, cfg["U"])
    return dims, cfg, lat


def test_import_export_roundtrip(setup):
    dims, cfg, lat = setup
    say("roundtrip", dims)
    b = dev(cfg["b"])
    for prec, rounder in ((q.F64, lambda a: a), (q.F32, storage.round_f32), (q.F16S, storage.round_f16s)):
        packed = lat.import_field(b, q.FULL, prec)
        back = host(lat.export_field(packed, q.FULL, prec, nrhs=2))
        want = rounder(cfg["b"])
        assert np.array_equal(back, want), prec   # the rounding decisions are bit-exact
        for par in (0, 1):
            half = lat.import_field(b, par, prec)
            out = lat.canon(2)
            lat.export_field(half, par, prec, nrhs=2, out=out)
            got = host(out)
            for r in range(2):
                assert np.array_equal(W.project(got[r], par), W.project(want[r], par))
                assert np.count_nonzero(W.project(got[r], 1 - par)) == 0


@pytest.mark.parametrize("prec", [q.F64, q.F32, q.F16S], ids=["f64", "f32", "f16s"])
@pytest.mark.parametrize("dag", [0, 1])
def test_dslash_eo(setup, prec, dag):
    dims, cfg, lat = setup
    say("dslash_eo", dims, prec, dag)
    U, b = cfg["U"], cfg["b"]
    if prec == q.F64:
        Ur, br = U, b
    elif prec == q.F32:
        Ur, br = storage.round_links_r12(U, np.complex64), storage.round_f32(b)
    else:
        Ur, br = storage.round_links_r12(U, "f16"), storage.round_f16s(b)
    inp = lat.import_field(dev(b), q.FULL, prec)
    hb = q.qiral_field_bytes(dims, q.EVEN, prec)
    for p in (0, 1):
        # input: the (1-p) halves of both right-hand sides, packed consecutively
        src = torch.cat([inp[r * 2 * hb + (1 - p) * hb: r * 2 * hb + (2 - p) * hb] for r in range(2)])
        out = lat.field(q.EVEN, prec, nrhs=2)
        lat.dslash_eo(out, src, p, dag, prec, nrhs=2)
        got = host(lat.export_field(out, p, prec, nrhs=2))
        for r in range(2):
            want = W.hop_eo(Ur, br[r], p, dagger=bool(dag))
            rel = parity_rel(got[r], want, p)
            if prec == q.F64:
                assert rel < 1e-12 and parity_maxabs(got[r], want, p) < 1e-12 * np.abs(want).max(), rel
            elif prec == q.F32:
                # element by element against the largest element (the FP32 sums of
                # up to 8 terms, each rounded a few times)
                assert rel < 2e-6 and parity_maxabs(got[r], want, p) < 5e-6 * np.abs(want).max(), rel
            else:
                # output quantised to FP16 with a per-site scale
                diff = np.abs(W.project(got[r], p) - want).reshape(-1, 12).max(axis=1)
                scale = np.abs(np.stack([want.real, want.imag])).reshape(2, -1, 12).max(axis=(0, 2))
                assert np.all(diff <= (2.0 ** -11) * scale * 1.01 + 1e-6 * scale.max()), diff.max()
            assert np.count_nonzero(W.project(got[r], 1 - p)) == 0


@pytest.mark.parametrize("op", [q.OP_D, q.OP_DDAG, q.OP_SCHUR, q.OP_SCHUR_DAG], ids=["D", "Ddag", "S", "Sdag"])
def test_apply_M_f64(setup, op):
    dims, cfg, lat = setup
    say("apply_M", dims, op)
    U, b, k = cfg["U"], cfg["b"][0], 0.12
    if op in (q.OP_D, q.OP_DDAG):
        inp = lat.import_field(dev(b[None]), q.FULL, q.F64)
        out = lat.field(q.FULL, q.F64)
        lat.apply_M(out, inp, None, op, q.F64)
        got = host(lat.export_field(out, q.FULL, q.F64))[0]
        want = W.apply_D(U, k, 0.0, b) if op == q.OP_D else W.apply_Ddag(U, k, 0.0, b)
        rel = np.sqrt(W.norm2(got - want) / W.norm2(want))
        assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    else:
        bo = W.project(b, 1)
        inp = lat.import_field(dev(b[None]), q.ODD, q.F64)
        out = lat.field(q.ODD, q.F64)
        tmp = lat.field(q.EVEN, q.F64)
        lat.apply_M(out, inp, tmp, op, q.F64)
        got = host(lat.export_field(out, q.ODD, q.F64))[0]
        want = W.schur(U, k, 0.0, bo, dagger=(op == q.OP_SCHUR_DAG))
        rel = parity_rel(got, want, 1)
        assert parity_maxabs(got, want, 1) < 1e-12 * np.abs(want).max()
    assert rel < 1e-12, rel


def test_dslash_sampled_24x48():
    """24^3x48 in the launch configuration of the benchmarks, checked on sampled
    sites against the oracle's single-site hop."""
    dims = (24, 24, 24, 48)
    say("dslash sampled", dims)
    cfg = latgen.make_config(2, with_source=False)
    U = cfg["U"]
    psi = latgen.gaussian_source(2, 0, dims, 1)
    lat = q.Lattice(dims, cfg["kappa"], U)
    rng = np.random.default_rng(5)
    for prec in (q.F64, q.F32):
        inp = lat.import_field(dev(psi), q.FULL, prec)
        hb = q.qiral_field_bytes(dims, q.EVEN, prec)
        Ur, pr = (U, psi[0]) if prec == q.F64 else (None, storage.round_f32(psi[0]))
        for p in (0, 1):
            out = lat.field(q.EVEN, prec)
            lat.dslash_eo(out, inp[(1 - p) * hb:(2 - p) * hb], p, 0, prec)
            got = host(lat.export_field(out, p, prec))[0]
            for _ in range(40):
                x = [int(rng.integers(0, L)) for L in dims]
                x[0] = (x[0] & ~1) | ((p + x[1] + x[2] + x[3]) & 1)
                src = W.project(pr, 1 - p)
                if prec == q.F64:
                    want = W.hop_site(U, src, tuple(x))
                    tol = 1e-12
                else:
                    # FP32 links rounded through reconstruct-12, only around this site
                    want = W.hop_site(_r12_near(U, x), src, tuple(x))
                    tol = 2e-6
                g = got[x[3], x[2], x[1], x[0]]
                assert np.abs(g - want).max() <= tol * np.abs(want).max() * 4, (prec, x)


def _r12_near(U, x):
    """Links rounded as an FP32 reconstruct-12 store on the 9 sites a hop at x reads."""
    Ur = U.copy()
    for mu in range(4):
        for dx in (0, -1):
            y = list(x)
            y[mu] = (y[mu] + dx) % U.shape[3 - mu]
            t, z, yy, xx = y[3], y[2], y[1], y[0]
            Ur[t, z, yy, xx] = storage.round_links_r12(U[t, z, yy, xx], np.complex64)
    return Ur


@pytest.mark.parametrize("prec", [q.F64, q.F32, q.F16S], ids=["f64", "f32", "f16s"])
def test_launch_shapes_multi_rhs(prec, monkeypatch):
    """Every hop launch shape (1 (F16S), 2 or 4 waves per site block, 1..4
    right-hand sides per lane, including a last group with fewer) gives the
    oracle's result; shapes a precision does not build fall back to a built one."""
    dims = (6, 4, 2, 4)
    say("launch shapes", prec)
    cfg = latgen.small_config(dims, seed=50, kind="expih", eps=0.4, nrhs=5)
    lat = q.Lattice(dims, 0.12, cfg["U"])
    U, b = cfg["U"], cfg["b"]
    if prec == q.F64:
        Ur, br = U, b
    elif prec == q.F32:
        Ur, br = storage.round_links_r12(U, np.complex64), storage.round_f32(b)
    else:
        Ur, br = storage.round_links_r12(U, "f16"), storage.round_f16s(b)
    src = lat.import_field(dev(b), q.ODD, prec)
    want = [W.hop_eo(Ur, br[r], 0) for r in range(5)]
    for t in (1, 2, 4):
        for nr in (1, 2, 3, 4):
            monkeypatch.setenv("QIRAL_HOP_SPLIT", str(t))
            monkeypatch.setenv("QIRAL_HOP_NR", str(nr))
            out = lat.field(q.EVEN, prec, nrhs=5)
            lat.dslash_eo(out, src, 0, 0, prec, nrhs=5)
            got = host(lat.export_field(out, 0, prec, nrhs=5))
            for r in range(5):
                bar = {q.F64: 1e-12, q.F32: 2e-6, q.F16S: 2e-3}[prec]
                assert parity_rel(got[r], want[r], 0) < bar, (t, nr, r)
                # element by element: F16S stores the output to half an FP16 ulp of its site's scale
                ebar = {q.F64: 1e-12, q.F32: 5e-6, q.F16S: 1e-3}[prec]
                assert parity_maxabs(got[r], want[r], 0) < ebar * np.abs(want[r]).max(), (t, nr, r)


def test_tune_and_tuned_solve(tmp_path, monkeypatch):
    dims = (8, 8, 8, 8)
    say("tune")
    monkeypatch.setenv("QIRAL_TUNE_CACHE", str(tmp_path / "tune.json"))
    cfg = latgen.small_config(dims, seed=51, kind="expih", eps=0.3, nrhs=4)
    lat = q.Lattice(dims, 0.12, cfg["U"])
    t, nr, us = lat.tune(q.F32, 4)
    assert t in (2, 4) and 1 <= nr <= 4 and us > 0
    assert (tmp_path / "tune.json").exists()
    lat2 = q.Lattice(dims, 0.12, cfg["U"])
    t2, nr2, us2 = lat2.tune(q.F32, 4)   # served from the cache
    assert (t2, nr2, us2) == (t, nr, 0.0)
    x, st, info = lat2.solve(dev(cfg["b"]), tol=1e-10, inner_prec=q.F32)
    assert st == 0
    for r in range(4):
        assert S.true_rel_residual(cfg["U"], 0.12, 0.0, host(x)[r], cfg["b"][r]) <= 1e-10


def test_f16s_tiny_scales():
    """Sites whose largest component is an FP32 denormal (far from a point source)
    go through the F16S hop output without overflow."""
    dims = (4, 4, 2, 4)
    say("f16s tiny scales")
    cfg = latgen.small_config(dims, seed=52, kind="expih", eps=0.4)
    b = cfg["b"].copy()
    b[0, :2] *= 1e-41    # two t-slices with denormal magnitudes
    b[0, 2] *= 1e-30
    lat = q.Lattice(dims, 0.12, cfg["U"])
    br = storage.round_f16s(b)
    src = lat.import_field(dev(b), q.ODD, q.F16S)
    out = lat.field(q.EVEN, q.F16S)
    lat.dslash_eo(out, src, 0, 0, q.F16S)
    got = host(lat.export_field(out, 0, q.F16S))[0]
    assert np.all(np.isfinite(got))
    want = W.hop_eo(storage.round_links_r12(cfg["U"], "f16"), br[0], 0)
    diff = np.abs(W.project(got, 0) - want).reshape(-1, 12).max(axis=1)
    scale = np.abs(np.stack([want.real, want.imag])).reshape(2, -1, 12).max(axis=(0, 2))
    assert np.all(diff <= (2.0 ** -11) * scale * 1.01 + 1e-6 * scale), diff.max()


@pytest.mark.parametrize("prec", [q.F64, q.F32, q.F16S], ids=["f64", "f32", "f16s"])
@pytest.mark.parametrize("dims,orders", [((8, 16, 8, 8), ("2", "4")), ((12, 4, 16, 4), ("8",))],
                         ids=["planes", "chunks"])
def test_block_order_bitwise(prec, monkeypatch, dims, orders):
    """The z-tiled block order visits every block once: hop outputs equal those
    of the plain order bit for bit, for one and for three right-hand sides (a
    last group with fewer; traversal tiles of 5 blocks), forward and dagger.
    8x16x8x8: a z-plane is one 64-site block (tiles of 2 and 4 planes);
    12x4x16x4: a plane is 24 sites, so chunks of 8 planes (3 blocks)."""
    say("block order", prec, dims)
    cfg = latgen.small_config(dims, seed=53, kind="expih", eps=0.4, nrhs=3)
    lat = q.Lattice(dims, 0.12, cfg["U"])
    src = lat.import_field(dev(cfg["b"]), q.ODD, prec)
    monkeypatch.setenv("QIRAL_HOP_TILE", "5")
    for nrhs in (1, 3):
        for dag in (0, 1):
            outs = []
            for order in ("0",) + tuple(orders):
                monkeypatch.setenv("QIRAL_HOP_ORDER", order)
                out = lat.field(q.EVEN, prec, nrhs=nrhs)
                out.fill_(0xFF)   # NaN patterns where a block were skipped
                lat.dslash_eo(out, src[: out.numel()], 0, dag, prec, nrhs=nrhs)
                outs.append(out)
            assert all(torch.equal(outs[0], o) for o in outs[1:]), (nrhs, dag)
    # and the z-tiled order is the oracle's result
    monkeypatch.setenv("QIRAL_HOP_ORDER", orders[0])
    out = lat.field(q.EVEN, q.F64, nrhs=1)
    lat.dslash_eo(out, lat.import_field(dev(cfg["b"][:1]), q.ODD, q.F64), 0, 0, q.F64)
    got = host(lat.export_field(out, 0, q.F64))[0]
    want = W.hop_eo(cfg["U"], cfg["b"][0], 0)
    assert parity_rel(got, want, 0) < 1e-12
