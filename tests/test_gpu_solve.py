"""GPU solves through qiral_solve / qiral_solve_batch, judged by the oracle.

Every solve must reach the requested true residual ||b - D x|| / ||b|| <= tol,
computed by the oracle's complex128 operator from the exported x; the plain
FP64 even-odd CGNR must also take the oracle's iteration count within 2 and
agree with the oracle's solution to the error the residual allows."""
import numpy as np
import pytest
import torch

import latgen
from oracle import solvers as S, wilson as W
import paper_1401_2039_amd as q
from gpu_util import say, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c0():
    say("solve setup C0")
    cfg = latgen.make_config(0)
    lat = q.Lattice(cfg["dims"], cfg["kappa"], cfg["U"])
    xo, info = S.solve_eo_cgnr(cfg["U"], cfg["kappa"], 0.0, cfg["b"][0], tol=1e-10)
    return cfg, lat, xo, info


def _resid(cfg, x, r=0):
    return S.true_rel_residual(cfg["U"], cfg["kappa"], 0.0, x, cfg["b"][r])


def test_cgnr_f64_c0(c0):
    cfg, lat, xo, oinfo = c0
    say("cgnr f64 C0")
    x, st, info = lat.solve(dev(cfg["b"]), tol=1e-10)
    xg = host(x)[0]
    assert st == 0 and info[0]["converged"] == 1
    res = _resid(cfg, xg)
    assert res <= 1e-10 and abs(res - info[0]["true_rel_resid"]) <= 1e-3 * res
    assert abs(info[0]["iterations"] - oinfo["iterations"]) <= 2
    assert np.sqrt(W.norm2(xg - xo) / W.norm2(xo)) < 1e-9


@pytest.mark.parametrize("graph", [0, 1])
def test_bicgstab_f64_c0(c0, graph):
    cfg, lat, xo, _ = c0
    say("bicgstab f64 C0 graph", graph)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        x, st, info = lat.solve(dev(cfg["b"]), tol=1e-10, solver=q.BICGSTAB_EO, use_graph=graph)
    torch.cuda.synchronize()
    assert st == 0
    assert _resid(cfg, host(x)[0]) <= 1e-10


@pytest.mark.parametrize("prec", [q.F32, q.F16S], ids=["f32", "f16s"])
@pytest.mark.parametrize("solver", [q.CGNR_EO, q.BICGSTAB_EO], ids=["cgnr", "bicgstab"])
def test_mixed_c0(c0, prec, solver):
    cfg, lat, xo, _ = c0
    say("mixed C0", prec, solver)
    x, st, info = lat.solve(dev(cfg["b"]), tol=1e-10, inner_prec=prec, solver=solver, delta=0.1)
    assert st == 0, info
    assert info[0]["reliable_updates"] >= 1
    assert _resid(cfg, host(x)[0]) <= 1e-10


def test_crnr_f64_c0(c0):
    """Conjugate residual on the Schur normal equations: the oracle's D judges the
    residual, the oracle's CR the iteration count (within 2) and the solution."""
    cfg, lat, _, _ = c0
    say("crnr f64 C0")
    x, st, info = lat.solve(dev(cfg["b"]), tol=1e-10, solver=q.CRNR_EO)
    assert st == 0, info
    xg = host(x)[0]
    assert _resid(cfg, xg) <= 1e-10
    xc, ci = S.solve_eo_crnr(cfg["U"], cfg["kappa"], 0.0, cfg["b"][0], tol=1e-10)
    assert abs(info[0]["iterations"] - ci["iterations"]) <= 2, (info[0]["iterations"], ci["iterations"])
    assert np.sqrt(W.norm2(xg - xc) / W.norm2(xc)) < 1e-9
    # 4 hops per iteration plus the start (r: 2, z, v, w: 6)
    assert info[0]["hop_applications"] == 4 * info[0]["iterations"] + 8


def test_crnr_multi_rhs_and_batch():
    say("crnr multi-rhs and batch")
    dims = (4, 4, 2, 4)
    cfg = latgen.small_config(dims, seed=32, kind="expih", eps=0.4, nrhs=3)
    lat = q.Lattice(dims, 0.12, cfg["U"])
    x, st, info = lat.solve(dev(cfg["b"]), tol=1e-10, solver=q.CRNR_EO)
    assert st == 0
    xs = host(x)
    for r in range(3):
        assert S.true_rel_residual(cfg["U"], 0.12, 0.0, xs[r], cfg["b"][r]) <= 1e-10
        x1, st1, _ = lat.solve(dev(cfg["b"][r:r + 1]), tol=1e-10, solver=q.CRNR_EO)
        assert st1 == 0 and np.array_equal(host(x1)[0], xs[r])
    dimss = [(4, 4, 4, 4), (2, 2, 4, 2), (6, 4, 2, 4)]
    cfgs = [latgen.small_config(d, seed=40 + i, kind="expih", eps=0.3, kappa=0.10 + 0.01 * i) for i, d in enumerate(dimss)]
    lats = [q.Lattice(c["dims"], c["kappa"], c["U"]) for c in cfgs]
    bs = [dev(c["b"]) for c in cfgs]
    xs = [torch.zeros_like(b) for b in bs]
    st, info = q.qiral_solve_batch([l.handle for l in lats], dimss, xs, bs, q.solve_params(tol=1e-10, solver=q.CRNR_EO))
    assert st == 0
    for c, xx in zip(cfgs, xs):
        assert S.true_rel_residual(c["U"], c["kappa"], 0.0, host(xx)[0], c["b"][0]) <= 1e-10


def test_multi_rhs_equals_single():
    dims = (4, 4, 2, 4)
    say("multi-rhs", dims)
    cfg = latgen.small_config(dims, seed=31, kind="expih", eps=0.4, nrhs=5)
    lat = q.Lattice(dims, 0.12, cfg["U"])
    for prec in (q.F64, q.F32):
        x, st, info = lat.solve(dev(cfg["b"]), tol=1e-10, inner_prec=prec)
        assert st == 0
        xs = host(x)
        for r in range(5):
            assert S.true_rel_residual(cfg["U"], 0.12, 0.0, xs[r], cfg["b"][r]) <= 1e-10
            x1, st1, _ = lat.solve(dev(cfg["b"][r:r + 1]), tol=1e-10, inner_prec=prec)
            assert st1 == 0
            if prec == q.F64:
                # same reductions in the same order: the batch solve equals the single one bit for bit
                assert np.array_equal(host(x1)[0], xs[r])


def test_batch_uneven():
    say("batch uneven")
    dimss = [(4, 4, 4, 4), (2, 2, 4, 2), (6, 4, 2, 4)]
    cfgs = [latgen.small_config(d, seed=40 + i, kind="expih", eps=0.3, kappa=0.10 + 0.01 * i) for i, d in enumerate(dimss)]
    lats = [q.Lattice(c["dims"], c["kappa"], c["U"]) for c in cfgs]
    bs = [dev(c["b"]) for c in cfgs]
    xs = [torch.zeros_like(b) for b in bs]
    for prec in (q.F64, q.F32):
        st, info = q.qiral_solve_batch([l.handle for l in lats], dimss, xs, bs, q.solve_params(tol=1e-10, inner_prec=prec))
        assert st == 0
        for c, x, inf in zip(cfgs, xs, info):
            res = S.true_rel_residual(c["U"], c["kappa"], 0.0, host(x)[0], c["b"][0])
            assert res <= 1e-10 and inf["converged"] == 1


def test_deterministic(c0):
    cfg, lat, _, _ = c0
    say("determinism")
    a, _, ia = lat.solve(dev(cfg["b"]), tol=1e-10, inner_prec=q.F32)
    b, _, ib = lat.solve(dev(cfg["b"]), tol=1e-10, inner_prec=q.F32)
    assert torch.equal(a, b) and ia[0]["iterations"] == ib[0]["iterations"]


def test_not_converged_and_nonfinite(c0):
    cfg, lat, _, _ = c0
    say("failure paths")
    x, st, info = lat.solve(dev(cfg["b"]), tol=1e-10, maxiter=1)
    assert st == q._lib.ERR_NOT_CONVERGED and info[0]["iterations"] == 1 and info[0]["true_rel_resid"] > 1e-10
    bad = cfg["b"].copy()
    bad[0, 0, 0, 0, 1, 2, 3] = np.nan
    with pytest.raises(q.QiralError) as e:
        lat.solve(dev(bad), tol=1e-10)
    assert e.value.status == q._lib.ERR_NONFINITE


def test_x0_guess(c0):
    cfg, lat, xo, _ = c0
    say("x0 guess")
    x = dev(xo[None])
    x, st, info = lat.solve(dev(cfg["b"]), x_canon=x, tol=1e-10, x0_is_guess=1)
    assert st == 0 and info[0]["iterations"] <= 2


def test_cgnr_c1_mixed_vs_f64():
    """16^3x32, exp(0.3 i H) links: FP64 eo-CGNR and the FP32 reconstruct-12 solve with
    FP64 reliable updates both reach 1e-10, judged by the oracle."""
    say("C1 solves")
    cfg = latgen.make_config(1)
    lat = q.Lattice(cfg["dims"], cfg["kappa"], cfg["U"])
    for prec in (q.F64, q.F32, q.F16S):
        x, st, info = lat.solve(dev(cfg["b"]), tol=1e-10, inner_prec=prec)
        say("C1", prec, info[0])
        assert st == 0
        assert _resid(cfg, host(x)[0]) <= 1e-10


@pytest.mark.parametrize("nr", [2, 3])
def test_batched_point_sources_split2(nr, monkeypatch):
    """Point sources (values spanning many decades) through the grouped multi-RHS
    mixed solve with 2 waves per site block and nr right-hand sides per lane."""
    dims = (8, 8, 8, 8)
    say("batched point sources", nr)
    monkeypatch.setenv("QIRAL_HOP_SPLIT", "2")
    monkeypatch.setenv("QIRAL_HOP_NR", str(nr))
    U = latgen.gauge_field(1003, 0, dims, "expih", 0.4)
    b = latgen.point_sources(1003, 0, dims)[:5]
    lat = q.Lattice(dims, 0.12, U)
    for prec in (q.F16S, q.F32):
        x, st, info = lat.solve(dev(b), tol=1e-10, inner_prec=prec)
        assert st == 0, info
        xs = host(x)
        for r in range(5):
            assert S.true_rel_residual(U, 0.12, 0.0, xs[r], b[r]) <= 1e-10


@pytest.mark.parametrize("dims,order", [((8, 16, 8, 8), "2"), ((12, 4, 16, 4), "8")], ids=["planes", "chunks"])
def test_block_order_solve_bitwise(monkeypatch, dims, order):
    """Solves whose hops run in the z-tiled block order equal those in the plain
    order bit for bit (partials are indexed by block, not by visit order); also
    where a z-plane is not a whole number of blocks (12x4x16x4: a plane is 24
    sites, 8 planes make a chunk of 3 blocks)."""
    say("block order solve", dims)
    cfg = latgen.small_config(dims, seed=54, kind="expih", eps=0.3, nrhs=3)
    lat = q.Lattice(dims, 0.12, cfg["U"])
    for prec, nrhs in ((q.F64, 1), (q.F32, 1), (q.F32, 3), (q.F16S, 3)):
        res = []
        for order in ("0", order):
            monkeypatch.setenv("QIRAL_HOP_ORDER", order)
            x, st, info = lat.solve(dev(cfg["b"][:nrhs]), tol=1e-10, inner_prec=prec)
            assert st == 0, info
            res.append((x, [i["iterations"] for i in info]))
        assert torch.equal(res[0][0], res[1][0]) and res[0][1] == res[1][1], (prec, nrhs)
    for r in range(3):
        assert S.true_rel_residual(cfg["U"], 0.12, 0.0, host(res[1][0])[r], cfg["b"][r]) <= 1e-10


@pytest.mark.parametrize("solver", [q.CGNR_EO, q.BICGSTAB_EO, q.CRNR_EO], ids=["cgnr", "bicgstab", "crnr"])
def test_zero_source(solver):
    """b = 0: the solve stops at once with x = 0 (no 0/0 in the recurrences)."""
    dims = (4, 4, 2, 4)
    say("zero source", solver)
    cfg = latgen.small_config(dims, seed=33, kind="expih", eps=0.3)
    lat = q.Lattice(dims, 0.12, cfg["U"])
    b = np.zeros_like(cfg["b"])
    for prec in ((q.F64, q.F32) if solver != q.CRNR_EO else (q.F64,)):
        x, st, info = lat.solve(dev(b), tol=1e-10, solver=solver, inner_prec=prec)
        assert st == 0 and info[0]["iterations"] == 0 and info[0]["true_rel_resid"] == 0.0
        assert np.count_nonzero(host(x)) == 0


def test_kappa_zero_is_the_identity():
    """kappa = 0 leaves D = 1 (the twisted term 2 i kappa mu g5 vanishes with it):
    the solve returns x = b after at most one iteration."""
    dims = (4, 2, 2, 4)
    say("kappa zero")
    cfg = latgen.small_config(dims, seed=34, kind="haar")
    for mu in (0.0, 0.3):
        lat = q.Lattice(dims, 0.0, cfg["U"], mu=mu)
        x, st, info = lat.solve(dev(cfg["b"]), tol=1e-12)
        assert st == 0 and info[0]["iterations"] <= 1
        want = W.apply_Ainv(0.0, mu, cfg["b"][0])
        assert np.abs(host(x)[0] - want).max() <= 1e-15 * np.abs(want).max()


def test_255_right_hand_sides():
    """The largest batch one call takes (255 systems: the work items' system field
    is 8 bits), on a 2^4 lattice; a few are compared with single solves."""
    dims = (2, 2, 2, 2)
    say("255 rhs")
    cfg = latgen.small_config(dims, seed=35, kind="expih", eps=0.4, nrhs=255)
    lat = q.Lattice(dims, 0.12, cfg["U"])
    x, st, info = lat.solve(dev(cfg["b"]), tol=1e-10)
    assert st == 0 and len(info) == 255
    xs = host(x)
    for r in (0, 31, 32, 127, 254):
        assert S.true_rel_residual(cfg["U"], 0.12, 0.0, xs[r], cfg["b"][r]) <= 1e-10
        x1, st1, _ = lat.solve(dev(cfg["b"][r:r + 1]), tol=1e-10)
        assert st1 == 0 and np.array_equal(host(x1)[0], xs[r])
    with pytest.raises(q.QiralError):
        q.qiral_solve(lat.handle, dims, torch.zeros((256,) + cfg["b"].shape[1:], dtype=torch.complex128, device="cuda"),
                      torch.zeros((256,) + cfg["b"].shape[1:], dtype=torch.complex128, device="cuda"), 256,
                      q.solve_params(tol=1e-10))


@pytest.mark.parametrize("k", [1, 6])
def test_fp64_cgnr_iterate_after_k_steps(c0, k):
    """A plain FP64 solve stopped by maxiter = k returns the CGNR iterate after k
    steps (the last x += alpha p applied after the loop): equal to the oracle's
    CGNR stopped after k steps, reconstructed the same way, to FP64 rounding."""
    cfg, lat, _, _ = c0
    say("fp64 iterate after", k)
    U, kap, b = cfg["U"], cfg["kappa"], cfg["b"][0]
    bhat = W.schur_source(U, kap, 0.0, b)
    xo, its, _ = S.cgnr(lambda v: W.schur(U, kap, 0.0, v), lambda v: W.schur(U, kap, 0.0, v, dagger=True), bhat,
                        0.0, maxiter=k)
    want = W.reconstruct_even(U, kap, 0.0, b, xo) + xo
    x, st, info = lat.solve(dev(cfg["b"]), tol=1e-10, maxiter=k)
    assert st == q._lib.ERR_NOT_CONVERGED and info[0]["iterations"] == k
    got = host(x)[0]
    assert np.sqrt(W.norm2(got - want) / W.norm2(want)) < 1e-13
