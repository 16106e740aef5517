"""GPU parity with a twisted mass (mu != 0): D = A - kappa H with the
site-diagonal A = 1 + 2 i kappa mu g5, its Schur complement on the odd sites
S = A - kappa^2 H_oe A^-1 H_eo (and the daggers), the source and reconstruction
maps, and every solver form, against the complex128 oracle.  Bars as for mu = 0:
FP64 operators within 1e-12 relative and of the largest element, FP32 within
2e-6 relative and 5e-6 of the largest element on the oracle applied to the same
rounded inputs, solves to the requested true residual of the oracle's
own D."""
import numpy as np
import pytest
import torch

import latgen
from oracle import solvers as S, storage, wilson as W
import paper_1401_2039_amd as q
from gpu_util import say, dev, host, parity_rel, parity_maxabs

pytestmark = pytest.mark.gpu

MU = 0.35


@pytest.fixture(scope="module", params=[(4, 4, 4, 4), (6, 4, 2, 4)], ids=lambda d: "x".join(map(str, d)))
def tm(request):
    dims = request.param
    say("twisted setup", dims)
    cfg = latgen.small_config(dims, seed=60, kind="expih", eps=0.4, nrhs=2)
    lat = q.Lattice(dims, 0.12, cfg["U"], mu=MU)
    return dims, cfg, lat


@pytest.mark.parametrize("prec", [q.F64, q.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("op", [q.OP_D, q.OP_DDAG, q.OP_SCHUR, q.OP_SCHUR_DAG], ids=["D", "Ddag", "S", "Sdag"])
def test_apply_M_twisted(tm, op, prec):
    dims, cfg, lat = tm
    say("twisted apply_M", dims, op, prec)
    U, k = cfg["U"], 0.12
    if prec == q.F64:
        Ur, br, bar, ebar = U, cfg["b"], 1e-12, 1e-12
    else:
        Ur, br, bar, ebar = storage.round_links_r12(U, np.complex64), storage.round_f32(cfg["b"]), 2e-6, 5e-6
    if op in (q.OP_D, q.OP_DDAG):
        inp = lat.import_field(dev(cfg["b"]), q.FULL, prec)
        out = lat.field(q.FULL, prec, nrhs=2)
        lat.apply_M(out, inp, None, op, prec, nrhs=2)
        got = host(lat.export_field(out, q.FULL, prec, nrhs=2))
        for r in range(2):
            want = (W.apply_D if op == q.OP_D else W.apply_Ddag)(Ur, k, MU, br[r])
            assert np.sqrt(W.norm2(got[r] - want) / W.norm2(want)) < bar
            assert np.abs(got[r] - want).max() < ebar * np.abs(want).max()
    else:
        inp = lat.import_field(dev(cfg["b"]), q.ODD, prec)
        out = lat.field(q.ODD, prec, nrhs=2)
        tmp = lat.field(q.EVEN, prec, nrhs=2)
        lat.apply_M(out, inp, tmp, op, prec, nrhs=2)
        got = host(lat.export_field(out, q.ODD, prec, nrhs=2))
        for r in range(2):
            want = W.schur(Ur, k, MU, W.project(br[r], 1), dagger=(op == q.OP_SCHUR_DAG))
            assert parity_rel(got[r], want, 1) < bar
            assert parity_maxabs(got[r], want, 1) < ebar * np.abs(want).max()


def test_twisted_mass_changes_the_operator(tm):
    """The same links with mu = 0 give a different D (the factor is applied)."""
    dims, cfg, lat = tm
    lat0 = q.Lattice(dims, 0.12, cfg["U"])
    inp = lat.import_field(dev(cfg["b"][:1]), q.FULL, q.F64)
    outs = []
    for l in (lat, lat0):
        out = l.field(q.FULL, q.F64)
        l.apply_M(out, inp, None, q.OP_D, q.F64)
        outs.append(host(l.export_field(out, q.FULL, q.F64))[0])
    diff = np.sqrt(W.norm2(outs[0] - outs[1]) / W.norm2(outs[1]))
    want = np.sqrt(W.norm2(2j * 0.12 * MU * W.spin_mul(W.GAMMA5, cfg["b"][0])) / W.norm2(outs[1]))
    assert abs(diff - want) < 1e-12 * max(1.0, want)


@pytest.mark.parametrize("form", ["cgnr_f64", "cgnr_f32", "cgnr_f16s", "bicgstab_f64", "bicgstab_f32", "crnr_f64"])
def test_twisted_solves(tm, form):
    dims, cfg, lat = tm
    say("twisted solve", dims, form)
    kw = {"cgnr_f64": {}, "cgnr_f32": dict(inner_prec=q.F32), "cgnr_f16s": dict(inner_prec=q.F16S),
          "bicgstab_f64": dict(solver=q.BICGSTAB_EO), "bicgstab_f32": dict(solver=q.BICGSTAB_EO, inner_prec=q.F32),
          "crnr_f64": dict(solver=q.CRNR_EO)}[form]
    x, st, info = lat.solve(dev(cfg["b"]), tol=1e-10, **kw)
    assert st == 0, info
    xs = host(x)
    for r in range(2):
        assert S.true_rel_residual(cfg["U"], 0.12, MU, xs[r], cfg["b"][r]) <= 1e-10
    if form == "cgnr_f64":
        xo, inf = S.solve_eo_cgnr(cfg["U"], 0.12, MU, cfg["b"][0], tol=1e-10)
        assert abs(info[0]["iterations"] - inf["iterations"]) <= 2
        # both solutions are within the residual-allowed distance of D^-1 b
        assert np.sqrt(W.norm2(xs[0] - xo) / W.norm2(xo)) < 1e-8


def test_twisted_batch_per_system_mu():
    """An uneven batch where each system has its own kappa and mu (one of them 0)."""
    say("twisted batch")
    dimss = [(4, 4, 4, 4), (2, 2, 4, 2), (6, 4, 2, 4)]
    mus = [0.2, 0.0, 0.5]
    cfgs = [latgen.small_config(d, seed=61 + i, kind="expih", eps=0.3, kappa=0.10 + 0.01 * i) for i, d in enumerate(dimss)]
    lats = [q.Lattice(c["dims"], c["kappa"], c["U"], mu=m) for c, m in zip(cfgs, mus)]
    bs = [dev(c["b"]) for c in cfgs]
    for prec in (q.F64, q.F32):
        xs = [torch.zeros_like(b) for b in bs]
        st, info = q.qiral_solve_batch([l.handle for l in lats], dimss, xs, bs, q.solve_params(tol=1e-10, inner_prec=prec))
        assert st == 0
        for c, m, x, inf in zip(cfgs, mus, xs, info):
            assert S.true_rel_residual(c["U"], c["kappa"], m, host(x)[0], c["b"][0]) <= 1e-10
            assert inf["converged"] == 1


def test_twisted_fgmres():
    """FGMRES with the network preconditioner (Neumann-2 weights, exact for
    mu = 0 only) on a twisted-mass D still reaches the tolerance, with the
    network trained on pairs generated by the twisted operator."""
    dims = (4, 4, 4, 4)
    say("twisted fgmres")
    cfg = latgen.small_config(dims, seed=64, kind="expih", eps=0.3)
    lat = q.Lattice(dims, 0.12, cfg["U"], mu=MU)
    net = q.Network(lat, 2)
    x, st, info = lat.solve(dev(cfg["b"]), tol=1e-10, solver=q.FGMRES_NN, restart=20, maxiter=400, precond=net.handle)
    assert st == 0, info
    assert S.true_rel_residual(cfg["U"], 0.12, MU, host(x)[0], cfg["b"][0]) <= 1e-10
    net.close()
