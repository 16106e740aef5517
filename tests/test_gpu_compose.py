"""Solver x system x preconditioner compositions on the GPU (qiral_solve with
params.system and params.precond) against the oracle's compositions
(oracle/compose.py) on the same inputs.

Each composition -- FGMRES(20), right-preconditioned BiCGStab and FCG(1) on the
normal equations; on D or on the odd-site Schur system; with the network
(created with the Neumann-2 weights, run in FP32) or with no preconditioner;
and CGNR on the full system -- must reach 1e-10 under the oracle's own D
(judged from the exported x) and take the oracle composition's iteration
count: BiCGStab exactly without a preconditioner (FP64 throughout), FCG within
one step and FGMRES within one step per restart cycle (their stopping tests
differ from the oracle's by that much), and two more with the FP32 network.  Lattices: 4^4 Haar (kappa 0.12) and the ragged 6x4x2x4 with
exp(0.4 i H) links and a twisted mass mu = 0.35."""
import numpy as np
import pytest

import latgen
from oracle import compose as C, ptc, solvers as S
import paper_1401_2039_amd as q
from gpu_util import say, dev, host

pytestmark = pytest.mark.gpu

SOLVERS = {"fgmres": q.FGMRES_NN, "bicgstab": q.BICGSTAB_EO, "fcg": q.FCG_NN}
SYSTEMS = {"full": q.SYSTEM_FULL, "schur": q.SYSTEM_SCHUR}


@pytest.fixture(scope="module", params=["c0", "ragged_tm"])
def lattice(request):
    if request.param == "c0":
        cfg = latgen.make_config(0)
        U, k, mu, b = cfg["U"], cfg["kappa"], 0.0, cfg["b"]
    else:
        cfg = latgen.small_config((6, 4, 2, 4), seed=95, kind="expih", eps=0.4, nrhs=1)
        U, k, mu, b = cfg["U"], 0.12, 0.35, cfg["b"]
    say("compose setup", request.param)
    lat = q.Lattice(U.shape[3::-1], k, U, mu=mu)
    net = q.Network(lat, 8)   # the Neumann-2 weights
    w = ptc.neumann2_weights(k)
    yield dict(U=U, k=k, mu=mu, b=b, lat=lat, net=net, w=w)
    net.close()
    lat.close()


@pytest.mark.parametrize("solver", list(SOLVERS))
@pytest.mark.parametrize("system", list(SYSTEMS))
@pytest.mark.parametrize("with_net", [False, True], ids=["none", "net"])
def test_composition(lattice, solver, system, with_net):
    L = lattice
    U, k, mu, b = L["U"], L["k"], L["mu"], L["b"][0]
    say("compose", solver, system, with_net)
    w = L["w"]
    M = (lambda v: ptc.network(U, w, v)) if with_net else None
    Md = (lambda v: ptc.network_adjoint(U, w, v)) if with_net else None
    xo, io = C.solve(U, k, mu, b, solver, system, M, Md, tol=1e-10, m=20, maxiter=2000)
    x, st, info = L["lat"].solve(dev(L["b"]), tol=1e-10, solver=SOLVERS[solver], system=SYSTEMS[system],
                                 precond=L["net"].handle if with_net else None, restart=20, maxiter=2000,
                                 fallback_cg=0)
    assert st == 0 and info[0]["converged"] == 1 and info[0]["fell_back"] == 0, info[0]
    xg = host(x)[0]
    res = S.true_rel_residual(U, k, mu, xg, b)
    assert res <= 1e-10, res
    assert abs(res - info[0]["true_rel_resid"]) <= 1e-3 * res + 1e-16
    # FP64 BiCGStab follows the oracle's iterates; FCG stops on its updated
    # residual (the oracle on the recomputed one), one step either way; FGMRES
    # closes each restart cycle at half the target with classical Gram-Schmidt
    # (the oracle: at the target, modified Gram-Schmidt), one step per cycle;
    # the FP32 network adds two more
    cycles = 1 + io["iterations"] // 20 if solver == "fgmres" else 1
    slack = (2 if with_net else 0) + (0 if solver == "bicgstab" else cycles)
    assert abs(info[0]["iterations"] - io["iterations"]) <= slack, (info[0]["iterations"], io["iterations"])
    assert np.sqrt(np.vdot(xg - xo, xg - xo).real / np.vdot(xo, xo).real) < 1e-8


def test_cgnr_on_the_full_system(lattice):
    """CGNR on D^dagger D x = D^dagger b: the oracle's CGNR iterates (FP64)."""
    L = lattice
    U, k, mu, b = L["U"], L["k"], L["mu"], L["b"][0]
    say("cgnr full system")
    from oracle import wilson as W
    D = lambda v: W.apply_D(U, k, mu, v)
    Dd = lambda v: W.apply_Ddag(U, k, mu, v)
    lim = (1e-10 * np.sqrt(W.norm2(b)))
    xo, io, _ = S.fcg(lambda v: Dd(D(v)), Dd(b), lambda r: r, maxiter=2000,
                      done=lambda z: np.sqrt(W.norm2(b - D(z))) <= lim)
    x, st, info = L["lat"].solve(dev(L["b"]), tol=1e-10, solver=q.CGNR_EO, system=q.SYSTEM_FULL, maxiter=2000,
                                 fallback_cg=0)
    assert st == 0 and info[0]["converged"] == 1
    # it stops on the updated residual, the oracle here on the recomputed one
    assert abs(info[0]["iterations"] - io) <= 1, (info[0]["iterations"], io)
    assert S.true_rel_residual(U, k, mu, host(x)[0], b) <= 1e-10


@pytest.mark.parametrize("solver", ["bicgstab", "fcg"])
@pytest.mark.parametrize("steps", [1, 2])
def test_schur_network_iterates(lattice, solver, steps):
    """On the Schur system the network's path-pair products run on bf16 matrix
    cores (hi and lo parts, three products); BiCGStab applies it, FCG applies it
    and its adjoint.  Stopped after `steps` iterations, x equals the oracle
    composition's iterate with the FP64 network to the precision of that split."""
    L = lattice
    U, k, mu, b = L["U"], L["k"], L["mu"], L["b"][0]
    say("schur network iterates", solver, steps)
    w = L["w"]
    xo, io = C.solve(U, k, mu, b, solver, "schur", lambda v: ptc.network(U, w, v),
                     lambda v: ptc.network_adjoint(U, w, v), tol=1e-10, m=20, maxiter=steps)
    assert io["iterations"] == steps
    x, st, info = L["lat"].solve(dev(L["b"]), tol=1e-10, solver=SOLVERS[solver], system=q.SYSTEM_SCHUR,
                                 precond=L["net"].handle, restart=20, maxiter=steps, fallback_cg=0)
    assert info[0]["iterations"] == steps and info[0]["converged"] == 0, info[0]
    xg = host(x)[0]
    rel = np.sqrt(np.vdot(xg - xo, xg - xo).real / np.vdot(xo, xo).real)
    say("  relative difference", rel)
    assert rel < 1e-5, rel


@pytest.mark.parametrize("system,with_net", [("full", False), ("full", True), ("schur", True)],
                         ids=["full-none", "full-net", "schur-net"])
def test_bicgstab_lockstep_equals_one_by_one(lattice, system, with_net):
    """The preconditioned and the full-system BiCGStab solve several right-hand
    sides in lockstep (one launch of each vector step for all, the Schur
    operator's hops on all at once); each takes the iterates it takes alone, bit
    for bit."""
    import torch
    L = lattice
    say("bicgstab lockstep", system, with_net)
    b1 = L["b"][0]
    rng = np.random.default_rng(7)
    extra = rng.standard_normal((2,) + b1.shape) + 1j * rng.standard_normal((2,) + b1.shape)
    B = np.concatenate([b1[None], extra])
    kw = dict(tol=1e-10, solver=q.BICGSTAB_EO, system=SYSTEMS[system],
              precond=L["net"].handle if with_net else None, restart=20, maxiter=2000, fallback_cg=0)
    x3, st3, info3 = L["lat"].solve(dev(B), **kw)
    x3 = x3.clone()
    assert st3 == 0 and all(i["converged"] == 1 for i in info3), info3
    for r in range(3):
        x1, st1, info1 = L["lat"].solve(dev(B[r:r + 1]), **kw)
        assert st1 == 0
        assert info1[0]["iterations"] == info3[r]["iterations"], (r, info1[0], info3[r])
        assert info1[0]["true_rel_resid"] == info3[r]["true_rel_resid"], (r, info1[0], info3[r])
        assert torch.equal(x3[r:r + 1], x1), r


def test_bicgstab_lockstep_from_a_guess(lattice):
    """Lockstep BiCGStab on the Schur system with the network, started from a
    guess (the initial residual then takes the operator's hops for all systems
    at once): each system again equals its own solve bit for bit, and reaches
    1e-10 under the oracle's D."""
    import torch
    L = lattice
    say("bicgstab lockstep from a guess")
    b1 = L["b"][0]
    rng = np.random.default_rng(11)
    extra = rng.standard_normal((2,) + b1.shape) + 1j * rng.standard_normal((2,) + b1.shape)
    B = np.concatenate([b1[None], extra])
    X0 = 0.1 * (rng.standard_normal(B.shape) + 1j * rng.standard_normal(B.shape))
    kw = dict(tol=1e-10, solver=q.BICGSTAB_EO, system=q.SYSTEM_SCHUR, precond=L["net"].handle, maxiter=2000,
              fallback_cg=0, x0_is_guess=1)
    x3, st3, info3 = L["lat"].solve(dev(B), x_canon=dev(X0), **kw)
    x3 = x3.clone()
    assert st3 == 0 and all(i["converged"] == 1 for i in info3), info3
    for r in range(3):
        x1, st1, info1 = L["lat"].solve(dev(B[r:r + 1]), x_canon=dev(X0[r:r + 1]), **kw)
        assert st1 == 0
        assert info1[0]["iterations"] == info3[r]["iterations"], (r, info1[0], info3[r])
        assert info1[0]["true_rel_resid"] == info3[r]["true_rel_resid"], (r, info1[0], info3[r])
        assert torch.equal(x3[r:r + 1], x1), r
        assert S.true_rel_residual(L["U"], L["k"], L["mu"], host(x3)[r], B[r]) <= 1e-10


def test_bicgstab_lockstep_many_systems(lattice):
    """70 right-hand sides in lockstep (more than one 64-thread group of the
    per-system scalar kernels): systems on either side of that boundary equal
    their solves alone bit for bit, and every system converges."""
    import torch
    L = lattice
    say("bicgstab lockstep, 70 systems")
    rng = np.random.default_rng(17)
    b1 = L["b"][0]
    B = rng.standard_normal((70,) + b1.shape) + 1j * rng.standard_normal((70,) + b1.shape)
    kw = dict(tol=1e-10, solver=q.BICGSTAB_EO, system=q.SYSTEM_SCHUR, precond=L["net"].handle, maxiter=2000,
              fallback_cg=0)
    x70, st, info = L["lat"].solve(dev(B), **kw)
    x70 = x70.clone()
    assert st == 0 and all(i["converged"] == 1 for i in info), [i for i in info if not i["converged"]][:3]
    for r in (0, 63, 64, 69):
        x1, st1, info1 = L["lat"].solve(dev(B[r:r + 1]), **kw)
        assert st1 == 0 and info1[0]["iterations"] == info[r]["iterations"], (r, info1[0], info[r])
        assert info1[0]["true_rel_resid"] == info[r]["true_rel_resid"], r
        assert torch.equal(x70[r:r + 1], x1), r
    assert S.true_rel_residual(L["U"], L["k"], L["mu"], host(x70)[69], B[69]) <= 1e-10


def test_bicgstab_lockstep_larger_lattice():
    """The same on 12^3x16 (216 site blocks): large enough that the per-system
    state sits past the partial sums of a full-field norm."""
    import torch
    dims = (12, 12, 12, 16)
    say("bicgstab lockstep", dims)
    cfg = latgen.small_config(dims, seed=41, kind="expih", eps=0.4, nrhs=3)
    lat = q.Lattice(dims, 0.12, cfg["U"])
    net = q.Network(lat, 8)
    kw = dict(tol=1e-10, solver=q.BICGSTAB_EO, system=q.SYSTEM_SCHUR, precond=net.handle, maxiter=2000, fallback_cg=0)
    x3, st3, info3 = lat.solve(dev(cfg["b"]), **kw)
    x3 = x3.clone()
    assert st3 == 0, info3
    for r in range(3):
        x1, st1, info1 = lat.solve(dev(cfg["b"][r:r + 1]), **kw)
        assert st1 == 0 and info1[0]["iterations"] == info3[r]["iterations"]
        assert info1[0]["true_rel_resid"] == info3[r]["true_rel_resid"], r
        assert torch.equal(x3[r:r + 1], x1), r
        assert S.true_rel_residual(cfg["U"], 0.12, 0.0, host(x3)[r], cfg["b"][r]) <= 1e-10
    net.close()
    lat.close()
