"""The caller-owned memory contract of the C ABI on the GPU, and the packed link
stores it exposes.

* The FP32 and FP16 reconstruct-12 link stores hold rows 0 and 1 of every link
  exactly as the oracle's store defines them (each real rounded once from FP64
  to the nearest FP32 / FP16), bit for bit, on the 16^3x32 exp(0.3 i H) links;
  the FP64 store holds the links unchanged.
* A workspace one byte short of qiral_solve_workspace_bytes is refused with
  QIRAL_ERR_WORKSPACE and leaves x untouched; one of exactly that size, at an
  offset inside a larger buffer, gives the same solution as a fresh one.
* The automatic convergence-check interval changes only how many iterations
  the host queues ahead: x and the iteration counts equal those of a fixed
  interval of 4, for FP64, FP32 mixed and a batch of right-hand sides; so does
  replaying the iteration from a HIP graph (twice, with eager solves between)."""
import ctypes

import numpy as np
import pytest
import torch

import latgen
from oracle import storage
import paper_1401_2039_amd as q
from paper_1401_2039_amd import _lib as L
from gpu_util import say, dev, host

pytestmark = pytest.mark.gpu


def _cb_order(dims, parity):
    """Lexicographic site indices of one parity in checkerboard order (s = lex >> 1)."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    par = ((x + y + z + t) & 1).ravel()
    return np.nonzero(par == parity)[0]


def _unpack_rows01(store, dims, real_dtype):
    """Rows 0-1 of every forward link from a reconstruct-12 store: blocks of 64
    sites, block index (parity * 4 + mu) * nb + s / 64, 3 units of 2 complex
    entries (row-major over rows 0-1) per site.  Returns [parity][mu][s][2][3]."""
    vh = int(np.prod(dims)) // 2
    nb = (vh + 63) // 64
    a = store.cpu().numpy().view(real_dtype).reshape(2, 4, nb, 3, 64, 4)
    c = a[..., 0::2].astype(np.float64) + 1j * a[..., 1::2].astype(np.float64)   # [2][4][nb][3 units][64][2]
    c = np.moveaxis(c, 4, 3).reshape(2, 4, nb * 64, 6)[:, :, :vh]
    return c.reshape(2, 4, vh, 2, 3)


def test_link_stores_bit_exact():
    say("link stores 16^3x32")
    cfg = latgen.make_config(1, with_source=False)
    dims, U = cfg["dims"], cfg["U"]
    lat = q.Lattice(dims, cfg["kappa"], U)
    Uflat = U.reshape(-1, 4, 3, 3)
    for prec, store, dt, rnd in ((q.F32, lat.gauge_f32, np.float32, np.complex64),
                                 (q.F16S, lat.gauge_f16, np.float16, "f16")):
        got = _unpack_rows01(store, dims, dt)
        want_all = storage.round_links_r12(U, rnd).reshape(-1, 4, 3, 3)
        for p in (0, 1):
            lex = _cb_order(dims, p)
            want = np.moveaxis(want_all[lex][:, :, :2, :], 1, 0)   # [mu][s][2][3]
            ndiff = int(np.count_nonzero(got[p] != want))
            assert ndiff == 0, (prec, p, ndiff)
    # FP64 reconstruct-18: 9 complex entries per link, the link itself
    vh = int(np.prod(dims)) // 2
    nb = (vh + 63) // 64
    a = lat.gauge_f64.cpu().numpy().view(np.float64).reshape(2, 4, nb, 9, 64, 2)
    c = (a[..., 0] + 1j * a[..., 1])
    c = np.moveaxis(c, 4, 3).reshape(2, 4, nb * 64, 9)[:, :, :vh]
    for p in (0, 1):
        lex = _cb_order(dims, p)
        assert np.array_equal(c[p], np.moveaxis(Uflat[lex].reshape(-1, 4, 9), 1, 0))
    lat.close()


def test_link_store_f16_rounding_cases():
    """The FP16 store of links whose rows 0 and 1 hold doubles where rounding
    through FP32 first would give a different FP16, values in the FP16 subnormal
    range and exact ties: each real is the nearest FP16 (ties to even)."""
    say("FP16 link store rounding cases")
    dims = (4, 4, 4, 4)
    rng = np.random.default_rng(93)
    n = int(np.prod(dims)) * 4 * 12
    e = rng.integers(-26, 1, n).astype(np.float64)
    m = rng.integers(0, 1 << 10, n).astype(np.float64)
    base = (1.0 + (m + 0.5) / 1024.0) * 2.0 ** e          # exact FP16 ties (and below half the smallest subnormal)
    nudge = rng.choice([-1.0, 0.0, 1.0], n) * 2.0 ** (e - 30)   # just below, at, just above the tie
    vals = np.where(rng.random(n) < 0.5, -1.0, 1.0) * (base + nudge)
    vals[:4] = [1.0 + 2.0 ** -11 + 2.0 ** -30, 2.0 ** -25 + 2.0 ** -60, -(0.5 + 2.0 ** -12 + 2.0 ** -40), 0.0]
    U = np.zeros(tuple(dims[::-1]) + (4, 3, 3), dtype=np.complex128)
    v = vals.reshape(-1, 4, 12)
    rows = v[..., 0::2] + 1j * v[..., 1::2]                # 6 complex entries per link
    U.reshape(-1, 4, 3, 3)[:, :, :2, :] = rows.reshape(-1, 4, 2, 3)
    U.reshape(-1, 4, 3, 3)[:, :, 2, 2] = 1.0
    lat = q.Lattice(dims, 0.12, U)
    got = _unpack_rows01(lat.gauge_f16, dims, np.float16)
    Uf = U.reshape(-1, 4, 3, 3)
    for p in (0, 1):
        lex = _cb_order(dims, p)
        r = np.moveaxis(Uf[lex][:, :, :2, :], 1, 0)
        want = r.real.astype(np.float16).astype(np.float64) + 1j * r.imag.astype(np.float16).astype(np.float64)
        assert np.array_equal(got[p], want), (p, int(np.count_nonzero(got[p] != want)))
    lat.close()


def test_workspace_size_contract():
    say("workspace contract")
    dims = (8, 8, 8, 8)
    cfg = latgen.small_config(dims, seed=70, kind="expih", eps=0.3, nrhs=2)
    lat = q.Lattice(dims, 0.12, cfg["U"])
    b = dev(cfg["b"])
    for kw in (dict(), dict(inner_prec=q.F16S), dict(solver=q.BICGSTAB_EO, inner_prec=q.F32)):
        prm = q.solve_params(tol=1e-10, **kw)
        need = q.qiral_solve_workspace_bytes(lat.handle, prm, 2)
        assert need > 0
        big = torch.zeros(need + 4096, dtype=torch.uint8, device="cuda")
        x_ref = torch.zeros_like(b)
        st, _ = q.qiral_solve(lat.handle, dims, x_ref, b, 2, prm, ws=big)
        assert st == 0
        # one byte short: refused before any work, x untouched
        x = torch.full_like(b, 3.0 + 1.0j)
        short = big[:need - 1]
        with pytest.raises(q.QiralError) as e:
            q.qiral_solve(lat.handle, dims, x, b, 2, prm, ws=short)
        assert e.value.status == L.ERR_WORKSPACE
        assert torch.all(x == (3.0 + 1.0j))
        # exactly the size, 256 bytes into a buffer filled with garbage
        big.fill_(0xA5)
        exact = big[256:256 + need]
        st, _ = q.qiral_solve(lat.handle, dims, x, b, 2, prm, ws=exact)
        assert st == 0 and torch.equal(x, x_ref), kw
        del big
    # the batch entry point checks its own size
    prm = q.solve_params(tol=1e-10)
    need = q.qiral_solve_batch_workspace_bytes([lat.handle, lat.handle], prm)
    assert need == q.qiral_solve_workspace_bytes(lat.handle, prm, 2)
    lat.close()


@pytest.mark.parametrize("kw", [dict(), dict(inner_prec=q.F32)], ids=["f64", "f32"])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_adaptive_check_interval_same_iterates(kw, nrhs):
    dims = (8, 8, 8, 16)
    say("check interval", kw, nrhs)
    cfg = latgen.small_config(dims, seed=71, kind="expih", eps=0.3, nrhs=nrhs)
    lat = q.Lattice(dims, 0.12, cfg["U"])
    b = dev(cfg["b"])
    xa, sa, ia = lat.solve(b, tol=1e-10, check_every=0, **kw)
    xa = xa.clone()
    xf, sf, i_f = lat.solve(b, tol=1e-10, check_every=4, **kw)
    xf = xf.clone()
    assert sa == 0 and sf == 0
    assert torch.equal(xa, xf)
    assert [i["iterations"] for i in ia] == [i["iterations"] for i in i_f]
    assert [i["reliable_updates"] for i in ia] == [i["reliable_updates"] for i in i_f]
    # the iteration captured in a HIP graph and replayed (a side stream: the
    # default stream is not captured), twice in a row with eager solves between
    stream = torch.cuda.Stream()
    for _ in range(2):
        with torch.cuda.stream(stream):
            xg, sg, ig = lat.solve(b, tol=1e-10, use_graph=1, **kw)
        stream.synchronize()
        assert sg == 0 and torch.equal(xa, xg)
        assert [i["iterations"] for i in ia] == [i["iterations"] for i in ig]
        xe, se, _ = lat.solve(b, tol=1e-10, **kw)
        assert se == 0 and torch.equal(xa, xe)
    lat.close()
