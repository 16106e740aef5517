"""Benchmark of the even-odd Wilson-Dirac solve on one MI355X.

A step is the paper's plain method on its 24^3x48 lattice: even-odd CGNR in
FP64 (the FP64 hop, which reads rows 0-1 of each stored FP64 link and rebuilds
row 2; Schur source, reconstruction and FP64 true residual included) for each of the 12 point sources of the workload
(exp(0.4 i H) links, kappa 0.12, one source per spin-colour at a seeded site),
solved one after the other through qiral_solve to ||b - D x|| / ||b|| <= 1e-10.
Inputs (canonical links packed once, canonical sources and the workspace) are
resident in device memory before the timed region.

value: Dslash GFLOP/s sustained over the step: 1320 flop per output site and
hop application, times the hop applications of the 12 solves, divided by the
step's wall time.

The JSON line also carries:
- the same 12 sources solved in one batched qiral_solve call in FP64, and in
  the mixed-precision forms (F32 and F16S hop with FP64 reliable updates), each
  with its time to solution and speedup over the step (plain FP64 eo-CGNR);
- roofline: the dominant kernel of the step, the FP64 even-odd hop on this
  lattice with one right-hand side (8 links x 96 B (rows 0-1 of a link) + 192 B
  in + 192 B out = 1152 B per output site, 331776 sites, 382 MB per launch:
  1.5 times the 256 MB last-level cache), launched through qiral_dslash_eo and timed with HIP events
  on its stream: warm (back-to-back launches) and cold (single launches, each
  after a 1 GiB read that replaces the cache's contents); HBM traffic from the
  committed counter summary while the hop sources are unchanged;
- learned: the learned preconditioner against plain FP64 eo-CGNR on the
  24^3x48, exp(0.5 i H), kappa 0.125 lattice with 12 Gaussian sources (the
  network trained on 2048 pairs (D v, v) first, training time reported apart,
  with the break-even count of 12-source solves);
- the one-time link packing time, a measured 1 GiB device copy, and the CPU
  oracle timed on a bounded sample (a few CGNR iterations of the same system).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--suite]
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hop_f64_24x24x24x48_traffic.md")
HOP_SOURCES = [os.path.join(ROOT, "paper_1401_2039_amd", "csrc", f) for f in ("qiral_dev.h", "api.hip")]
FLOP_PER_SITE = 1320           # one even-odd hop, per output site
# algorithmic bytes per output site of one hop: 8 links + 1 input + 1 output spinor
# (every hop reads rows 0-1 of a link: 96 B in FP64, 48 B in FP32, 24 B in FP16)
LINK_READ_BYTES = {"f64": 96, "f32": 48, "f16s": 24}
HOP_BYTES = {"f64": 8 * 96 + 192 + 192, "f32": 8 * 48 + 96 + 96, "f16s": 8 * 24 + 52 + 52}
ROOFLINE_KERNEL = "k_hop<0, 0, false, 0, 4, 1, true>"   # S_F64, L_F64R18, H (not dagger), plain epilogue, T 4, NR 1, streaming
WORKLOAD = ("24^3x48 lattice, exp(0.4iH) links, kappa=0.12, 12 point sources (one per spin-colour): even-odd CGNR "
            "in FP64 with the FP64 hop, the sources solved one after the other, to 1e-10 true residual")


def hop_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in HOP_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the roofline kernel from the committed counter
    summary, or None if it is missing or was taken on different kernel sources."""
    try:
        kv = {}
        for line in open(TRAFFIC_SUMMARY):
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                kv[k.strip()] = v.strip().strip("`")
        if kv.get("source_sha256") != hop_source_hash():
            return None
        return int(float(kv["hbm_bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--hop-reps", type=int, default=50, help="back-to-back hop launches per warm trial")
    ap.add_argument("--cpu-iters", type=int, default=3, help="oracle CGNR iterations timed for the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner comparison")
    ap.add_argument("--suite", action="store_true", help="also measure the other workloads (stderr JSON lines)")
    ap.add_argument("--suite-out", default=None, help="append the suite's JSON lines to this file")
    ap.add_argument("--parts", default="c1,c0,c2,c3,c99,c4", help="suite parts to run")
    ap.add_argument("--suite-hop-reps", type=int, default=None,
                    help="timed launches per hop measurement in the suite (default 100, 50 on 32^3x64)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import latgen
    import paper_1401_2039_amd as q

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    t_gen = time.time()
    cfg = latgen.make_config(2)
    log(f"[bench] generated 24^3x48 inputs in {time.time() - t_gen:.1f}s")
    dims, kappa = cfg["dims"], cfg["kappa"]
    nrhs = cfg["b"].shape[0]
    vh = int(np.prod(dims)) // 2
    Ud = torch.from_numpy(cfg["U"]).to(dev)
    torch.cuda.synchronize()
    t_pack = time.perf_counter()
    lat = q.Lattice(dims, kappa, Ud)
    torch.cuda.synchronize()
    pack_ms = (time.perf_counter() - t_pack) * 1e3   # one-time link packing, outside the timed solves
    del Ud
    b = torch.from_numpy(cfg["b"]).to(dev)
    srcs = [b[r:r + 1].contiguous() for r in range(nrhs)]
    xs = [torch.zeros_like(s) for s in srcs]
    stream = torch.cuda.current_stream()
    p64 = q.solve_params(tol=1e-10, inner_prec=q.F64)
    ws = torch.empty(q.qiral_solve_workspace_bytes(lat.handle, p64, 1), dtype=torch.uint8, device=dev)

    def step():
        infos = []
        for r in range(nrhs):
            st, info = q.qiral_solve(lat.handle, dims, xs[r], srcs[r], 1, p64, ws=ws)
            if st != 0:
                raise RuntimeError(f"solve of source {r} failed: status {st} {info}")
            infos.append(info[0])
        return infos

    # ---- timed steps: plain FP64 even-odd CGNR, the 12 sources one after the other
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    hops, times, infos = 0, [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        infos = step()
        times.append(time.perf_counter() - ts)
        hops += sum(i["hop_applications"] for i in infos)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = FLOP_PER_SITE * vh * hops / elapsed / 1e9
    its = [i["iterations"] for i in infos]
    log(f"[bench] step (12 FP64 eo-CGNR solves): {elapsed / args.steps * 1e3:.2f} ms, iterations {its}, "
        f"{value:.0f} GFLOP/s")

    # ---- the same 12 sources in one batched call: FP64, and the mixed-precision forms
    batched = {}
    for name, prec in (("f64", q.F64), ("f32_mixed", q.F32), ("f16s_mixed", q.F16S)):
        lat.tune(prec, nrhs)
        prm = q.solve_params(tol=1e-10, inner_prec=prec)
        wsb = torch.empty(q.qiral_solve_workspace_bytes(lat.handle, prm, nrhs), dtype=torch.uint8, device=dev)
        xb = torch.zeros_like(b)
        q.qiral_solve(lat.handle, dims, xb, b, nrhs, prm, ws=wsb)   # warm-up
        ts_ = []
        for _ in range(3):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            st, binfo = q.qiral_solve(lat.handle, dims, xb, b, nrhs, prm, ws=wsb)
            ts_.append(time.perf_counter() - ts)
            if st != 0:
                raise RuntimeError(f"batched {name} solve failed: status {st}")
        t = statistics.median(ts_)
        batched[name] = {"time_to_solution_s": round(t, 5), "speedup_vs_fp64_cgnr": round(statistics.median(times) / t, 3),
                         "iterations_max": max(i["iterations"] for i in binfo),
                         "reliable_updates_max": max(i["reliable_updates"] for i in binfo),
                         "true_rel_resid_max": max(i["true_rel_resid"] for i in binfo)}
        log(f"[bench] batched {name}: {t * 1e3:.2f} ms ({batched[name]['speedup_vs_fp64_cgnr']}x the step)")
        del wsb, xb

    # ---- roofline of the dominant kernel: the FP64 even-odd hop, one right-hand side
    psi = torch.from_numpy(latgen.gaussian_source(2, 1, dims, 1)).to(dev)
    src = lat.import_field(psi, q.ODD, q.F64)
    out = lat.field(q.EVEN, q.F64)
    del psi
    for _ in range(5):
        lat.dslash_eo(out, src, 0, 0, q.F64)
    trials = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        e0.record(stream)
        for _ in range(args.hop_reps):
            lat.dslash_eo(out, src, 0, 0, q.F64)
        e1.record(stream)
        e1.synchronize()
        trials.append(e0.elapsed_time(e1) * 1e3 / args.hop_reps)
    warm_us = statistics.median(trials)
    flush = torch.zeros(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
    cold = []
    for _ in range(11):
        flush.sum()   # a read: the cache then holds clean, unrelated lines
        e0.record(stream)
        lat.dslash_eo(out, src, 0, 0, q.F64)
        e1.record(stream)
        e1.synchronize()
        cold.append(e0.elapsed_time(e1) * 1e3)
    cold_us = statistics.median(cold)
    del flush
    hop_bytes = HOP_BYTES["f64"] * vh
    achieved = hop_bytes / (warm_us * 1e-6) / 1e9
    log(f"[bench] FP64 hop 24^3x48: warm {warm_us:.2f} us ({achieved:.0f} GB/s), cold {cold_us:.2f} us "
        f"({hop_bytes / (cold_us * 1e-6) / 1e9:.0f} GB/s)")

    # ---- a plain 1 GiB device copy: the measured copy ceiling, and the reference a
    # counter run scales FETCH_SIZE / WRITE_SIZE by
    cx = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    cy = torch.empty_like(cx)
    cy.copy_(cx)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(5):
        cy.copy_(cx)
    e1.record(stream)
    e1.synchronize()
    copy_gbs = 2 * (1 << 30) * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del cx, cy

    learned = None if args.no_learned else learned_vs_cgnr(q, latgen, torch, dev)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(cfg, args.cpu_iters)

    res = {
        "metric": "Dslash GFLOP/s + %HBM roofline; time-to-1e-10 solve, mixed/learned vs FP64 CG",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "dims": list(dims), "kappa": kappa, "nrhs": nrhs, "tol": 1e-10,
                   "links": "exp(0.4 i H) per link, H a seeded Gaussian traceless Hermitian 3x3"},
        "time_to_solution_s": round(statistics.median(times), 6),
        "iterations": its,
        "true_rel_resid_max": max(i["true_rel_resid"] for i in infos),
        "hop_applications_per_step": hops // args.steps,
        "batched": batched,
        "learned": learned,
        "roofline": {"bound": "hbm", "kernel": ROOFLINE_KERNEL + " (qiral_dslash_eo, FP64, links read as rows 0-1, 1 RHS)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                     "bytes_per_launch": hop_bytes, "launch_us": round(warm_us, 3),
                     "cold_launch_us": round(cold_us, 3),
                     "cold_frac": round(hop_bytes / (cold_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                     "dslash_gflops": round(FLOP_PER_SITE * vh / (warm_us * 1e-6) / 1e9, 1),
                     "source_sha256": hop_source_hash(), "fits_last_level_cache": False,
                     "copy_ceiling_GBs": round(copy_gbs, 1), "frac_of_copy_ceiling": round(achieved / copy_gbs, 4)},
        "gauge_pack_ms": round(pack_ms, 3),
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)
    del ws, src, out
    if args.suite:
        suite(q, latgen, np, torch, args.suite_out, args.parts.split(','), args.suite_hop_reps)
    lat.close()


def learned_vs_cgnr(q, latgen, torch, dev, steps=2048):
    """The learned preconditioner against plain FP64 eo-CGNR on the 24^3x48,
    exp(0.5 i H), kappa 0.125 lattice with 12 Gaussian sources: the 2-layer
    network (8 hidden channels) trained on `steps` pairs (D v, v), then BiCGStab
    on the Schur system with it as right preconditioner, all 12 sources in one
    qiral_solve call, against the 12 sources solved one after the other by FP64
    eo-CGNR; both to a 1e-10 true residual, each timed once after a warm-up."""
    c4 = latgen.make_config(4)
    lat = q.Lattice(c4["dims"], c4["kappa"], c4["U"])
    b = torch.from_numpy(c4["b"]).to(dev)
    n = b.shape[0]
    del c4
    net = q.Network(lat, 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = net.train(steps, lr=1e-3, seed=4)
    t_train = time.perf_counter() - t0
    pl = q.solve_params(solver=q.BICGSTAB_EO, system=q.SYSTEM_SCHUR, tol=1e-10, maxiter=4000)
    pl.precond = net.handle
    p64 = q.solve_params(tol=1e-10, inner_prec=q.F64)
    wl = torch.empty(q.qiral_solve_workspace_bytes(lat.handle, pl, n), dtype=torch.uint8, device=dev)
    w64 = torch.empty(q.qiral_solve_workspace_bytes(lat.handle, p64, 1), dtype=torch.uint8, device=dev)
    x = torch.zeros_like(b)

    def learned():
        st, info = q.qiral_solve(lat.handle, lat.dims, x, b, n, pl, ws=wl)
        if st != 0:
            raise RuntimeError(f"learned solve failed: status {st}")
        return info

    def cgnr():
        infos = []
        for r in range(n):
            st, info = q.qiral_solve(lat.handle, lat.dims, x[r:r + 1], b[r:r + 1], 1, p64, ws=w64)
            if st != 0:
                raise RuntimeError(f"FP64 eo-CGNR solve failed: status {st}")
            infos.append(info[0])
        return infos

    out = {}
    for name, fn in (("learned", learned), ("cgnr", cgnr)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = fn()
        torch.cuda.synchronize()
        out[name] = (time.perf_counter() - t0, info)
    tl, il = out["learned"]
    tc, ic = out["cgnr"]
    res = {"workload": "24^3x48 lattice, exp(0.5iH) links, kappa=0.125, 12 Gaussian sources",
           "form": "BiCGStab on the Schur system, trained 2-layer PTC network (8 hidden) as right preconditioner",
           "time_to_solution_s": round(tl, 5), "fp64_cgnr_12_sequential_s": round(tc, 5),
           "speedup_vs_fp64_cgnr": round(tc / tl, 3), "iterations": [i["iterations"] for i in il],
           "cgnr_iterations": [i["iterations"] for i in ic],
           "true_rel_resid_max": max(i["true_rel_resid"] for i in il),
           "training_s": round(t_train, 3), "training_pairs": steps,
           "loss_first64": round(float(sum(hist[:64]) / 64), 5), "loss_last64": round(float(sum(hist[-64:]) / 64), 5),
           "break_even_solves_of_12": round(t_train / (tc - tl), 1) if tc > tl else None}
    log(f"[bench] learned: {tl * 1e3:.1f} ms against FP64 eo-CGNR {tc * 1e3:.1f} ms "
        f"({res['speedup_vs_fp64_cgnr']}x), training {t_train:.1f}s")
    net.close()
    lat.close()
    return res


def cpu_baseline(cfg, iters):
    """The oracle as it is, single thread, on `iters` CGNR iterations of the same
    24^3x48 Schur system (the first point source)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import solvers, wilson
    U, k, b = cfg["U"], cfg["kappa"], cfg["b"][0]
    vh = int(np.prod(cfg["dims"])) // 2
    with threadpool_limits(limits=1):
        bhat = wilson.schur_source(U, k, 0.0, b)
        A = lambda v: wilson.schur(U, k, 0.0, v)
        Ad = lambda v: wilson.schur(U, k, 0.0, v, dagger=True)
        t0 = time.perf_counter()
        solvers.cgnr(A, Ad, bhat, eps=0.0, maxiter=iters)
        dt = time.perf_counter() - t0
    hops = 2 + 4 * iters   # initial S^dagger r, then S and S^dagger per iteration
    val = FLOP_PER_SITE * vh * hops / dt / 1e9
    log(f"[bench] oracle: {iters} CGNR iterations on 24^3x48 in {dt:.1f}s ({val:.3f} GFLOP/s)")
    return {"value": round(val, 4), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} CGNR iterations (plus the initial S^dagger r) of the oracle on the same 24^3x48 "
                      f"Schur system (first point source), {dt:.1f}s, BLAS limited to 1 thread",
            "seconds": round(dt, 3), "sec_x_core": round(dt, 3), "host_cores": len(os.sched_getaffinity(0))}


def _emit(rec, path):
    log("[suite] " + json.dumps(rec))
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(rec) + "\n")


def timed_launches(torch, stream, launch, reps, trials=5):
    """Median over `trials` of the per-launch time of `reps` back-to-back calls of
    `launch`, from HIP events on `stream`.  Each trial first queues a spin kernel
    long enough to cover the host's enqueueing of all `reps` launches, so the
    events bracket GPU time only (the kernels and the gaps the hardware leaves
    between them), not the Python binding's per-call cost.  Returns (us per
    launch, host us per enqueued launch)."""
    import statistics
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # spin-kernel clock rate: cycles per microsecond
    e0.record(stream)
    torch.cuda._sleep(1 << 20)
    e1.record(stream)
    e1.synchronize()
    cyc_per_us = (1 << 20) / max(e0.elapsed_time(e1) * 1e3, 1.0)
    host_us, per_launch = 50.0, []
    for _ in range(trials):
        torch.cuda._sleep(int(cyc_per_us * min(2.0 * host_us * reps + 500.0, 1e5)))   # at most 0.1 s
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(reps):
            launch()
        e1.record(stream)
        host_us = (time.perf_counter() - t0) * 1e6 / reps
        e1.synchronize()
        per_launch.append(e0.elapsed_time(e1) * 1e3 / reps)
    return statistics.median(per_launch), host_us


def hop_rates(q, lat, dims, torch, prec, nrhs=1, reps=100, flush=None, psi=None):
    """Average duration of one even-odd hop launch (HIP events on the launch stream):
    warm (back to back) and, with a flush buffer, cold (median of single launches,
    each after a 1 GiB read that replaces the 256 MB last-level cache's contents)."""
    import numpy as np
    import latgen
    vh = int(np.prod(dims)) // 2
    if psi is None:
        psi = torch.from_numpy(latgen.gaussian_source(5, 0, dims, nrhs)).cuda()
    src = lat.import_field(psi, q.ODD, prec)
    out = lat.field(q.EVEN, prec, nrhs)
    del psi
    stream = torch.cuda.current_stream()
    for _ in range(5):
        lat.dslash_eo(out, src, 0, 0, prec, nrhs)
    warm, _ = timed_launches(torch, stream, lambda: lat.dslash_eo(out, src, 0, 0, prec, nrhs), reps, trials=3)
    cold = None
    if flush is not None:
        ts = []
        for _ in range(max(11, reps // 5)):
            # read 1 GiB: the caches then hold clean unrelated lines (a write
            # would also leave 256 MB of dirty lines for the hop to write back)
            flush.sum()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            lat.dslash_eo(out, src, 0, 0, prec, nrhs)
            b.record(stream)
            b.synchronize()
            ts.append(a.elapsed_time(b) * 1e3)
        cold = float(np.median(ts))
    key = {q.F64: "f64", q.F32: "f32", q.F16S: "f16s"}[prec]
    link_b = LINK_READ_BYTES[key] * 8
    sp_b = {"f64": 192, "f32": 96, "f16s": 52}[key]
    bytes_ = vh * (link_b + 2 * sp_b * nrhs)
    res = {"kind": "hop", "dims": list(dims), "prec": key, "nrhs": nrhs, "bytes_per_launch": bytes_,
           "warm_us": round(warm, 3), "warm_GBs": round(bytes_ / warm / 1e3, 1),
           "warm_GFLOPs": round(FLOP_PER_SITE * vh * nrhs / warm / 1e3, 1),
           "warm_frac_hbm": round(bytes_ / warm / 1e3 / HBM_PEAK_GBS, 4),
           "fits_last_level_cache": bytes_ < 256e6}
    if cold is not None:
        res.update({"cold_us": round(cold, 3), "cold_GBs": round(bytes_ / cold / 1e3, 1),
                    "cold_GFLOPs": round(FLOP_PER_SITE * vh * nrhs / cold / 1e3, 1),
                    "cold_frac_hbm": round(bytes_ / cold / 1e3 / HBM_PEAK_GBS, 4)})
    return res


def suite(q, latgen, np, torch, path=None, parts=(), hop_reps=None):
    """Extra measurements: hop throughput of every storage class on the workloads'
    lattices (warm and cache-flushed) and time to solution of each solver form."""
    import time as _t
    flush = torch.zeros(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
    dims1 = (16, 16, 16, 32)
    lat1 = None
    if "c1" in parts:
        c1 = latgen.make_config(1, with_source=False)
        lat1 = q.Lattice(c1["dims"], c1["kappa"], c1["U"])
        del c1
        for prec in (q.F64, q.F32, q.F16S):
            _emit(hop_rates(q, lat1, dims1, torch, prec, reps=hop_reps or 100, flush=flush), path)

    def timed_solve(lat, b, reps=2, **kw):
        x = torch.zeros_like(b)
        st, info = q.qiral_solve(lat.handle, lat.dims, x, b, b.shape[0], q.solve_params(**kw))
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = _t.perf_counter()
            st, info = q.qiral_solve(lat.handle, lat.dims, x, b, b.shape[0], q.solve_params(**kw))
            ts.append(_t.perf_counter() - t0)
        return min(ts), st, info, x

    if "c1" in parts:
        suite_c1(lat1, q, latgen, torch, path, timed_solve)
        lat1.close()
    if "c0" in parts:
        suite_c0(q, latgen, torch, path, timed_solve)
    if "c2" in parts:
        suite_c2(q, latgen, torch, path, timed_solve, flush)
    if "c3" in parts:
        suite_c3(q, latgen, torch, path, timed_solve)
    if "c99" in parts:
        c99 = latgen.make_config(99, with_source=False)
        lat99 = q.Lattice(c99["dims"], c99["kappa"], c99["U"])
        del c99
        for prec in (q.F64, q.F32, q.F16S):
            _emit(hop_rates(q, lat99, (32, 32, 32, 64), torch, prec, reps=hop_reps or 50, flush=flush), path)
        lat99.close()
    if "c4" in parts:
        suite_c4(q, latgen, torch, path, timed_solve)
    if "c64" in parts:
        suite_c64(q, latgen, torch, path, timed_solve, flush, hop_reps)
    if "compose" in parts:
        suite_compose(q, latgen, torch, path, timed_solve)
    if "shard" in parts:
        suite_shard(q, latgen, torch, path, flush, hop_reps)


def suite_c1(lat1, q, latgen, torch, path, timed_solve):
    """Every solver form on the 16^3x32 workload, each judged against the oracle:
    its true residual under the oracle's D, and its distance to the oracle's own
    FP64 eo-CGNR solution."""
    import time as _t
    import numpy as np
    from oracle import solvers as S, wilson as W
    cfg = latgen.make_config(1)
    b1 = torch.from_numpy(cfg["b"]).cuda()
    t0 = _t.perf_counter()
    xo, oinfo = S.solve_eo_cgnr(cfg["U"], cfg["kappa"], 0.0, cfg["b"][0], tol=1e-10)
    log(f"[suite] oracle eo-CGNR on 16^3x32: {oinfo['iterations']} iterations in {_t.perf_counter() - t0:.1f}s")
    for name, kw in [("cgnr_f64", dict(inner_prec=q.F64)), ("cgnr_f32", dict(inner_prec=q.F32)),
                     ("cgnr_f16s", dict(inner_prec=q.F16S)), ("bicgstab_f64", dict(solver=q.BICGSTAB_EO)),
                     ("bicgstab_f32", dict(solver=q.BICGSTAB_EO, inner_prec=q.F32)),
                     ("crnr_f64", dict(solver=q.CRNR_EO)),
                     ("cgnr_f32_graph", dict(inner_prec=q.F32, use_graph=1))]:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            t, st, info, x = timed_solve(lat1, b1, tol=1e-10, **kw)
        stream.synchronize()
        xg = x.cpu().numpy()[0]
        _emit({"kind": "solve", "workload": "16^3x32 eps0.3 k0.12 1rhs", "form": name, "seconds": round(t, 6),
               "status": st, "iterations": info[0]["iterations"], "reliable_updates": info[0]["reliable_updates"],
               "true_rel_resid": info[0]["true_rel_resid"], "hops": info[0]["hop_applications"],
               "oracle_judged_resid": S.true_rel_residual(cfg["U"], cfg["kappa"], 0.0, xg, cfg["b"][0]),
               "rel_err_vs_oracle_x": float(np.sqrt(W.norm2(xg - xo) / W.norm2(xo))),
               "oracle_iterations": oinfo["iterations"]}, path)



def suite_c0(q, latgen, torch, path, timed_solve):
    import time as _t
    # 4^4 Haar (plain method): GPU FP64 eo-CGNR vs the oracle in CPU seconds
    c0 = latgen.make_config(0)
    lat0 = q.Lattice(c0["dims"], c0["kappa"], c0["U"])
    b0 = torch.from_numpy(c0["b"]).cuda()
    t, st, info, _ = timed_solve(lat0, b0, reps=5, tol=1e-10)
    from oracle import solvers
    t0 = _t.perf_counter()
    _, oinfo = solvers.solve_eo_cgnr(c0["U"], c0["kappa"], 0.0, c0["b"][0], tol=1e-10)
    tcpu = _t.perf_counter() - t0
    _emit({"kind": "solve", "workload": "4^4 haar k0.12 1rhs", "form": "cgnr_f64", "seconds": round(t, 6),
           "iterations": info[0]["iterations"], "oracle_seconds": round(tcpu, 4),
           "oracle_iterations": oinfo["iterations"], "true_rel_resid": info[0]["true_rel_resid"]}, path)
    lat0.close()



def suite_c2(q, latgen, torch, path, timed_solve, flush):
    # 24^3x48: hop rates (1 RHS all classes, 12 RHS F16S), 12 point sources
    c2 = latgen.make_config(2)
    lat2 = q.Lattice(c2["dims"], c2["kappa"], c2["U"])
    for prec in (q.F64, q.F32, q.F16S):
        _emit(hop_rates(q, lat2, c2["dims"], torch, prec, flush=flush), path)
    _emit(hop_rates(q, lat2, c2["dims"], torch, q.F16S, nrhs=12, reps=50, flush=flush), path)
    _emit(hop_rates(q, lat2, c2["dims"], torch, q.F32, nrhs=12, reps=50, flush=flush), path)
    b2 = torch.from_numpy(c2["b"]).cuda()
    for prec, nm in ((q.F16S, "f16s"), (q.F32, "f32"), (q.F64, "f64")):
        t_, nr_, us_ = lat2.tune(prec, 12)
        _emit({"kind": "tune", "dims": list(c2["dims"]), "prec": nm, "nrhs": 12, "waves_per_block": t_,
               "rhs_per_lane": nr_, "us": round(us_, 2)}, path)
    for name, kw in [("batched12_f16s", dict(inner_prec=q.F16S)), ("batched12_f32", dict(inner_prec=q.F32)),
                     ("batched12_f64", dict(inner_prec=q.F64))]:
        t, st, info, _ = timed_solve(lat2, b2, reps=1, tol=1e-10, **kw)
        _emit({"kind": "solve", "workload": "24^3x48 eps0.4 k0.12 12 point sources", "form": name,
               "seconds": round(t, 4), "status": st, "iterations": [i["iterations"] for i in info],
               "max_true_rel_resid": max(i["true_rel_resid"] for i in info)}, path)
    tseq = 0.0
    its = []
    for r in range(12):
        t, st, info, _ = timed_solve(lat2, b2[r:r + 1].contiguous(), reps=1, tol=1e-10)
        tseq += t
        its.append(info[0]["iterations"])
    _emit({"kind": "solve", "workload": "24^3x48 eps0.4 k0.12 12 point sources", "form": "sequential12_f64",
           "seconds": round(tseq, 4), "iterations": its}, path)
    lat2.close()
    del b2



def suite_c3(q, latgen, torch, path, timed_solve):
    import time as _t
    # uneven batch of 32 systems
    cfgs = [latgen.make_config(3, s) for s in range(32)]
    lats = [q.Lattice(c["dims"], c["kappa"], c["U"]) for c in cfgs]
    bs = [torch.from_numpy(c["b"]).cuda() for c in cfgs]
    xs = [torch.zeros_like(b) for b in bs]
    for name, kw in [("batch32_mixed_f32", dict(inner_prec=q.F32)), ("batch32_f64", dict(inner_prec=q.F64)),
                     ("batch32_mixed_f32_graph", dict(inner_prec=q.F32, use_graph=1))]:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            q.qiral_solve_batch([l.handle for l in lats], [l.dims for l in lats], xs, bs, q.solve_params(tol=1e-10, **kw))
            torch.cuda.synchronize()
            t0 = _t.perf_counter()
            st, info = q.qiral_solve_batch([l.handle for l in lats], [l.dims for l in lats], xs, bs,
                                           q.solve_params(tol=1e-10, **kw))
            t = _t.perf_counter() - t0
        _emit({"kind": "solve", "workload": "uneven batch 32 systems", "form": name, "seconds": round(t, 4),
               "status": st, "max_true_rel_resid": max(i["true_rel_resid"] for i in info),
               "iterations": [i["iterations"] for i in info]}, path)
    tseq = 0.0
    for l, b in zip(lats, bs):
        t, st, info, _ = timed_solve(l, b, reps=1, tol=1e-10)
        tseq += t
    _emit({"kind": "solve", "workload": "uneven batch 32 systems", "form": "sequential32_f64", "seconds": round(tseq, 4)},
          path)
    for l in lats:
        l.close()
    del bs, xs



def suite_c4(q, latgen, torch, path, timed_solve):
    """24^3x48, exp(0.5 i H), kappa 0.125, 12 Gaussian sources: the 2-layer network
    (8 hidden channels) trained on 2048 pairs (D v, v), FGMRES(20) and FCG with it,
    against plain even-odd CGNR in FP64 and the mixed batched CGNR."""
    import time as _t
    import numpy as np
    c4 = latgen.make_config(4)
    lat = q.Lattice(c4["dims"], c4["kappa"], c4["U"])
    b = torch.from_numpy(c4["b"]).cuda()
    del c4["U"]
    lat.tune(q.F16S, 12)
    net = q.Network(lat, 8)
    # the untrained network (Neumann series 1 + kH + k^2 H^2) on one source first
    params = q.solve_params(solver=q.FGMRES_NN, tol=1e-10, restart=20, maxiter=2000)
    params.precond = net.handle
    x = torch.zeros_like(b[:1])
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    st, info = q.qiral_solve(lat.handle, lat.dims, x, b[:1].contiguous(), 1, params)
    _emit({"kind": "solve", "workload": "24^3x48 eps0.5 k0.125 1 of 12 gaussian", "form": "fgmres20_neumann2",
           "seconds": round(_t.perf_counter() - t0, 4), "status": st, "iterations": info[0]["iterations"],
           "fell_back": info[0]["fell_back"], "true_rel_resid": info[0]["true_rel_resid"]}, path)
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    hist = net.train(2048, lr=1e-3, seed=4)
    t_train = _t.perf_counter() - t0
    _emit({"kind": "train", "workload": "24^3x48 eps0.5 k0.125", "pairs": 2048, "seconds": round(t_train, 3),
           "loss_first64": float(np.mean(hist[:64])), "loss_last64": float(np.mean(hist[-64:]))}, path)
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    st, info = q.qiral_solve(lat.handle, lat.dims, x, b, 12, params)
    t_nn = _t.perf_counter() - t0
    _emit({"kind": "solve", "workload": "24^3x48 eps0.5 k0.125 12 gaussian", "form": "fgmres20_trained",
           "seconds": round(t_nn, 4), "status": st, "iterations": [i["iterations"] for i in info],
           "fell_back": [i["fell_back"] for i in info],
           "max_true_rel_resid": max(i["true_rel_resid"] for i in info)}, path)
    # flexible CG on the normal equations with N N^dagger, same network
    pf = q.solve_params(solver=q.FCG_NN, tol=1e-10, maxiter=4000)
    pf.precond = net.handle
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    st, info = q.qiral_solve(lat.handle, lat.dims, x, b, 12, pf)
    t_fcg = _t.perf_counter() - t0
    _emit({"kind": "solve", "workload": "24^3x48 eps0.5 k0.125 12 gaussian", "form": "fcg_trained",
           "seconds": round(t_fcg, 4), "status": st, "iterations": [i["iterations"] for i in info],
           "fell_back": [i["fell_back"] for i in info],
           "max_true_rel_resid": max(i["true_rel_resid"] for i in info)}, path)
    # the Schur-system compositions with the trained network (M_S v = P_o N (0 + v))
    learned = {"fgmres20_full": t_nn, "fcg_full": t_fcg}
    for name, solver in (("bicgstab_schur", q.BICGSTAB_EO), ("fgmres20_schur", q.FGMRES_NN)):
        ps = q.solve_params(solver=solver, system=q.SYSTEM_SCHUR, tol=1e-10, restart=20, maxiter=4000)
        ps.precond = net.handle
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        st, info = q.qiral_solve(lat.handle, lat.dims, x, b, 12, ps)
        learned[name] = _t.perf_counter() - t0
        _emit({"kind": "solve", "workload": "24^3x48 eps0.5 k0.125 12 gaussian", "form": name + "_trained",
               "seconds": round(learned[name], 4), "status": st, "iterations": [i["iterations"] for i in info],
               "fell_back": [i["fell_back"] for i in info],
               "max_true_rel_resid": max(i["true_rel_resid"] for i in info)}, path)
    tseq = 0.0
    its = []
    for r in range(12):
        t, st, info, _ = timed_solve(lat, b[r:r + 1].contiguous(), reps=1, tol=1e-10)
        tseq += t
        its.append(info[0]["iterations"])
    _emit({"kind": "solve", "workload": "24^3x48 eps0.5 k0.125 12 gaussian", "form": "sequential12_cgnr_f64",
           "seconds": round(tseq, 4), "iterations": its}, path)
    t, st, info, _ = timed_solve(lat, b, reps=1, tol=1e-10, inner_prec=q.F16S)
    _emit({"kind": "solve", "workload": "24^3x48 eps0.5 k0.125 12 gaussian", "form": "batched12_cgnr_f16s",
           "seconds": round(t, 4), "iterations": [i["iterations"] for i in info],
           "max_true_rel_resid": max(i["true_rel_resid"] for i in info)}, path)
    # plain FP64 methods batched the same way as the learned form: eo-CGNR, and
    # BiCGStab on the Schur system, the strongest of them here
    t, st, info, _ = timed_solve(lat, b, reps=1, tol=1e-10, inner_prec=q.F64)
    _emit({"kind": "solve", "workload": "24^3x48 eps0.5 k0.125 12 gaussian", "form": "batched12_cgnr_f64",
           "seconds": round(t, 4), "status": st, "iterations": [i["iterations"] for i in info],
           "max_true_rel_resid": max(i["true_rel_resid"] for i in info)}, path)
    t, st, info, _ = timed_solve(lat, b, reps=1, tol=1e-10, solver=q.BICGSTAB_EO, inner_prec=q.F64)
    _emit({"kind": "solve", "workload": "24^3x48 eps0.5 k0.125 12 gaussian", "form": "batched12_bicgstab_f64",
           "seconds": round(t, 4), "status": st, "iterations": [i["iterations"] for i in info],
           "max_true_rel_resid": max(i["true_rel_resid"] for i in info)}, path)
    best = min(learned, key=learned.get)
    gain = tseq - learned[best]
    _emit({"kind": "summary", "workload": "24^3x48 eps0.5 k0.125", "training_s": round(t_train, 3),
           "learned_12rhs_s": {k: round(v, 4) for k, v in learned.items()}, "best_learned": best,
           "cgnr_f64_12rhs_s": round(tseq, 4), "speedup_best_vs_cgnr_f64": round(tseq / learned[best], 3),
           "break_even_solves_of_12": (round(t_train / gain, 2) if gain > 0 else None)}, path)
    net.close()
    lat.close()


def suite_compose(q, latgen, torch, path, timed_solve):
    """Time per iteration against total time of every solver x system x
    preconditioner composition (Sec. 5's comparison of its solvers), FP64, on the
    24^3x48 exp(0.5 i H), kappa 0.125 lattice with one Gaussian source; the network
    carries the Neumann-2 weights of 1 + kappa H + kappa^2 H^2."""
    c4 = latgen.make_config(4)
    lat = q.Lattice(c4["dims"], c4["kappa"], c4["U"])
    b = torch.from_numpy(c4["b"][:1].copy()).cuda()
    del c4
    net = q.Network(lat, 8)
    forms = [("cgnr", "schur", False), ("bicgstab", "schur", False), ("crnr", "schur", False),
             ("cgnr", "full", False), ("bicgstab", "full", False), ("bicgstab", "schur", True),
             ("bicgstab", "full", True), ("fgmres", "full", False), ("fgmres", "full", True),
             ("fgmres", "schur", False), ("fgmres", "schur", True), ("fcg", "full", True), ("fcg", "schur", True)]
    sol = {"cgnr": q.CGNR_EO, "bicgstab": q.BICGSTAB_EO, "crnr": q.CRNR_EO, "fgmres": q.FGMRES_NN, "fcg": q.FCG_NN}
    sysd = {"schur": q.SYSTEM_SCHUR, "full": q.SYSTEM_FULL}
    for solver, system, with_net in forms:
        kw = dict(solver=sol[solver], system=sysd[system], restart=20, maxiter=20000, fallback_cg=0)
        if with_net:
            kw["precond"] = net.handle
        t, st, info, _ = timed_solve(lat, b, reps=2, tol=1e-10, **kw)
        it = info[0]["iterations"]
        _emit({"kind": "compose", "workload": "24^3x48 eps0.5 k0.125 1 gaussian", "solver": solver, "system": system,
               "preconditioner": "network" if with_net else "none", "status": st, "iterations": it,
               "hops": info[0]["hop_applications"], "seconds": round(t, 5),
               "ms_per_iteration": round(1e3 * t / max(it, 1), 4), "true_rel_resid": info[0]["true_rel_resid"]}, path)
    net.close()
    lat.close()


def suite_c64(q, latgen, torch, path, timed_solve, flush, hop_reps=None):
    """The paper's largest lattice, 64^3x128 (the 32^3x64 exp(0.3 i H) links tiled
    2x2x2x2), on one GPU: hop throughput of each storage class, the FP64 hop
    checked on sampled sites against the oracle's single-site hop, and time to a
    1e-10 true residual for plain FP64 eo-CGNR and the mixed forms."""
    import time as _t
    import numpy as np
    from oracle import wilson as W
    t0 = _t.perf_counter()
    cfg = latgen.tiled_config()
    dims, reps = cfg["dims"], cfg["reps"]
    cell = torch.from_numpy(cfg["U_cell"]).cuda()
    U = cell.repeat(reps[3], reps[2], reps[1], reps[0], 1, 1, 1)   # [t][z][y][x][mu][3][3]
    del cell
    lat = q.Lattice(dims, cfg["kappa"], U)
    del U
    b = latgen.device_gaussian_source(100, 0, dims, 1)
    torch.cuda.synchronize()
    log(f"[suite] 64^3x128 inputs and lattice in {_t.perf_counter() - t0:.1f}s")
    for prec in (q.F64, q.F32, q.F16S):
        _emit(hop_rates(q, lat, dims, torch, prec, reps=hop_reps or 20, flush=flush, psi=b), path)
    # sampled-site parity of the FP64 hop (links read through the tiling)
    class Tiled:
        def __init__(self, u, cdims):
            self.u, self.c = u, cdims

        def __getitem__(self, i):
            t, z, y, x = i[0] % self.c[3], i[1] % self.c[2], i[2] % self.c[1], i[3] % self.c[0]
            return self.u[(t, z, y, x) + tuple(i[4:])]
    class DevField:   # reads the device source one site at a time
        def __init__(self, f):
            self.f, self.shape = f, tuple(f.shape)

        def __getitem__(self, i):
            return self.f[i].cpu().numpy()
    Ut = Tiled(cfg["U_cell"], cfg["cell_dims"])
    bsrc = DevField(b[0])
    src = lat.import_field(b, q.ODD, q.F64)
    out = lat.field(q.EVEN, q.F64)
    lat.dslash_eo(out, src, 0, 0, q.F64)
    got = lat.export_field(out, q.EVEN, q.F64)
    rng = np.random.default_rng(64)
    worst = 0.0
    for _ in range(24):
        x = [int(rng.integers(0, L)) for L in dims]
        x[0] = (x[0] & ~1) | ((x[1] + x[2] + x[3]) & 1)   # an even site
        # the 8 neighbours of an even site are odd: the full source stands for its odd half
        want = W.hop_site(Ut, bsrc, tuple(x))
        g = got[0, x[3], x[2], x[1], x[0]].cpu().numpy()
        worst = max(worst, float(np.abs(g - want).max() / np.abs(want).max()))
    del src, out, got
    _emit({"kind": "parity", "workload": "64^3x128 tiled exp(0.3iH)", "what": "FP64 hop on 24 sampled even sites",
           "max_rel_err": worst}, path)
    for name, kw in [("cgnr_f64", dict(inner_prec=q.F64)), ("cgnr_f32", dict(inner_prec=q.F32)),
                     ("cgnr_f16s", dict(inner_prec=q.F16S))]:
        t, st, info, _ = timed_solve(lat, b, reps=1, tol=1e-10, **kw)
        _emit({"kind": "solve", "workload": "64^3x128 tiled exp(0.3iH) k0.12 1rhs", "form": name, "seconds": round(t, 4),
               "status": st, "iterations": info[0]["iterations"], "reliable_updates": info[0]["reliable_updates"],
               "true_rel_resid": info[0]["true_rel_resid"],
               "device_gb": round(torch.cuda.max_memory_allocated() / 1e9, 1)}, path)
    lat.close()


def suite_shard(q, latgen, torch, path, flush, hop_reps=None):
    """One GPU's share of a lattice split along t over 8 GPUs, at its real shape:
    the hop over the local volume, periodic (the exchange of boundary planes is
    not built).  24^3x6 (24^3x48 / 8) takes the first 6 t-slices of the 24^3x48
    links; 64^3x16 (64^3x128 / 8) the first 16 t-slices of the 32^3x64 links,
    tiled twice along x, y and z."""
    c2 = latgen.make_config(2, with_source=False)
    dims = (24, 24, 24, 6)
    lat = q.Lattice(dims, c2["kappa"], c2["U"][:6].copy())
    del c2
    for prec in (q.F64, q.F32, q.F16S):
        rec = hop_rates(q, lat, dims, torch, prec, reps=hop_reps or 200, flush=flush)
        rec["share_of"] = "24^3x48 over 8 GPUs (t split)"
        _emit(rec, path)
    lat.close()
    cell = latgen.make_config(99, with_source=False)
    dims = (64, 64, 64, 16)
    U = torch.from_numpy(cell["U"][:16].copy()).cuda().repeat(1, 2, 2, 2, 1, 1, 1)
    lat = q.Lattice(dims, cell["kappa"], U)
    del U, cell
    b = latgen.device_gaussian_source(101, 0, dims, 1)
    for prec in (q.F64, q.F32, q.F16S):
        rec = hop_rates(q, lat, dims, torch, prec, reps=hop_reps or 20, flush=flush, psi=b)
        rec["share_of"] = "64^3x128 over 8 GPUs (t split)"
        _emit(rec, path)
    lat.close()

if __name__ == "__main__":
    main()
