#!/usr/bin/env python3
"""Throughput of the fused QLA time step on one MI355X.

Workload (default): the cylinder run -- a 4096 x 4096 periodic lattice,
delta = 0.3, Eq. (28) potentials, an E_z Gaussian pulse of width 160 cells
moving in +x toward a centred anisotropic cylinder of radius 400 cells
(tanh edge width 6, n_x, n_y, n_z drawn U[1.2, 3.0] with seed 2), with the
energy and div B diagnostics taken every 500 steps. One "step" is one full
QLA time step of the whole lattice. Inputs are resident in HBM before the
timed region starts.

Prints one JSON line with the site-update rate, the roofline of the step
kernel and the FP64 oracle timed on the host cores on a bounded sample of
the same workload. The step kernel's algorithmic HBM bytes are 24 B read +
24 B written of FP32 state and 12 B of FP32 index per site and launch; a
launch that fuses two steps moves them once for two site-updates, so the
roofline's `frac` is that traffic's rate against the HBM peak, and
`site_update_rate_frac` (site-updates/s x 60 B / peak) the same rate
counted per site-update. For a single-polarisation workload it also times
the polarised kernel (the E_z triple only: 12 B read + 12 B written + 4 B
of n_z per site and launch, results bitwise equal on that triple) and
reports it beside, not as, the headline value.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
ALGO_BYTES_PER_SITE = 60         # 6*4 read + 6*4 written + 3*4 index read
TM_BYTES_PER_SITE = 28           # 3*4 read + 3*4 written + 1*4 index read
DIAG_EVERY = 500
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_cylinder_4096_traffic.json")
# the step kernel, its instances and the host code that plans its launch
KERNEL_SRCS = [os.path.join(ROOT, "paper_2301_13601_amd", "csrc", f)
               for f in ("qla_step.hpp", "qla_step_inst.hip", "qla.hip")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_record(triple: str = "all"):
    """The committed counter summary of a step-kernel instance (triple
    "all" or "tm"): HBM bytes per launch and, when recorded, the VALU busy
    share; None unless it was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("kernels", {}).get(triple)


def measured_traffic(triple: str = "all"):
    """HBM bytes per step-kernel launch from the committed counter runs, if
    they were taken on the current kernel source."""
    rec = measured_record(triple)
    return rec.get("bytes_per_launch") if rec else None


def copy_bandwidth_gbs(dev, mib: int = 1024, reps: int = 5) -> float:
    """Device-to-device copy rate of this GPU (bytes read + written per
    second, best of a few 1 GiB copies): the practical HBM ceiling beside
    the published peak."""
    import torch
    a = torch.empty(mib * (1 << 18), dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del a, b
    return 2.0 * mib * (1 << 20) / best / 1e9


_TRIPLE_NAMES = {"0": "all", "1": "tm", "2": "te"}


def _triple_of(kernel_name: str):
    """Field triple of a step-kernel instance from its demangled name
    (the fifth option of its KOpt), or None for other kernels."""
    import re
    m = re.search(r"qla_step_kernel<\d+, (?:qla_dev::)?KOpt<[^,]+, [^,]+, [^,]+, [^,]+, (\d+), \d+(?:, \d+)?>", kernel_name)
    return _TRIPLE_NAMES.get(m.group(1)) if m else None


SIMDS = 256 * 4                  # MI355X: 256 compute units of 4 SIMDs
XCDS = 8                         # GRBM_GUI_ACTIVE sums the busy cycles of the 8 XCDs
VALU_CYCLES = 4                  # a wave64 VALU instruction holds a 16-lane SIMD 4 cycles


def summarize_counters(fetch_csv: str, write_csv: str, copy_mib: int, out_path: str, sq_csv: str = None) -> dict:
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per
    dispatch) of this script into HBM bytes per step-kernel launch, per
    kernel instance (all six components, TM triple), scaled by what the same
    counters read for the plain device copy of copy_mib MiB the runs include
    (--calib-copy-mib). With a third run of SQ_INSTS_VALU and
    GRBM_GUI_ACTIVE, also the share of the SIMDs' cycles that issued VALU
    instructions during the step kernel (valu_busy)."""
    import csv

    def rows(path):
        with open(path) as f:
            return list(csv.DictReader(f))

    copy_bytes = copy_mib * (1 << 20)
    out = {"kernel_source_sha256_16": kernel_source_hash(), "copy_bytes": copy_bytes, "kernels": {}}
    for tag, path in (("fetch", fetch_csv), ("write", write_csv)):
        rs = rows(path)
        # the calibration copy is the largest copy dispatch of the run
        copies = [float(r["Counter_Value"]) for r in rs if "copy" in r["Kernel_Name"].lower()]
        cal = max(copies) * 1024.0
        factor = copy_bytes / cal
        per = {}
        for r in rs:
            t = _triple_of(r["Kernel_Name"])
            if t is not None:
                per.setdefault(t, []).append(float(r["Counter_Value"]))
        for t, vals in per.items():
            k = out["kernels"].setdefault(t, {})
            k[tag] = {"kib_per_launch_raw": sum(vals) / len(vals), "launches": len(vals),
                      "copy_kib_raw": cal / 1024.0, "scale": factor,
                      "bytes_per_launch": sum(vals) / len(vals) * 1024.0 * factor}
    for k in out["kernels"].values():
        if "fetch" in k and "write" in k:
            k["bytes_per_launch"] = k["fetch"]["bytes_per_launch"] + k["write"]["bytes_per_launch"]
    if sq_csv:
        per = {}
        for r in rows(sq_csv):
            t = _triple_of(r["Kernel_Name"])
            if t is not None:
                per.setdefault(t, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        for t, cs in per.items():
            valu = sum(cs["SQ_INSTS_VALU"]) / len(cs["SQ_INSTS_VALU"])
            grbm = sum(cs["GRBM_GUI_ACTIVE"]) / len(cs["GRBM_GUI_ACTIVE"])
            k = out["kernels"].setdefault(t, {})
            k["sq_insts_valu_per_launch"] = valu
            k["grbm_gui_active_per_launch"] = grbm
            k["valu_busy"] = valu * VALU_CYCLES / (SIMDS * grbm / XCDS)
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    return out


def make_workload(name: str, steps: int):
    from paper_2301_13601_amd import scenes
    if name == "cylinder_4096":
        sc = scenes.config_scale(seed=2, N=4096, steps=steps)
        desc = ("cylinder_4096: 4096x4096 periodic lattice, delta=0.3, Eq.(28) potentials, "
                "E_z pulse width 160 at x0=1024, disk radius 400 edge 6, n~U[1.2,3.0] seed 2, "
                "energy+divB every 500 steps")
    elif name == "batch_64":
        specs = scenes.batch_instance_specs(64, seed=3)
        scs = [scenes.scene_from_spec(sp, steps=steps) for sp in specs]
        desc = ("batch_64: 64 periodic lattices, sides ~U{512,768,1024,1536,2048} (seed 3), "
                "n_c~U[1.1,3.5], ellipse/rectangle/two-disk objects edge 6, E_y or E_z pulse "
                "width 20, delta=0.3, Eq.(28) potentials, one launch per step for the whole batch, "
                "energy+divB every 500 steps")
        return scs, desc
    elif name == "single_256":
        sc = scenes.config_single()
        desc = ("single_256: 256x256 periodic lattice, delta=0.3, Eq.(28) potentials, E_z pulse "
                "width 20 at x0=48, ellipse 30x20 edge 6, n=(1.5,2.0,3.0), energy+divB every 500 steps")
    else:
        raise SystemExit(f"unknown workload {name}")
    return sc, desc


def cpu_baseline(sc, sample_steps: int, sample_n: int, pot_mode: str = "eq28", v_form: str = "printed",
                 one_core_n: int = 1024, one_core_steps: int = 6):
    """The FP64 oracle on the host cores, on a sample of the workload: the
    same scene generator at sample_n x sample_n for sample_steps steps on
    every host thread; beside it the same on one thread (one_core_n^2 for
    one_core_steps steps) and the whole 256 x 256, 500-step parity run (the
    elliptic-object scene) on every thread."""
    from oracle import oracle as O
    from paper_2301_13601_amd import scenes

    def sample(N, steps):
        if N == sc.nx:
            return sc.n, sc.q
        s2 = scenes.config_scale(seed=2, N=N, steps=steps)
        return s2.n, s2.q

    def timed(n, q, delta, steps, nthreads):
        n32 = n.astype(np.float32).astype(np.float64)
        q32 = q.astype(np.float32).astype(np.float64)
        t0 = time.perf_counter()
        O.run(n32, q32, delta, steps, pot_mode, "phys", nthreads=nthreads, v_form=v_form)
        return time.perf_counter() - t0

    threads = O.threads(0)
    n, q = sample(sample_n, sample_steps)
    dt = timed(n, q, sc.delta, sample_steps, threads)
    rate = sample_n * sample_n * sample_steps / dt
    n1, q1 = sample(one_core_n, one_core_steps)
    dt1 = timed(n1, q1, sc.delta, one_core_steps, 1)
    O.threads(threads)
    c1 = scenes.config_single()
    dtc = timed(c1.n, c1.q, c1.delta, c1.steps, threads)
    sites_c1 = c1.nx * c1.ny * c1.steps
    return {"value": rate, "unit": "site-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample_n}x{sample_n} lattice of the same scene family, {sample_steps} steps, "
                      f"{dt:.1f} s wall, FP64, OpenMP over {threads} threads",
            "one_core": {"value": one_core_n * one_core_n * one_core_steps / dt1, "unit": "site-updates/s",
                         "cores": 1, "sample": f"{one_core_n}x{one_core_n}, {one_core_steps} steps, {dt1:.1f} s wall"},
            "single_256_full_run": {"seconds": dtc, "value": sites_c1 / dtc, "unit": "site-updates/s",
                                    "cores": threads,
                                    "sample": "the whole 256x256 elliptic-object run, 500 steps (parity scene)"}}


def is_tm_only(q) -> bool:
    """True if the state lives in the E_z triple (q0 = q1 = q5 = 0)."""
    return all(not np.any(q[c]) for c in (0, 1, 5))


def time_polarised(make_sim, stream, sites: int, steps: int, warmup: int, traffic=None) -> dict:
    """The same workload on the polarised kernel (TM triple only), timed
    like the headline run (whole job on the wall clock, kernel time from
    HIP events on the launch stream)."""
    import torch
    sim = make_sim("tm")
    sim.step(warmup)
    torch.cuda.synchronize()
    sim.close()
    sim = make_sim("tm")
    torch.cuda.synchronize()
    ev = []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(DIAG_EVERY, steps - done)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        sim.step(k)
        b.record(stream)
        ev.append((a, b, k))
        done += k
        sim.diagnostics()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    spp = sim.launch()["steps_per_pass"]
    avg = sum(a.elapsed_time(b) for a, b, _ in ev) / 1e3 / (steps // spp)
    sim.close()
    achieved = sites * TM_BYTES_PER_SITE / avg / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "avg_launch_us": avg * 1e6,
            "steps_per_launch": spp, "algo_bytes_per_launch": sites * TM_BYTES_PER_SITE,
            "site_update_rate_frac": spp * sites * TM_BYTES_PER_SITE / avg / 1e9 / HBM_PEAK_GBS}
    if traffic:
        roof["traffic_gbs"] = traffic / avg / 1e9
        roof["traffic_frac"] = roof["traffic_gbs"] / HBM_PEAK_GBS
    return {"polarisation": "tm (q2, q3, q4 = n_z E_z, B_x, B_y)", "steps": steps,
            "value": sites * steps / wall, "unit": "site-updates/s", "roofline": roof}


def sweep_workload(args) -> dict:
    """Surrogate-accelerated sweep against plain QLA on the same GPU.

    Trains the U-net surrogate on QLA runs the library generates (2048 runs
    at 256 x 256, snapshots every K = 256 steps) or loads the weights a
    previous run saved (--net-file), evaluates it on 256 held-out runs, then
    advances --sweep-lattices lattices of --sweep-side^2 (the batched scene
    family, seed 5) by --steps steps: plain QLA; the checked sweep (QLA
    checks at the first and every --check-every-th jump, fallback when the
    field or energy error of a check exceeds the tolerance) at each of
    --tolerances; and surrogate jumps with no checks.
    value = plain QLA seconds / checked-sweep seconds at the last (tightest)
    tolerance, 1e-3 by default, at the final field error the record states
    (max over lattices of |Q - Q_plain| / |Q_plain|)."""
    import torch
    from paper_2301_13601_amd import qnn, scenes, surrogate as S

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    K = 256
    tols = [float(v) for v in args.tolerances.split(",")]
    log = lambda msg: print(f"[sweep] {msg}", file=sys.stderr, flush=True)
    last = [time.perf_counter()]

    def tick(k):
        # a progress line at most every 20 s of a long sweep
        if time.perf_counter() - last[0] > 20.0:
            last[0] = time.perf_counter()
            log(f"  {k} steps")
    net = S.UNet(seed=0)
    netrec = {"train_runs": 2048}
    if args.net_file and os.path.exists(args.net_file):
        with np.load(args.net_file) as z:
            net.load({k: z[k] for k in z.files})
        netrec.update({"loaded_from": os.path.basename(args.net_file), "train_steps": int(net.t)})
        log(f"network loaded from {args.net_file} ({net.t} Adam steps)")
    else:
        t0 = time.perf_counter()
        data = S.generate(2048, seed=11, L=256, K=K, snaps=9)
        netrec["data_seconds"] = time.perf_counter() - t0
        log(f"data: {netrec['data_seconds']:.1f} s")
        t0 = time.perf_counter()
        S.train(net, data, steps=args.train_steps, batch=16, lr=args.lr, seed=1, log_every=5000,
                log=lambda r: log(f"train step {r['step']} loss {r['loss']:.4f}"
                                  + (f" rolled back, lr x{r['lr_scale']:g}" if r.get("rolled_back") else "")))
        torch.cuda.synchronize()
        netrec.update({"train_steps": args.train_steps, "peak_lr": args.lr, "train_seconds": time.perf_counter() - t0})
        del data
        if args.net_file:
            np.savez(args.net_file, **net.state())
    held = S.generate(256, seed=999, L=256, K=K, snaps=9)
    err = S.evaluate(net, held)
    del held
    netrec.update({"heldout_median_error": float(np.median(err)), "heldout_p90_error": float(np.percentile(err, 90)),
                   "macs_per_pixel": S.macs_per_pixel()})
    log(f"held-out median error {netrec['heldout_median_error']:.4f}")

    L, B, steps = args.sweep_side, args.sweep_lattices, args.steps
    specs = scenes.batch_instance_specs(B, seed=5, sides=(L,))
    # one device tensor each for every lattice's n and initial Q, filled a
    # lattice at a time (a 256 x 2048^2 batch would not fit host memory in
    # FP64 at once); the lists hold views of them
    n_all = torch.empty((B, 3, L, L), dtype=torch.float32, device=dev)
    q_all = torch.empty((B, 6, L, L), dtype=torch.float32, device=dev)
    for k, sp in enumerate(specs):
        sc = scenes.scene_from_spec(sp, steps=steps)
        n_all[k].copy_(torch.as_tensor(sc.n.astype(np.float32)))
        q_all[k].copy_(torch.as_tensor(sc.q.astype(np.float32)))
        delta = sc.delta
    ns, qs = list(n_all), list(q_all)
    log(f"{B} scenes of {L}x{L} on the device")

    # forward throughput of the network on these lattices (one chunk)
    c = min(B, S.default_chunk(L, L))
    cur = q_all[:c].clone()
    n_dev = n_all[:c]
    out = torch.empty_like(cur)
    net.predict(cur, n_dev, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(net.stream)
    net.predict(cur, n_dev, out)
    e1.record(net.stream)
    torch.cuda.synchronize()
    fwd_s = e0.elapsed_time(e1) / 1e3
    del cur, out, n_dev

    plain_out = torch.empty((B, 6, L, L), dtype=torch.float32, device=dev)
    plain_s, _ = S.plain(ns, qs, delta, steps, stream=net.stream, out=plain_out,
                         progress=lambda k: log(f"plain QLA: {k} steps"))
    log(f"plain QLA {plain_s:.1f} s")
    rel = torch.empty(B, dtype=torch.float64, device=dev)
    en = torch.empty(B, dtype=torch.float64, device=dev)
    work = torch.empty(qnn.qnn_compare_work_doubles(B), dtype=torch.float64, device=dev)
    fin = torch.empty_like(plain_out)

    def final_error():
        qnn.qnn_compare(B, 6 * L * L, fin, plain_out, rel, en, work, net.stream)
        return float(rel.max().item())

    def record(res, tol=None):
        r = {"seconds": res.seconds, "speedup": plain_s / res.seconds, "final_field_error": final_error(),
             "jumps": res.jumps, "unchecked": res.unchecked, "checks": res.checks, "rejected": res.rejected,
             "fell_back": res.fell_back, "max_check_error": res.max_check_error,
             "max_check_energy": res.max_check_energy, "energy_change": res.energy_change}
        if tol is not None:
            r = {"tolerance": tol, **r}
        return r

    table = []
    for tol in tols:
        res, _ = S.sweep(net, ns, qs, delta, steps, K=K, window=args.sweep_window, check_every=args.check_every,
                         tol=tol, out=fin, progress=tick)
        table.append(record(res, tol))
        log(f"tol {tol:g}: {table[-1]['speedup']:.2f}x, final error {table[-1]['final_field_error']:.3e}, "
            f"fell back {res.fell_back}")
    unchecked = None
    if not args.no_unchecked:
        free, _ = S.sweep(net, ns, qs, delta, steps, K=K, check_every=0, out=fin, progress=tick)
        unchecked = record(free)
        log(f"unchecked: {unchecked['speedup']:.2f}x, final error {unchecked['final_field_error']:.3e}")
    stated = table[-1]
    return {
        "metric": "surrogate vs plain QLA speedup at stated field error",
        "value": stated["speedup"],
        "unit": "x",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 QLA, bf16 x bf16 -> f32 network",
        "data": "synthetic",
        "stated_error": stated["final_field_error"],
        "config": {"workload": f"sweep: {B} lattices of {L}x{L} (batched scene family, seed 5), {steps} steps, "
                               f"surrogate jumps of K={K}, QLA windows of {args.sweep_window} steps, checks at the "
                               f"first and every {args.check_every}th jump, fallback at {stated['tolerance']:g} "
                               "field or energy error",
                   "fallback_tolerance": stated["tolerance"]},
        "checked_sweeps": table,
        "unchecked_sweep": unchecked,
        "plain_qla": {"seconds": plain_s, "site_updates_per_s": B * L * L * steps / plain_s},
        "network": {**netrec,
                    "forward_seconds_per_pixel": fwd_s / (c * L * L),
                    "forward_tflops": 2.0 * S.macs_per_pixel() * c * L * L / fwd_s / 1e12,
                    "qla_seconds_per_site_for_K_steps": plain_s / steps * K / (B * L * L)},
    }


def unet_workload(args) -> dict:
    """Inference throughput of the surrogate network (the U-net of the
    sweep, random-init weights: the cost does not depend on their values).

    --unet-lattices lattices of 1024 x 1024 from the batched scene family
    (seed 5) are packed, run through the network and unpacked; one "step"
    is one such pass over the whole batch. value = pixels/s; the roofline
    is the BF16 matrix-core peak, with 2 x (multiply-accumulates per pixel)
    flops per pixel. Also times training steps (batch 16 x 256^2) beside
    the headline. The CPU baseline is the FP64 oracle network on one
    --cpu-unet-side square sample."""
    import torch
    from paper_2301_13601_amd import scenes, surrogate as S

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    L, B = 1024, args.unet_lattices
    specs = scenes.batch_instance_specs(B, seed=5, sides=(L,))
    scs = [scenes.scene_from_spec(sp, steps=0) for sp in specs]
    q = torch.as_tensor(np.stack([s.q.astype(np.float32) for s in scs])).to(dev)
    n = torch.as_tensor(np.stack([s.n.astype(np.float32) for s in scs])).to(dev)
    out = torch.empty_like(q)
    net = S.UNet(seed=0)
    for _ in range(args.warmup):
        net.predict(q, n, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(net.stream)
    for _ in range(args.steps):
        net.predict(q, n, out)
    e1.record(net.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sec = e0.elapsed_time(e1) / 1e3 / args.steps
    pixels = B * L * L
    flop = 2.0 * S.macs_per_pixel() * pixels
    rec = {
        "metric": "surrogate inference pixels/s",
        "value": pixels / sec,
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "wall_s": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 x bf16 -> f32",
        "data": "synthetic (batched scene family, random-init weights)",
        "config": {"workload": f"unet_forward: {B} lattices of {L}x{L}, one network pass each (pack, "
                               "U-net 32/64/128/128 with fused decoder steps, unpack)",
                   "macs_per_pixel": S.macs_per_pixel(), "seconds_per_pixel": sec / pixels},
        "roofline": {"bound": "mfma", "achieved": flop / sec / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": flop / sec / 1e12 / 2500.0, "traffic": None,
                     "kernel": "whole network pass (the convolution kernels: ~90 % of it)"},
    }
    # training steps (forward, relative-L2 loss, backward, Adam) at batch 16
    # x 256^2 on pairs the library generates; flops per step: forward + data
    # gradient (every layer but the first) + weight gradient
    data = S.generate(64, seed=11, L=256, K=256, snaps=3)
    S.train(net, data, steps=3, batch=16, lr=1e-3, seed=1, log_every=0)
    torch.cuda.synchronize()
    tsteps = max(10, args.steps)
    t0 = time.perf_counter()
    S.train(net, data, steps=tsteps, batch=16, lr=1e-3, seed=2, log_every=0)
    torch.cuda.synchronize()
    tstep = (time.perf_counter() - t0) / tsteps
    macs = sum(sp.n_w / 4 ** sp.level * (2 if sp.name == "e0a" else 3) for sp in S.layer_specs())
    tflop = 2.0 * macs * 16 * 256 * 256
    rec["training"] = {"batch": 16, "side": 256, "steps": tsteps, "ms_per_step": tstep * 1e3,
                       "macs_per_pixel": macs, "tflops": tflop / tstep / 1e12,
                       "note": "wall clock per step, host loop included"}
    if not args.no_cpu_baseline:
        from oracle import nn_oracle as NO
        from threadpoolctl import threadpool_info
        side = args.cpu_unet_side
        rng = np.random.default_rng(7)
        x = rng.standard_normal((1, side, side, 48))
        x[..., 33:] = 0
        p = net.p.cpu().numpy().astype(np.float64)
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        t0 = time.perf_counter()
        NO.unet_forward(p, x, bf16=True)
        dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": side * side / dt, "unit": "pixels/s", "cores": threads, "kind": "oracle",
                               "sample": f"one {side}x{side} sample through the FP64 oracle network "
                                         f"(numpy, BLAS threads), {dt:.1f} s"}
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 20000; batch_64 5000; sweep 4096; unet_forward 20 passes)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps first (default 100; unet_forward 3)")
    ap.add_argument("--workload", default="cylinder_4096",
                    choices=["cylinder_4096", "single_256", "batch_64", "sweep", "unet_forward"])
    ap.add_argument("--train-steps", type=int, default=20000, help="sweep workload: network training steps")
    ap.add_argument("--lr", type=float, default=1e-3, help="sweep workload: peak Adam learning rate")
    ap.add_argument("--sweep-lattices", type=int, default=16, help="sweep workload: lattices per sweep")
    ap.add_argument("--sweep-side", type=int, default=1024, help="sweep workload: lattice side")
    ap.add_argument("--sweep-window", type=int, default=0, help="sweep workload: QLA steps after each jump")
    ap.add_argument("--check-every", type=int, default=4, help="sweep workload: QLA check every n-th jump")
    ap.add_argument("--tolerances", default="1e-1,3e-2,1e-2,3e-3,1e-3",
                    help="sweep workload: fallback tolerances of the checked sweeps (the last is the stated one)")
    ap.add_argument("--no-unchecked", action="store_true", help="sweep workload: skip the unchecked sweep")
    ap.add_argument("--net-file", default="",
                    help="sweep workload: load the network from this .npz if it exists, else train and save it")
    ap.add_argument("--unet-lattices", type=int, default=16, help="unet_forward workload: lattices of 1024 x 1024")
    ap.add_argument("--cpu-unet-side", type=int, default=1024, help="unet_forward: side of the oracle's sample")
    ap.add_argument("--pot-mode", choices=["eq28", "eq23"], default="eq28",
                    help="placement of the potentials: Eq. (28) (default) or Eq. (23)")
    ap.add_argument("--v-form", choices=["printed", "skew"], default="printed",
                    help="potentials as printed (default) or their skew-symmetric form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batch_64: keep the library's default launch geometry instead of the autotuned one")
    ap.add_argument("--cpu-sample-steps", type=int, default=18,
                    help="oracle steps of the CPU baseline (about 10 s on 16 host threads at 4096^2)")
    ap.add_argument("--cpu-sample-n", type=int, default=4096)
    ap.add_argument("--polarised-steps", type=int, default=2000,
                    help="steps of the polarised (E_z triple) kernel timed after the headline run; 0 skips")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    ap.add_argument("--counters", nargs="+", metavar="CSV",
                    help="FETCH_CSV WRITE_CSV COPY_MIB [SQ_CSV]: summarise rocprofv3 counter CSVs into the "
                         "committed traffic record and exit")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = {"sweep": 4096, "unet_forward": 20, "batch_64": 5000}.get(args.workload, 20000)
    if args.warmup is None:
        args.warmup = 3 if args.workload == "unet_forward" else 100

    if args.counters:
        c = args.counters
        if len(c) not in (3, 4):
            raise SystemExit("--counters takes FETCH_CSV WRITE_CSV COPY_MIB [SQ_CSV]")
        rec = summarize_counters(c[0], c[1], int(c[2]), TRAFFIC_FILE, c[3] if len(c) == 4 else None)
        print(json.dumps(rec))
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the lattice step is a single-GPU kernel here).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2301_13601_amd import qla

    if args.workload == "sweep":
        print(json.dumps(sweep_workload(args)), flush=True)
        return
    if args.workload == "unet_forward":
        print(json.dumps(unet_workload(args)), flush=True)
        return

    sc, desc = make_workload(args.workload, args.steps)
    if args.pot_mode != "eq28":
        desc = desc.replace("Eq.(28) potentials", "Eq.(23) potentials")
    if args.v_form != "printed":
        desc = desc.replace(" potentials", " skew-symmetric potentials", 1)
    batch = isinstance(sc, list)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)

    def make_sim(pol="both"):
        if batch:
            return qla.Batch([s.n.astype(np.float32) for s in sc], [s.q.astype(np.float32) for s in sc],
                             [s.delta for s in sc], args.pot_mode, "phys", device="cuda:0", stream=stream,
                             v_form=args.v_form)
        n32, q32 = sc.as_f32()
        return qla.Simulation(n32, q32, sc.delta, args.pot_mode, "phys", device="cuda:0", stream=stream,
                              polarisation=pol, v_form=args.v_form)

    sim = make_sim()
    sites = sim.sites if batch else sc.nx * sc.ny
    tuned = None
    if batch and not args.no_autotune:
        # the batched workload runs with autotuned launch geometry (measured
        # here, before the warmup; cached per GPU and lattice shapes)
        from paper_2301_13601_amd import autotune
        rec = autotune.tune([s.n for s in sc], [s.delta for s in sc])
        tuned = rec["launch"]

    # warmup (then restore the initial state so the timed run is the workload)
    if tuned:
        sim.set_launch(**tuned)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    sim.close()
    sim = make_sim()
    if tuned:
        sim.set_launch(**tuned)

    def energy_and_divb():
        ds = sim.diagnostics() if batch else [sim.diagnostics()]
        e = sum(d["energy"] for d in ds)
        r = max((d["divB_max"] / d["B_max"]) if d["B_max"] > 0 else 0.0 for d in ds)
        return e, r, ds[0]["step"]

    e_start, _, _ = energy_and_divb()
    torch.cuda.synchronize()

    # timed region: the whole job, diagnostics included
    ev_pairs = []
    log = []
    done = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while done < args.steps:
        k = min(DIAG_EVERY, args.steps - done)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(k)
        e1.record(stream)
        ev_pairs.append((e0, e1, k))
        done += k
        if done % DIAG_EVERY == 0 or done == args.steps:
            e, r, st = energy_and_divb()
            log.append({"step": st, "energy": e, "divB_ratio": r})
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    kernel_ms = sum(a.elapsed_time(b) for a, b, _ in ev_pairs)
    spp = sim.launch()["steps_per_pass"]
    if any(k % spp for _, _, k in ev_pairs):
        raise SystemExit(f"--steps must be a multiple of {spp} (steps per launch) for the launch timing")
    launches = sum(k for _, _, k in ev_pairs) // spp
    avg_launch_s = kernel_ms / 1e3 / launches

    if args.calib_copy_mib > 0:
        nb = args.calib_copy_mib * (1 << 20)
        a = torch.empty(nb // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    value = sites * args.steps / wall
    # Algorithmic HBM bytes of one launch: whatever number of steps a launch
    # fuses (spp), it has to read Q and n once and write Q once, 60 B per
    # site. Per site-update that is 60 / spp B.
    algo_bytes = sites * ALGO_BYTES_PER_SITE
    achieved = algo_bytes / avg_launch_s / 1e9
    # the committed counters were taken on the default kernel instance
    default_kernel = args.pot_mode == "eq28" and args.v_form == "printed"
    rec = measured_record("all") if args.workload == "cylinder_4096" and default_kernel else None
    traffic = rec.get("bytes_per_launch") if rec else None
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "qla_step_kernel", "avg_launch_us": avg_launch_s * 1e6, "steps_per_launch": spp,
                "algo_bytes_per_launch": algo_bytes,
                "algo_bytes_per_site_update": ALGO_BYTES_PER_SITE / spp,
                # the metric's %HBM roofline: site-updates/s x 60 B / peak. A
                # rate, not a bandwidth: above 1 once a launch fuses steps
                "site_update_rate_frac": spp * sites * ALGO_BYTES_PER_SITE / avg_launch_s / 1e9 / HBM_PEAK_GBS,
                "copy_gbs": copy_bandwidth_gbs(dev)}
    if traffic:
        roofline["traffic_gbs"] = traffic / avg_launch_s / 1e9
        roofline["traffic_frac"] = roofline["traffic_gbs"] / HBM_PEAK_GBS
    if rec and "valu_busy" in rec:
        roofline["valu_busy"] = rec["valu_busy"]

    out = {
        "metric": "lattice site-updates/s",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "sites_per_step": sites, "launch": sim.launch(), "autotuned": bool(tuned),
                   "energy_drift": log[-1]["energy"] / e_start - 1 if log else 0.0,
                   "divB_ratio_final": log[-1]["divB_ratio"] if log else 0.0},
        "roofline": roofline,
    }
    sim.close()
    if args.polarised_steps > 0 and not batch and is_tm_only(sc.q):
        out["polarised"] = time_polarised(make_sim, stream, sites, args.polarised_steps, args.warmup,
                                          measured_traffic("tm") if args.workload == "cylinder_4096" and default_kernel
                                          else None)
    if not args.no_cpu_baseline:
        first = sc[0] if batch else sc
        sample_n = min(args.cpu_sample_n, first.nx)
        out["cpu_baseline"] = cpu_baseline(first, args.cpu_sample_steps, sample_n, args.pot_mode, args.v_form)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
