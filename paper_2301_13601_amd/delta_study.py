"""The perturbation-parameter study of Sec. 3.1 and 4: the scattering scene
of the 256 x 256 run, held fixed in physical units, advanced with delta =
0.3, 0.1 and 0.03 for the same physical time, with both placements of the
potentials (Eq. (23) and Eq. (28)), logging the energy of Eq. (27) and the
divergence diagnostics over time.

Physical units: one cell is delta and one step is delta^2 (the ordering of
Eq. (26)). The scene at delta = 0.3 is the 256 x 256 run (domain 76.8,
ellipse semi-axes 9 x 6 with tanh edge 1.8, n = (1.5, 2.0, 3.0), pulse
width 6 starting at x = 14.4); at delta = 0.1 the same scene is 768 x 768
cells and at 0.03 it is 2560 x 2560. The E_z pulse (TM triple) logs
max|div B| / max|B|; the E_y pulse (TE triple) logs max|div D| / max|D|.
Polarised contexts advance only the live triple (bitwise the full method).

Every number comes from the HIP library through its C ABI. Run as

    python -m paper_2301_13601_amd.delta_study [--time T] [--logs N]

which prints one JSON record per (delta, placement, polarisation, form).
"""
from __future__ import annotations

import argparse
import json
import time
from typing import Dict, List, Sequence

import numpy as np

from . import qla, scenes

DOMAIN = 76.8          # physical side (256 cells at delta = 0.3)
SEMI_AXES = (9.0, 6.0)
EDGE = 1.8
N_OBJ = (1.5, 2.0, 3.0)
PULSE_X0 = 14.4
PULSE_W = 6.0


def scene(delta: float, pol: str):
    """(n, q0) of the scene at lattice spacing delta (cells = DOMAIN/delta)."""
    N = int(round(DOMAIN / delta))
    n = scenes.object_profile(N, N, "ellipse", (SEMI_AXES[0] / delta, SEMI_AXES[1] / delta), N_OBJ,
                              EDGE / delta)
    q = scenes.gaussian_pulse(N, N, pol, x0=PULSE_X0 / delta, width=PULSE_W / delta)
    return n.astype(np.float32), q.astype(np.float32)


def run_one(delta: float, mode: str, pol: str, t_end: float, logs: int, v_form: str = "printed",
            coarse: float = 0.3) -> Dict:
    """Advance one configuration to physical time t_end, logging `logs`
    times; also returns the final E_z (or E_y) field sampled on the coarse
    grid (every coarse/delta-th cell) for cross-delta comparison."""
    n, q = scene(delta, pol)
    triple = "tm" if pol == "Ez" else "te"
    sim = qla.Simulation(n, q, delta, mode, "phys", polarisation=triple, v_form=v_form)
    steps_total = int(round(t_end / delta ** 2))
    d0 = sim.diagnostics()
    e0 = d0["energy"]
    log = []
    done = 0
    t0 = time.perf_counter()
    for k in range(1, logs + 1):
        target = int(round(steps_total * k / logs))
        sim.step(target - done)
        done = target
        d = sim.diagnostics()
        rec = {"t": done * delta ** 2, "steps": done, "energy_rel": d["energy"] / e0 - 1.0}
        if pol == "Ez":
            rec["divB_ratio"] = d["divB_max"] / d["B_max"] if d["B_max"] > 0 else 0.0
        else:
            rec["divD_ratio"] = d["divD_max"] / d["D_max"] if d["D_max"] > 0 else 0.0
        log.append(rec)
    secs = time.perf_counter() - t0
    fields = sim.fields("EB")
    sim.close()
    stride = int(round(coarse / delta))
    comp = 2 if pol == "Ez" else 1
    sample = fields[comp, ::stride, ::stride].astype(np.float64)
    return {"delta": delta, "placement": mode, "polarisation": pol, "v_form": v_form,
            "cells": int(n.shape[1]), "steps": done, "seconds": secs, "log": log, "_sample": sample}


def study(deltas: Sequence[float] = (0.3, 0.1, 0.03), modes: Sequence[str] = ("eq23", "eq28"),
          pols: Sequence[str] = ("Ez", "Ey"), forms: Sequence[str] = ("printed",), t_end: float = 45.0,
          logs: int = 10) -> List[Dict]:
    """All configurations; each record also carries, for every delta but the
    smallest, the max difference of its sampled field from the smallest
    delta's run of the same configuration, relative to that field's max."""
    out = []
    for form in forms:
        for pol in pols:
            for mode in modes:
                recs = [run_one(d, mode, pol, t_end, logs, form) for d in deltas]
                ref = recs[-1]["_sample"]
                for r in recs:
                    r["field_diff_vs_finest"] = float(np.abs(r["_sample"] - ref).max() / np.abs(ref).max())
                    del r["_sample"]
                out += recs
    return out


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--time", type=float, default=45.0, help="physical end time (500 steps at delta 0.3)")
    ap.add_argument("--logs", type=int, default=10)
    ap.add_argument("--deltas", type=float, nargs="+", default=[0.3, 0.1, 0.03])
    ap.add_argument("--forms", nargs="+", default=["printed", "skew"])
    args = ap.parse_args(argv)
    for rec in study(args.deltas, forms=args.forms, t_end=args.time, logs=args.logs):
        print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
