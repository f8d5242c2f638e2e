#!/usr/bin/env python3
"""Throughput of the fused multiphase lattice Boltzmann step on one MI355X.

Workload: 3-D Rayleigh-Taylor instability, D3Q27 cumulant flow + D3Q27
conservative Allen-Cahn populations, 128 x 128 x 512 lattice, periodic in x/y,
no-slip walls in z, Atwood 0.5, Re 1000, W 5, mobility 0.1, interface at
z = 256 with a two-mode cosine perturbation of amplitude 0.05 * 128, FP32
storage and arithmetic.  A "step" advances both population sets of every
cell by one time step (the order-parameter pass plus the fused collision).

Prints one JSON line: MLUPS (million lattice-cell updates per second) with a
roofline entry for the dominant kernel (fused collision, HBM-bound) and the
FP64 CPU oracle's rate on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# algorithmic bytes per cell for one launch of each kernel, FP32, D3Q27:
#   collide: read 27 f' + 27 g + phi, write 27 f' + 27 g  -> 4 * (27 * 4 + 1) = 436
#   phi:     read 27 g, write phi                          -> 4 * (27 + 1)     = 112
ALG_BYTES = {("fp32", 3): {"collide": 436, "phi": 112, "method": 440},
             ("fp64", 3): {"collide": 872, "phi": 224, "method": 880},
             ("fp16s", 3): {"collide": 2 * 27 * 2 + 2 * 27 * 4 + 4 + 8 * 2, "phi": 27 * 4 + 4,
                            "method": 340},
             ("fp32", 2): {"collide": 4 * (2 * 2 * 9 + 1), "phi": 4 * (9 + 1), "method": 152},
             ("fp64", 2): {"collide": 8 * (2 * 2 * 9 + 1), "phi": 8 * (9 + 1), "method": 304}}


def cpu_baseline(case_fn, min_seconds=10.0):
    """The FP64 oracle on a 128 x 128 x 128 slab of the same workload (the
    interface region), stepped until at least min_seconds have elapsed."""
    import oracle

    case = case_fn(nz=128)
    p = oracle.params_from_dict(case.params)
    f, g = oracle.init(p, case.phi, case.u, case.p)
    steps, t0 = 0, time.perf_counter()
    while True:
        f, g = oracle.step(p, f, g, 1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds:
            break
    return {"value": case.ncells * steps / el / 1e6, "unit": "MLUPS",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "%d step(s) of a 128x128x128 slab (%d cells) of the same Rayleigh-Taylor "
                      "case, FP64, %.1f s" % (steps, case.ncells, el)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp64", "fp16s"])
    ap.add_argument("--nz", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="instead of the benchmark, time a plain device-to-device copy of this "
                         "many MiB (reference kernel for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2101_06769_amd import inputs, mplb

    torch.cuda.set_device(0)
    if args.copy_probe:
        n = args.copy_probe << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(json.dumps({"copy_probe_bytes": n, "ms": ms, "GBs_read_plus_write": 2 * n / ms / 1e6}))
        return
    case = inputs.rti3d(nz=args.nz)
    N = case.ncells
    s = mplb.Solver(case.params, storage=args.storage)
    s.init(case.phi, case.u, case.p)
    s.step(args.warmup)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s.stream)
    ms_phi, ms_col = s.step_timed(args.steps)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    ms_step = ms / args.steps
    mlups = N * args.steps / (ms / 1e3) / 1e6

    red, rc = s.reduce()
    m0 = float(case.phi.sum())
    ab = ALG_BYTES[(args.storage, 3)]
    t_col = ms_col / args.steps / 1e3
    achieved = ab["collide"] * N / t_col / 1e9
    line = {
        "metric": "MLUPS (flow+phase field) and % HBM roofline at fixed error vs FP64",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "fp16s": "f16s+f32"}[args.storage],
        "data": "synthetic",
        "config": {"workload": "3-D Rayleigh-Taylor, D3Q27 cumulant + D3Q27 Allen-Cahn, "
                               "128x128x%d, At 0.5, Re 1000, W 5, %s storage" % (args.nz,
                                                                                args.storage),
                   "cells": N, "lattice": "D3Q27+D3Q27", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_collide", "alg_bytes_per_cell": ab["collide"],
                     "avg_launch_us": round(t_col * 1e6, 2),
                     "phi_pass_avg_launch_us": round(ms_phi / args.steps * 1e3, 2)},
        "method_alg_GBs": round(ab["method"] * N * args.steps / (ms / 1e3) / 1e9, 1),
        "phase_mass_rel_drift": abs(red[0] - m0) / m0,
        "status": "ok" if rc == mplb.OK else "unstable",
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(lambda nz: inputs.rti3d(nz=nz, amp=0.05 * 128),
                                            args.cpu_seconds)
        line["cpu_baseline"]["gpu_speedup"] = round(mlups / line["cpu_baseline"]["value"], 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
