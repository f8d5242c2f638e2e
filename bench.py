#!/usr/bin/env python3
"""Throughput of the multiphase lattice Boltzmann step on one MI355X.

Workload: 3-D Rayleigh-Taylor instability, D3Q27 cumulant flow + D3Q27
conservative Allen-Cahn populations, 128 x 128 x 512 lattice, periodic in x/y,
no-slip walls in z, Atwood 0.5, Re 1000, W 5, mobility 0.1, interface at
z = 256 with a two-mode cosine perturbation of amplitude 0.05 * 128, FP32
storage and arithmetic.  A "step" advances both population sets of every
cell by one time step: the order parameter of the current level (merged from
the partial sums the previous update wrote, or a pass over the pulled
populations) plus the update of every cell (both collisions, streaming).

Prints one JSON line: MLUPS (million lattice-cell updates per second) with a
roofline entry for the dominant kernel (the cell update, HBM-bound), the
error of the FP32 state against the FP64 CPU oracle on a slab of the same
workload, and the oracle's own rate on that slab.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# what a kernel that only loads and stores the update's 54 population planes
# moves on this part (measured, GB/s): the practical ceiling of the step
STREAM_CEILING_GBS = 5500.0
# algorithmic bytes per cell for one launch of each kernel, FP32, D3Q27:
#   collide: read 27 f' + 27 g + phi, write 27 f' + 27 g  -> 4 * (27 * 4 + 1) = 436
#   phi:     read 27 g, write phi                          -> 4 * (27 + 1)     = 112
ALG_BYTES = {("fp32", 3): {"collide": 436, "phi": 112, "method": 440},
             ("fp64", 3): {"collide": 872, "phi": 224, "method": 880},
             # FP16 flow set: 26 FP16 codes each way plus the FP32 rest value;
             # the order parameter travels as an 8-byte record (phi and the
             # cell's packed FP16 references), the references as 4 bytes
             # written by the update and read by the phi stage
             ("fp16s", 3): {"collide": 2 * (26 * 2 + 4) + 2 * 27 * 4 + 8 + 4,
                            "phi": 27 * 4 + 4 + 8,
                            "method": 2 * (26 * 2 + 4) + 2 * 27 * 4 + 8 + 8},
             # both sets in FP16 (rest values in FP32)
             ("fp16s_all", 3): {"collide": 4 * (26 * 2 + 4) + 8 + 4,
                                "phi": 26 * 2 + 4 + 4 + 8,
                                "method": 4 * (26 * 2 + 4) + 8 + 8},
             ("fp32", 2): {"collide": 4 * (2 * 2 * 9 + 1), "phi": 4 * (9 + 1), "method": 152},
             ("fp64", 2): {"collide": 8 * (2 * 2 * 9 + 1), "phi": 8 * (9 + 1), "method": 304}}


def nphi_bytes(storage, rows):
    """Algorithmic bytes per cell of the update that also sums the next phi
    (k_collide_nphi: the collide bytes plus its partial sums, three per cell
    and three more for each of the two edge rows of a tile of `rows` rows)
    and of the merge that adds them (k_phi_merge: the partial sums read,
    phi written)."""
    s = 8 if storage == "fp64" else 4
    part = s * (3 + 6.0 / rows)
    # the merge writes phi (FP16 formats: the 8-byte record, with the
    # reference it reads)
    out = s if storage in ("fp32", "fp64") else 8 + 4
    return ALG_BYTES[(storage, 3)]["collide"] + part, part + out


KERNEL_SOURCES = ("device.hpp", "k_step.hip", "k_nphi.hip", "k_host.hip", "k_batch.hip",
                  "lattice.hpp", "internal.h")
PROFILE_KERNELS = {"k_collide_nphi": "k_phi_merge", "k_collide": "k_phi"}
PROFILES_DIR = os.path.join(ROOT, "profiles")


def profiled_traffic(storage, workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of this workload and storage (each counter scaled by its
    reading for a plain copy of known size).  None unless such a summary exists
    and was taken on kernel sources identical to the ones in the tree."""
    import hashlib

    if kernel not in PROFILE_KERNELS:
        return None
    path = os.path.join(PROFILES_DIR, "%s_%s_%s_%s_hbm_bytes.md" %
                        (kernel, PROFILE_KERNELS[kernel], workload, storage))
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2101_06769_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    text = open(path).read()
    blob = text.split("```json", 1)[1].split("```", 1)[0]
    rec = json.loads(blob)
    if rec["sources_sha256"] != h.hexdigest() or rec["kernel"] != kernel:
        return None
    return rec["traffic_bytes_per_launch"]


def device_info():
    """The GPU the line was measured on (boxes of the same part differ by a few
    percent in streaming rate, so the line names its device)."""
    import torch

    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": p.gcnArchName, "compute_units": p.multi_processor_count,
            "hbm_GiB": round(p.total_memory / 2 ** 30, 1), "pci_bus_id": p.pci_bus_id}


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess

    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                return ln.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(case_fn, min_seconds=10.0):
    """The FP64 oracle on a 128 x 128 x 128 slab of the same workload (the
    interface region), stepped on every host thread until at least
    min_seconds have elapsed, then on one thread for one step of a
    128 x 128 x 16 slab.  Returns the baseline record and the oracle's final
    state (params, f, g, steps) for the error figure."""
    import oracle

    case = case_fn(128)
    p = oracle.params_from_dict(case.params)
    f, g = oracle.init(p, case.phi, case.u, case.p)
    steps, t0 = 0, time.perf_counter()
    while True:
        f, g = oracle.step(p, f, g, 1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds:
            break
    threads = oracle.num_threads()
    small = case_fn(16)
    ps = oracle.params_from_dict(small.params)
    fs, gs = oracle.init(ps, small.phi, small.u, small.p)
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.step(ps, fs, gs, 1)
        el1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    rec = {"value": case.ncells * steps / el / 1e6, "unit": "MLUPS",
           "cores": threads, "kind": "oracle",
           "sample": "%d step(s) of a 128x128x128 slab (%d cells) of the same Rayleigh-Taylor "
                     "case, FP64, %.1f s on %d threads" % (steps, case.ncells, el, threads),
           "cpu_model": cpu_model(),
           "value_1thread": small.ncells / el1 / 1e6,
           "sample_1thread": "1 step of a 128x128x16 slab (%d cells), FP64, %.1f s on 1 thread" %
                             (small.ncells, el1)}
    return rec, (p, f, g, steps)


def c1_timing():
    """The C1 case, the 2-D Rayleigh-Taylor run of Sec. 3.2's shape (64 x 256,
    At 0.5, Re 256, W 4, M 0.1, 2000 steps), in full: the FP64 oracle on the
    host's threads and the GPU in FP64 from the same initial state, with the
    per-field difference of their final states (U* = 0.06)."""
    import torch

    import oracle
    from paper_2101_06769_amd import inputs, mplb

    case = inputs.rti2d()
    po = oracle.params_from_dict(case.params)
    f, g = oracle.init(po, case.phi, case.u, case.p)
    t0 = time.perf_counter()
    f, g = oracle.step(po, f, g, case.steps)
    t_cpu = time.perf_counter() - t0
    want = oracle.fields(po, f, g)
    s = mplb.Solver(case.params, storage="fp64")
    s.init(case.phi, case.u, case.p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(case.steps)
    s.sync()
    t_gpu = time.perf_counter() - t0
    got = s.fields()
    U = inputs.U_STAR
    work = case.ncells * case.steps
    return {"workload": "2-D Rayleigh-Taylor 64x256, At 0.5, Re 256, 2000 steps, FP64",
            "oracle_s": round(t_cpu, 2), "oracle_mlups": round(work / t_cpu / 1e6, 2),
            "oracle_threads": oracle.num_threads(),
            "gpu_fp64_s": round(t_gpu, 4), "gpu_fp64_mlups": round(work / t_gpu / 1e6, 1),
            "max_abs_dphi": float(np.abs(got["phi"] - want["phi"]).max()),
            "max_abs_du_over_U": float(np.abs(got["u"] - want["u"]).max() / U),
            "max_abs_dp_over_rhoU2": float(np.abs(got["p"] - want["p"]).max() / (U * U))}


def error_vs_oracle(case, storage, ref):
    """Per-field error of the GPU state against the FP64 oracle after the same
    steps from the same initial state: max |dphi|, max |du| / U*, max |dp| /
    (rho_h U*^2) with U* = sqrt(g L_x) = 0.06, the Rayleigh-Taylor velocity
    scale.  Beside it the method's own sensitivity (the oracle against itself
    when every population carries one rounding of the storage format after
    every step); the tolerance is a multiple of that floor, as in the
    multi-step parity tests."""
    import oracle
    from paper_2101_06769_amd import inputs, mplb

    p, f, g, steps = ref
    want = oracle.fields(p, f, g)
    s = mplb.Solver(case.params, storage=storage)
    s.init(case.phi, case.u, case.p)
    s.step(steps)
    got = s.fields()
    del s
    U = inputs.U_STAR

    def fielderr(a, b):
        return {"phi": float(np.abs(a["phi"] - b["phi"]).max()),
                "u_over_U": float(np.abs(a["u"] - b["u"]).max() / U),
                "p_over_rhoU2": float(np.abs(a["p"] - b["p"]).max() / (U * U))}

    err = fielderr(got, want)
    # the floor: the same run with one rounding per step (relative amp)
    amp = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24}.get(storage, 2.0 ** -11)
    rng = np.random.default_rng(0)
    fb, gb = oracle.init(p, case.phi, case.u, case.p)
    for _ in range(steps):
        fb, gb = oracle.step(p, fb, gb, 1)
        fb = fb * (1 + amp * rng.uniform(-1, 1, fb.shape))
        gb = gb * (1 + amp * rng.uniform(-1, 1, gb.shape))
    floor = fielderr(oracle.fields(p, fb, gb), want)
    # plus the rounding of the field's own evaluation in the storage's
    # arithmetic (the floor run evaluates in FP64): a few tens of ulps of
    # the field's magnitude, summed over the populations
    eps = 2.0 ** -52 if storage == "fp64" else 2.0 ** -23
    scale = {"phi": float(np.abs(want["phi"]).max()),
             "u_over_U": float(np.abs(want["u"]).max()) / U,
             "p_over_rhoU2": float(np.abs(want["p"]).max()) / (U * U)}
    tol = {k: ERROR_FLOOR_MULTIPLE * floor[k] + EVAL_ULPS * eps * scale[k] for k in floor}
    return {"steps": steps, "cells": case.ncells, "max_abs": err, "floor": floor,
            "tolerance": tol, "within_tolerance": all(err[k] <= tol[k] for k in err)}


# The multi-step bar of the parity tests: the GPU state within this multiple
# of the oracle's own sensitivity to one rounding of the storage format per step.
ERROR_FLOOR_MULTIPLE = 5.0
# ulps of a field's magnitude allowed for evaluating it from the populations
EVAL_ULPS = 64


def batch_cpu_baseline(cases, steps):
    """The batch workload's CPU leg: the FP64 oracle timed on the given
    domains (the two smallest of the batch) for `steps` steps on the host's
    threads, and the per-field errors of the same domains stepped in a batch
    (the shared launches) against it (U* = 0.06, the Rayleigh-Taylor velocity
    scale of every batch domain)."""
    import oracle
    from paper_2101_06769_amd import inputs, mplb

    b = mplb.Batch(3, "fp32", capacity=len(cases), max_tiles=1 << 16)
    solvers = []
    for c in cases:
        sv = mplb.Solver(c.params, storage="fp32", stream=b.stream)
        sv.init(c.phi, c.u, c.p)
        b.attach(sv, steps)
        solvers.append(sv)
    b.step(steps)
    errs, t_cpu, work = [], 0.0, 0
    U = inputs.U_STAR
    for c, sv in zip(cases, solvers):
        po = oracle.params_from_dict(c.params)
        f, g = oracle.init(po, c.phi, c.u, c.p)
        t0 = time.perf_counter()
        f, g = oracle.step(po, f, g, steps)
        t_cpu += time.perf_counter() - t0
        work += c.ncells * steps
        want, got = oracle.fields(po, f, g), sv.fields()
        errs.append({"n": list(c.params["n"]), "steps": steps,
                     "max_abs_dphi": float(np.abs(got["phi"] - want["phi"]).max()),
                     "max_abs_du_over_U": float(np.abs(got["u"] - want["u"]).max() / U),
                     "max_abs_dp_over_rhoU2": float(np.abs(got["p"] - want["p"]).max() / (U * U))})
    return {"value": work / t_cpu / 1e6, "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d steps of the %d smallest domains (%s), FP64, %.1f s" %
                      (steps, len(cases), ", ".join("x".join(map(str, c.params["n"])) for c in cases),
                       t_cpu),
            "cpu_model": cpu_model(), "batched_vs_oracle": errs}


def bench_batch(args):
    """64 independent 3-D Rayleigh-Taylor domains of uneven size (seed 0:
    edge in {32, 48, 64, 96, 128}, z = 4 edge, Atwood in [0.1, 0.9], Re in
    [100, 3000], random-phase multimode interface), FP32, `steps` steps each.
    Plain: one domain at a time, each with its own launches, on one stream.
    Batched: all domains in the same launches, block shape from the
    autotuner, chunks of steps replayed as a HIP graph.  States are resident
    before either timed region starts; both start from the same initial state."""
    import torch

    from paper_2101_06769_amd import inputs, mplb

    steps = args.batch_steps
    cases = inputs.batch_rti3d(count=args.domains, seed=0, steps=steps)
    cells = sum(c.ncells for c in cases)
    b = mplb.Batch(3, "fp32", capacity=len(cases), max_tiles=1 << 22)
    b.set_graph_chunk(16)
    solvers = [mplb.Solver(c.params, storage="fp32", stream=b.stream) for c in cases]

    def reset():
        for c, sv in zip(cases, solvers):
            sv.init(c.phi, c.u, c.p)

    # autotune the batch block on the workload itself, then start over
    reset()
    slots = [b.attach(sv, 10 ** 9) for sv in solvers]
    best, _ = b.tune_block(steps=3)
    for sl in slots:
        b.detach(sl)
    # plain: one domain per launch pair, sequentially
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sv in solvers:
        sv.step(steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    plain_phi = [sv.read(0) for sv in solvers]
    def batched(solo_cells):
        # one untimed chunk captures the step graph, then start over
        b.set_solo_cells(solo_cells)
        reset()
        slots = [b.attach(sv, steps) for sv in solvers]
        b.step(16)
        for sl in slots:
            b.detach(sl)
        reset()
        slots = [b.attach(sv, steps) for sv in solvers]
        nsolo = sum(b.is_solo(sl) for sl in slots)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        same = all(np.array_equal(a, sv.read(0)) for a, sv in zip(plain_phi, solvers))
        for sl in slots:
            b.detach(sl)
        return el, same, nsolo

    # every domain in the shared launches, then the default split (domains
    # of 2^20 cells and more with their own kernels beside them)
    t_shared, same_shared, _ = batched(1 << 62)
    t_batch, same, nsolo = batched(args.solo_cells)
    line = {
        "metric": "batched jobs/s (64 uneven 3-D Rayleigh-Taylor domains)",
        "value": round(len(cases) / t_batch, 3),
        "unit": "jobs/s",
        "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": round(t_batch / steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "64 independent 3-D Rayleigh-Taylor domains, edge in "
                               "{32,48,64,96,128}, z = 4 edge, At U[0.1,0.9], Re U[100,3000], "
                               "FP32, %d steps each" % steps,
                   "cells": cells, "parallelism": "single GPU"},
        "batched": {"jobs_per_s": round(len(cases) / t_batch, 3), "makespan_s": round(t_batch, 3),
                    "mlups": round(cells * steps / t_batch / 1e6, 1), "block": list(best),
                    "domains_with_own_kernels": nsolo, "solo_min_cells": args.solo_cells},
        "all_shared": {"jobs_per_s": round(len(cases) / t_shared, 3),
                       "makespan_s": round(t_shared, 3),
                       "mlups": round(cells * steps / t_shared / 1e6, 1),
                       "equals_plain_bitwise": bool(same_shared)},
        "plain": {"jobs_per_s": round(len(cases) / t_plain, 3), "makespan_s": round(t_plain, 3),
                  "mlups": round(cells * steps / t_plain / 1e6, 1)},
        "speedup_vs_plain": round(t_plain / t_batch, 3),
        "batched_equals_plain_bitwise": bool(same),
    }
    if not args.no_cpu_baseline:
        smallest = sorted(cases, key=lambda c: c.ncells)[:2]
        line["cpu_baseline"] = batch_cpu_baseline(smallest, args.oracle_steps)
    print(json.dumps(line), flush=True)


def bench_batch_groups(args):
    """The batch workload's 64 domains one domain per launch, timed group by
    group of equal edge, against the time each group would take streaming its
    algorithmic bytes at STREAM_CEILING_GBS (548 B/cell per step with the phi
    pass, 476 with the phi-summing update, FP32): where plain loses time, a
    batched form can win it back; elsewhere no form can.  Then the domains of
    edge 48 and less alone in the batch's shared launches."""
    import torch

    from paper_2101_06769_amd import inputs, mplb

    steps = args.batch_steps
    cases = inputs.batch_rti3d(count=args.domains, seed=0, steps=steps)
    b = mplb.Batch(3, "fp32", capacity=len(cases), max_tiles=1 << 22)
    b.set_graph_chunk(16)
    solvers = [mplb.Solver(c.params, storage="fp32", stream=b.stream) for c in cases]
    edges = [c.params["n"][0] for c in cases]
    groups, total, bound = [], 0.0, 0.0
    for e in sorted(set(edges)):
        idx = [i for i, ee in enumerate(edges) if ee == e]
        for i in idx:
            solvers[i].init(cases[i].phi, cases[i].u, cases[i].p)
        form = solvers[idx[0]].phi_partial_rows() > 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in idx:
            solvers[i].step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        cells = sum(cases[i].ncells for i in idx)
        bpc = 476 if form else 548
        at_ceiling = cells * bpc * steps / (STREAM_CEILING_GBS * 1e9)
        groups.append({"edge": e, "domains": len(idx), "cells": cells, "plain_s": round(el, 3),
                       "mlups": round(cells * steps / el / 1e6, 1),
                       "step_form": "phi-summing update" if form else "phi pass",
                       "bytes_per_cell": bpc, "s_at_ceiling": round(at_ceiling, 3)})
        total += el
        bound += min(at_ceiling, el)
    small = [i for i, e in enumerate(edges) if e <= 48]
    b.set_solo_cells(1 << 62)

    def attach_small():
        for i in small:
            solvers[i].init(cases[i].phi, cases[i].u, cases[i].p)
        return [b.attach(solvers[i], steps) for i in small]

    slots = attach_small()
    b.step(16)  # captures the chunk graph
    for sl in slots:
        b.detach(sl)
    slots = attach_small()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    t_small = time.perf_counter() - t0
    for sl in slots:
        b.detach(sl)
    print(json.dumps({
        "workload": "batch mix one domain per launch, by edge, %d steps" % steps,
        "groups": groups, "plain_total_s": round(total, 3),
        "best_any_form_s": round(bound, 3),
        "max_speedup_vs_plain": round(total / bound, 3),
        "stream_ceiling_GBs": STREAM_CEILING_GBS,
        "edge_le_48_shared_launches_s": round(t_small, 3),
        "edge_le_48_plain_s": round(sum(g["plain_s"] for g in groups if g["edge"] <= 48), 3)}),
        flush=True)


def splash_vs_oracle(storage):
    """Per-field max errors against the FP64 oracle of the same droplet impact
    on a reduced lattice (128 x 128 x 64, D = 16, 500 steps; the oracle's
    fields stored in tests/golden/splash3d_reduced.npz on whole planes through
    the sheet and the drop plus seeded random cells), with the oracle's own
    sensitivity to one FP32 rounding per step beside them."""
    from paper_2101_06769_amd import inputs, mplb

    with np.load(os.path.join(ROOT, "tests", "golden", "splash3d_reduced.npz"),
                 allow_pickle=False) as z:
        ref = {k: z[k] for k in ("cells", "phi", "u", "p")}
        meta = json.loads(str(z["meta"]))
    case = inputs.splash3d(nx=128, ny=128, nz=64, D=16.0, U0=0.05, Re=1000.0, We=8000.0)
    s = mplb.Solver(case.params, storage=storage)
    s.init(case.phi, case.u, case.p)
    s.step(meta["steps"])
    got = s.fields()
    cells = ref["cells"].astype(np.int64)
    U, rho_h = meta["U"], meta["rho_h"]
    return {"steps": meta["steps"], "cells_compared": int(cells.size),
            "phi": float(np.abs(got["phi"].ravel()[cells] - ref["phi"]).max()),
            "u_over_U0": float(np.abs(got["u"].reshape(3, -1)[:, cells] - ref["u"]).max() / U),
            "p_over_rhoU0sq": float(np.abs(got["p"].ravel()[cells] - ref["p"]).max() / (rho_h * U * U)),
            "oracle_fp32_rounding_floor": meta["floor_fp32_rounding"]}


def bench_splash(args):
    """3-D droplet impact on a thin liquid sheet, 512 x 512 x 256 (density
    ratio 1000, viscosity ratio 15, We 8000, Re 1000, D = 64, sheet 0.1 D,
    U0 0.05): the same `splash_steps` steps in FP64, FP32 and FP16-shifted
    storage.  Reports each format's MLUPS, its field errors against the FP64
    run, and its field errors against the FP64 oracle on a reduced lattice of
    the same case (splash_vs_oracle)."""
    import torch

    from paper_2101_06769_amd import inputs, mplb

    case = inputs.splash3d()
    U0 = case.meta["U0"]
    N = case.ncells
    out = {}
    ref = None
    rng = np.random.default_rng(7)
    # "fp64_floor": FP64 again, from inputs carrying one FP32 rounding
    # (relative 2^-24): the method's own sensitivity, the error any FP32
    # state would show against FP64 without any arithmetic difference
    for storage in ("fp64", "fp64_floor", "fp32", "fp16s", "fp16s_all"):
        s = mplb.Solver(case.params, storage=storage.split("_floor")[0])
        if storage == "fp64_floor":
            def pert(a):
                return a * (1.0 + 2.0 ** -24 * rng.uniform(-1.0, 1.0, a.shape))
            s.init(np.clip(pert(case.phi), 0.0, 1.0), pert(case.u), pert(case.p))
        else:
            s.init(case.phi, case.u, case.p)
        s.step(5)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.step(args.splash_steps)
        e1.record(s.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        f = s.fields()
        red, rc = s.reduce()
        rec = {"mlups": round(N * args.splash_steps / (ms / 1e3) / 1e6, 1),
               "ms_per_step": round(ms / args.splash_steps, 4),
               "alg_GBs": round(ALG_BYTES[(storage.split("_floor")[0], 3)]["method"] * N *
                                args.splash_steps / (ms / 1e3) / 1e9, 1),
               "status": "ok" if rc == mplb.OK else "unstable",
               "phase_mass_rel_drift": abs(red[0] - case.phi.sum()) / case.phi.sum()}
        if ref is None:
            ref = f
        else:
            rec["max_abs_dphi"] = float(np.abs(f["phi"] - ref["phi"]).max())
            rec["max_abs_du_over_U0"] = float(np.abs(f["u"] - ref["u"]).max() / U0)
            rec["max_abs_dp_over_rhoU0sq"] = float(np.abs(f["p"] - ref["p"]).max() / (U0 * U0))
        if storage != "fp64_floor":
            rec["vs_fp64_oracle_reduced"] = splash_vs_oracle(storage)
        out[storage] = rec
        print("splash: %s, %d steps in %.1f s" % (storage, args.splash_steps, ms / 1e3),
              file=sys.stderr, flush=True)
        del s, f
        torch.cuda.empty_cache()
    line = {
        "metric": "MLUPS (flow+phase field) at fixed error vs FP64: droplet splash, FP32 vs FP16",
        "value": out["fp16s"]["mlups"], "unit": "MLUPS", "n_gpus": 1,
        "steps": args.splash_steps, "warmup": 5,
        "ms_per_step": out["fp16s"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f16s+f32", "data": "synthetic",
        "config": {"workload": "3-D droplet impact on a thin liquid sheet, 512x512x256, density "
                               "ratio 1000, viscosity ratio 15, We 8000, Re 1000, D 64, U0 0.05",
                   "cells": N, "parallelism": "single GPU"},
        "by_storage": out,
    }
    print(json.dumps(line), flush=True)


def bench_rti2d_convergence(args):
    """Resolution study of the 2-D Rayleigh-Taylor case (Sec. 3.2): At 0.5,
    Re 256 and 2048, box L x 4L with L = 150, 300, 600 under acoustic scaling
    (U* = sqrt(g L) = 0.06, so g = 0.0036 / L and nu = 0.06 L / Re), interface
    2L + (L/10) cos(2 pi x / L), FP32.  Spike and bubble positions (in units
    of L from the bottom wall) at t/T = 0.5 .. 5, T = L / U*.  The six
    domains advance together in one batch; each is detached at its own sample
    times, read, and attached again for its next interval."""
    import torch

    from paper_2101_06769_amd import diagnostics, inputs, mplb

    runs = []
    b = mplb.Batch(2, "fp32", capacity=8, max_tiles=1 << 16)
    b.set_graph_chunk(16)
    for Re in (256.0, 2048.0):
        for L in (150, 300, 600):
            case = inputs.rti2d(nx=L, ny=4 * L, At=0.5, Re=Re, W=4.0, M=0.1, amp=0.1 * L)
            s = mplb.Solver(case.params, storage="fp32", stream=b.stream)
            s.init(case.phi, case.u, case.p)
            T = case.meta["T"]
            runs.append({"key": "Re%d_L%d" % (Re, L), "L": L, "s": s, "done": 0, "k": 1,
                         "targets": [int(round(0.5 * k * T)) for k in range(1, 11)],
                         "rows": [], "status": "ok", "slot": None})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in runs:
        r["slot"] = b.attach(r["s"], r["targets"][0])
    batched_steps = 0
    while any(r["slot"] is not None for r in runs):
        live = [r for r in runs if r["slot"] is not None]
        n = min(b.remaining(r["slot"]) for r in live)
        b.step(n)
        batched_steps += n
        bad = {sl for sl, st in b.status().items() if st == mplb.EUNSTABLE}
        for r in live:
            if r["slot"] in bad:
                r["status"] = "unstable"
            elif b.remaining(r["slot"]) > 0:
                continue
            b.detach(r["slot"])
            r["slot"] = None
            if r["status"] != "ok":
                continue
            L = r["L"]
            r["done"] = r["targets"][r["k"] - 1]
            spike, bubble = diagnostics.rti_positions(r["s"].read(0), 2)
            r["rows"].append([0.5 * r["k"], None if spike is None else round(spike / L, 4),
                              None if bubble is None else round(bubble / L, 4)])
            if r["k"] < len(r["targets"]):
                r["k"] += 1
                r["slot"] = b.attach(r["s"], r["targets"][r["k"] - 1] - r["done"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {}
    for r in runs:
        _, rc = r["s"].reduce()
        out[r["key"]] = {"t_over_T,spike/L,bubble/L": r["rows"],
                         "status": "ok" if rc == mplb.OK and r["status"] == "ok" else "unstable"}
    for Re in (256, 2048):
        a = out["Re%d_L300" % Re]["t_over_T,spike/L,bubble/L"]
        c = out["Re%d_L600" % Re]["t_over_T,spike/L,bubble/L"]
        out["Re%d_max_spike_change_300_to_600" % Re] = max(
            abs(x[1] - y[1]) for x, y in zip(a, c) if x[1] is not None and y[1] is not None)
    cells_steps = sum(r["s"].N * r["done"] for r in runs)
    print(json.dumps({"workload": "2-D Rayleigh-Taylor resolution study, At 0.5, Re 256/2048, "
                                  "L = 150/300/600, to t/T = 5, six domains in one batch",
                      "wall_s": round(wall, 2), "batch_steps": batched_steps,
                      "MLUPS": round(cells_steps / wall / 1e6, 1), "results": out}), flush=True)


def bench_stability(args):
    """Stability of the cumulant collision against single relaxation time
    (Sec. 2.3, 4): 2-D Rayleigh-Taylor, 128 x 512, density ratios 3, 19 and
    1000, Re 256 .. 65536 (relaxation rate omega up to 1.9999), FP32, 4000
    steps; the step by which the state first holds a non-finite value."""
    from paper_2101_06769_amd import inputs, mplb

    table = []
    for At in (0.5, 0.9, 0.998):
        for Re in (256.0, 2048.0, 16384.0, 65536.0):
            case = inputs.rti2d(nx=128, ny=512, At=At, Re=Re, W=4.0, M=0.1, amp=12.8)
            nu = case.params["nu_h"]
            row = {"At": At, "rho_ratio": round((1 + At) / (1 - At), 1), "Re": Re,
                   "omega": round(1.0 / (3.0 * nu + 0.5), 6)}
            for name, coll in (("cumulant", 0), ("srt", 1)):
                s = mplb.Solver(case.params, storage="fp32", collision=coll)
                s.init(case.phi, case.u, case.p)
                blown = None
                for k in range(20):
                    s.step(200)
                    red, rc = s.reduce()
                    if rc != mplb.OK or red[4] > 0.5:
                        blown = (k + 1) * 200
                        break
                row[name] = "stable" if blown is None else "diverged by step %d" % blown
            table.append(row)
            print(json.dumps(row), flush=True)
    print(json.dumps({"workload": "collision stability map, 2-D Rayleigh-Taylor 128x512, 4000 steps",
                      "rows": table}), flush=True)


def bench_splash2d(args):
    """2-D droplet impact on a liquid film (Sec. 3.4): D = 100, symmetry
    planes left and right, density ratio 1000, viscosity ratio 15; the
    paper's three cases (Re, We) = (200, 220), (1000, 220), (1000, 2200);
    spreading radius r_K / D at t / T = 0.1 .. 1.5 beside 1.1 sqrt(t / T)."""
    from paper_2101_06769_amd import diagnostics, inputs, mplb

    out = {}
    for Re, We in ((200.0, 220.0), (1000.0, 220.0), (1000.0, 2200.0)):
        case = inputs.splash2d(D=100.0, Re=Re, We=We)
        D, T = case.meta["D"], case.meta["T"]
        s = mplb.Solver(case.params, storage="fp32")
        s.init(case.phi, case.u, case.p)
        rows, done = [], 0
        for k in range(1, 16):
            target = int(round(0.1 * k * T))
            s.step(target - done)
            done = target
            r = diagnostics.spreading_radius(s.read(0), case.meta["x_axis"],
                                             case.meta["sheet"] + 0.5 * case.params["W"])
            rows.append([round(0.1 * k, 2), round(r / D, 4), round(1.1 * (0.1 * k) ** 0.5, 4)])
        red, rc = s.reduce()
        out["Re%d_We%d" % (Re, We)] = {"K": round(case.meta["K"], 1),
                                        "t_over_T,rK/D,1.1sqrt(t/T)": rows,
                                        "status": "ok" if rc == mplb.OK else "unstable"}
    print(json.dumps({"workload": "2-D droplet impact on a film, D 100, 800x400, symmetry sides, W 5",
                      "results": out}), flush=True)


def bench_edf(args):
    """The two phase-field equilibria of Sec. 2.2 (second-order, the paper's;
    first-order with the correction term): spike positions of the 2-D
    Rayleigh-Taylor case (At 0.5, L = 300, Re 256 and 2048) to t/T = 5 under
    each, and the step rate of each on the 128 x 128 x 512 3-D case (FP32)."""
    import torch

    from paper_2101_06769_amd import diagnostics, inputs, mplb

    out = {}
    for Re in (256.0, 2048.0):
        rows = {}
        for edf in (0, 1):
            case = inputs.rti2d(nx=300, ny=1200, At=0.5, Re=Re, W=4.0, M=0.1, amp=30.0)
            case.params["cac_edf"] = edf
            T = case.meta["T"]
            s = mplb.Solver(case.params, storage="fp32")
            s.init(case.phi, case.u, case.p)
            done, r = 0, []
            for k in range(1, 11):
                target = int(round(0.5 * k * T))
                s.step(target - done)
                done = target
                spike, _ = diagnostics.rti_positions(s.read(0), 2)
                r.append(None if spike is None else spike / 300.0)
            rows[edf] = r
        out["Re%d" % Re] = {"t_over_T": [0.5 * k for k in range(1, 11)],
                            "spike_over_L_second_order": [round(v, 4) for v in rows[0]],
                            "spike_over_L_first_order": [round(v, 4) for v in rows[1]],
                            "max_difference": round(max(abs(a - b) for a, b in
                                                        zip(rows[0], rows[1])), 4)}
    case = inputs.rti3d()
    rates = {}
    for edf in (0, 1):
        case.params["cac_edf"] = edf
        s = mplb.Solver(case.params, storage="fp32")
        s.init(case.phi, case.u, case.p)
        s.step(20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(300)
        torch.cuda.synchronize()
        rates["second_order" if edf == 0 else "first_order"] = round(
            case.ncells * 300 / (time.perf_counter() - t0) / 1e6, 1)
        del s
    print(json.dumps({"workload": "phase-field equilibrium orders: 2-D RTI spike positions, "
                                  "3-D RTI 128x128x512 MLUPS", "rti2d": out, "mlups_3d": rates}),
          flush=True)


def bench_serve(args):
    """Serving: seeded Poisson arrivals (20/s) of 2-D solves (Rayleigh-Taylor,
    static drop, impacting drop; edge log-uniform 64..1024, density ratio
    3..1000, steps 500..20000), FP32, replayed in real time through the
    continuous-batching server and through the one-at-a-time baseline."""
    import torch

    from paper_2101_06769_amd import inputs, mplb, serve

    specs = inputs.serving_spec(seed=1, count=args.requests, rate=args.rate)
    # warm-up: kernel loading and graph instantiation outside the replay
    warm = inputs.serving_spec(seed=99, count=2, rate=1000.0, edge_range=(64, 64),
                               steps_range=(40, 40))
    serve.serve_batched(warm, realtime=False)
    serve.serve_fifo(warm, realtime=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res_b, st = serve.serve_batched(specs, hbm_budget=int(args.hbm_budget_gb * (1 << 30)),
                                    capacity=args.capacity)
    wall_b = time.perf_counter() - t0
    print("serve: batched replay done in %.1f s" % wall_b, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    res_f = serve.serve_fifo(specs)
    wall_f = time.perf_counter() - t0
    sb, sf = serve.summary(res_b, wall_b), serve.summary(res_f, wall_f)
    line = {
        "metric": "serving p99 latency (continuous batching)",
        "value": None if sb["p99_s"] is None else round(sb["p99_s"], 4),
        "unit": "s", "n_gpus": 1, "steps": None, "warmup": 2,
        "ms_per_step": None,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%d Poisson arrivals at %.0f/s of 2-D solves (Rayleigh-Taylor, "
                               "static drop, impacting drop), edge 64..1024, density ratio "
                               "3..1000, 500..20000 steps, FP32" % (args.requests, args.rate),
                   "hbm_budget_gb": args.hbm_budget_gb, "parallelism": "single GPU"},
        "batched": dict(sb, wall_s=round(wall_b, 2), peak_active=st["peak_active"],
                        peak_gb=round(st["peak_bytes"] / 2 ** 30, 2)),
        "fifo": dict(sf, wall_s=round(wall_f, 2)),
        "unstable_requests": sum(r.status == mplb.EUNSTABLE for r in res_b),
        "unstable": [{k: (round(v, 6) if isinstance(v, float) else v)
                      for k, v in specs[r.id].items() if k != "arrival"}
                     for r in sorted(res_b, key=lambda r: r.id) if r.status == mplb.EUNSTABLE],
        "unstable_fifo_ids": sorted(r.id for r in res_f if r.status == mplb.EUNSTABLE),
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp64", "fp16s", "fp16s_all"])
    ap.add_argument("--nz", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--phi-partials", type=int, default=1, choices=[0, 1],
                    help="1: the update sums the next phi from the values it stores and the "
                         "next step merges the partial sums (default, where it applies); 0: a "
                         "phi pass over the pulled populations every step")
    ap.add_argument("--collision", default="cumulant", choices=["cumulant", "srt"],
                    help="rti3d / rti2d: the flow collision (srt: single relaxation time, the "
                         "ablation of Sec. 4)")
    ap.add_argument("--cac-edf", type=int, default=0, choices=[0, 1],
                    help="rti3d / rti2d: 1 takes the first-order phase-field equilibrium with "
                         "its correction term (Sec. 2.2), which keeps the previous (phi u) per cell")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--workload", default="rti3d",
                    choices=["rti3d", "rti2d", "batch", "batch_groups", "serve", "splash",
                             "rti2d_convergence", "stability", "splash2d", "edf"],
                    help="rti3d: the 128x128x512 step (default); rti2d: one 2-D Rayleigh-Taylor "
                         "domain of --n2d squared cells (the largest served size); batch: 64 "
                         "uneven domains, "
                         "batched vs one per launch; batch_groups: the same mix one domain per "
                         "launch, timed edge by edge; serve: request replay; splash: "
                         "512x512x256 droplet impact in FP64 / FP32 / FP16")
    ap.add_argument("--n2d", type=int, default=1024, help="rti2d: cells per side")
    ap.add_argument("--splash-steps", type=int, default=200)
    ap.add_argument("--domains", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--oracle-steps", type=int, default=100,
                    help="batch: steps of the two smallest domains checked against the oracle")
    ap.add_argument("--solo-cells", type=int, default=1 << 20,
                    help="batch: domains of at least this many cells step with their own "
                         "kernels beside the shared launches")
    ap.add_argument("--requests", type=int, default=1000)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--hbm-budget-gb", type=float, default=64.0)
    ap.add_argument("--capacity", type=int, default=256, help="serving: batch slots")
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
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "batch_groups":
        return bench_batch_groups(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "splash":
        return bench_splash(args)
    if args.workload == "rti2d_convergence":
        return bench_rti2d_convergence(args)
    if args.workload == "stability":
        return bench_stability(args)
    if args.workload == "splash2d":
        return bench_splash2d(args)
    if args.workload == "edf":
        return bench_edf(args)
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
    if args.workload == "rti2d":
        if args.storage not in ("fp32", "fp64"):
            sys.exit("rti2d: FP32 or FP64 storage")
        n2 = args.n2d
        case = inputs.rti2d(nx=n2, ny=n2, amp=0.05 * n2)
        label = ("2-D Rayleigh-Taylor, D2Q9 cumulant + D2Q9 Allen-Cahn, %dx%d, At 0.5, Re 256, W 4, "
                 "%s storage" % (n2, n2, args.storage))
        wtag = "rti2d_%dx%d" % (n2, n2)
    else:
        case = inputs.rti3d(nz=args.nz)
        label = ("3-D Rayleigh-Taylor, D3Q27 cumulant + D3Q27 Allen-Cahn, 128x128x%d, At 0.5, "
                 "Re 1000, W 5, %s storage" % (args.nz, args.storage))
        wtag = "rti3d_128x128x%d" % args.nz
    variant = ""
    if args.collision == "srt":
        case.params["collision"] = mplb.COLL_SRT
        label += ", SRT collision"
        variant += "_srt"
    if args.cac_edf:
        case.params["cac_edf"] = 1
        label += ", first-order phase-field equilibrium"
        variant += "_edf"
    dim = case.params["dim"]
    N = case.ncells
    s = mplb.Solver(case.params, storage=args.storage)
    s.set_phi_partials(args.phi_partials)
    s.init(case.phi, case.u, case.p)
    s.step(args.warmup)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s.stream)
    s.step(args.steps)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    # per-kernel launch durations for the roofline, from HIP events around
    # each launch on the solver's stream, over as many further steps (kept out
    # of the timed region above: the events between launches add gaps)
    ms_phi, ms_col = s.step_timed(args.steps)
    ms_step = ms / args.steps
    mlups = N * args.steps / (ms / 1e3) / 1e6

    red, rc = s.reduce()
    m0 = float(case.phi.sum())
    ab = ALG_BYTES[(args.storage, dim)]
    # the first-order equilibrium reads and writes the previous (phi u), three
    # values per cell in the arithmetic type
    hist = 6 * (8 if args.storage == "fp64" else 4) if args.cac_edf else 0
    rows = s.phi_partial_rows()
    if rows:
        kernel, phi_kernel = "k_collide_nphi", "k_phi_merge"
        kbytes = nphi_bytes(args.storage, rows)[0] + hist
    else:
        kernel, kbytes, phi_kernel = "k_collide", ab["collide"] + hist, "k_phi"
    method_bytes = ab["method"] + hist
    t_col = ms_col / args.steps / 1e3
    # roofline of the dominant kernel on the method's algorithmic bytes per
    # cell (read and write every population once, write and read phi once);
    # the kernel's own figure (its partial sums of phi included) beside it
    achieved = method_bytes * N / t_col / 1e9
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
        "dtype": {"fp32": "f32", "fp64": "f64", "fp16s": "f16s+f32",
                  "fp16s_all": "f16s"}[args.storage],
        "data": "synthetic",
        "config": {"workload": label, "cells": N,
                   "lattice": "D3Q27+D3Q27" if dim == 3 else "D2Q9+D2Q9",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": profiled_traffic(args.storage + variant, wtag, kernel),
                     "kernel": kernel, "alg_bytes_per_cell": method_bytes,
                     "kernel_bytes_per_cell": kbytes,
                     "kernel_frac": round(kbytes * N / t_col / 1e9 / HBM_PEAK_GBS, 4),
                     "avg_launch_us": round(t_col * 1e6, 2),
                     "phi_stage_kernel": phi_kernel,
                     "phi_stage_avg_launch_us": round(ms_phi / args.steps * 1e3, 2)},
        "method_alg_GBs": round(method_bytes * N * args.steps / (ms / 1e3) / 1e9, 1),
        "method_frac": round(method_bytes * N * args.steps / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "phase_mass_rel_drift": abs(red[0] - m0) / m0,
        "status": "ok" if rc == mplb.OK else "unstable",
        "device": device_info(),
    }
    del s
    # the oracle leg belongs to the default method's line (a variant's line is
    # compared with the default one, on the same box)
    if not args.no_cpu_baseline and dim == 3 and not variant:
        slab = lambda nz: inputs.rti3d(nz=nz, amp=0.05 * 128)  # noqa: E731
        cpu, ref = cpu_baseline(slab, args.cpu_seconds)
        cpu["gpu_speedup"] = round(mlups / cpu["value"], 1)
        line["cpu_baseline"] = cpu
        line["error_vs_fp64"] = error_vs_oracle(slab(128), args.storage, ref)
        line["cpu_baseline"]["c1"] = c1_timing()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
