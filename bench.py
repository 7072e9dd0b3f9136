#!/usr/bin/env python3
"""Benchmark of the coupled phase-field / hydrodynamic LBM step on one GPU.

One step = the phase-field sweep plus the hydrodynamic sweep over the whole
grid (walls, forces and the storage codec included).  Default workload: the
512^3 bubble swarm (200 bubbles, D ~ U[16, 32], rising-bubble physics, walls
at y = 0 and 511) with FP32 PDF storage and FP32 collision arithmetic.
Inputs are resident in HBM before the timed region starts.

Prints ONE JSON line: coupled MLUPS (fluid cells x steps / s / 1e6), the
roofline of the dominant kernel (the fused kernel: hydrodynamic sweep of one
step with the phase-field sweep of the next) from HIP-event timings on the
solver stream, the same measurements for the other storage formats (FP64,
the paper's arithmetic, and FP16/BF16 shifted populations) on the same
workload under "other_storages", the straightforward six-kernel algorithm
(Alg. naiveAlgorithm, Sec. 4.2) under "straightforward_algorithm" beside the
paper's 211 vs 550 MLUPS, every built pair of velocity sets (the stencil study
of Sec. 5.1) under "lattice_variants", the surrogate study's figures from its
committed summary (marked stale if the sources changed since), the surrogate
network's convolutions against the BF16 MFMA peak under "surrogate_network",
and the FP64 CPU oracle timed on the host on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD_KEYS = {
    "bubble_swarm_512": "bubble_swarm_512",
    "rising_bubble_128x512x128": "rising_bubble_128x512x128",
    "static_droplet_32": "static_droplet_32",
    "paper_bubble_260": "paper_bubble_260",
    "rising_bubble_256x1024x256": "rising_bubble_256x1024x256",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    from paper_2012_06144_amd import perf
    return perf.kernel_source_hash()


def load_traffic(kernel: str, workload: str, storage: str, src_hash: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{storage}_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^traffic_json:\s*(\{.*\})\s*$", text, flags=re.M)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("source_hash") != src_hash:
        return None
    return d


def surrogate_source_hash() -> str:
    from paper_2012_06144_amd import perf
    return perf.surrogate_source_hash()


def load_surrogate_study():
    """Speedup and rise-velocity error of the surrogate-accelerated run against
    the plain FP32 run (40000 steps, 256x1024x256), from the committed study
    summary if it was taken on the current sources (else marked stale)."""
    path = os.path.join(ROOT, "profiles", "surrogate_jump_rising_bubble_256x1024x256.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"^study_json:\s*(\{.*\})\s*$", open(path).read(), flags=re.M)
    if not m:
        return None
    d = json.loads(m.group(1))
    d["source"] = "profiles/surrogate_jump_rising_bubble_256x1024x256.md"
    d["stale"] = d.get("source_hash") != surrogate_source_hash()
    return d


def host_cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measure_storage(lbm, perf, setup, phi, u, ps, storage, steps, warmup, timed_steps, src_hash):
    """Throughput of the same workload with another PDF storage format: the
    coupled steps timed with HIP events on the solver stream, the dominant
    kernel's mean launch time (the fused kernel where the format has one,
    else the hydrodynamic sweep) and the relative drift of sum(phi)."""
    import torch
    fluid = setup.nx * setup.nz * (setup.ny - 2 if setup.walls_y else setup.ny)
    solver = lbm.Solver(setup.physics(), storage=storage, device="cuda:0")
    solver.init_fields(phi, u, ps)
    stream = torch.cuda.current_stream(torch.device("cuda:0"))
    m0 = solver.reduce_mass()
    if warmup > 0:
        solver.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    solver.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    m1 = solver.reduce_mass()
    bpc = perf.bytes_per_cell(storage)
    nt = max(2, min(timed_steps, 4096))
    fused_ms = None
    if os.environ.get("LBM_FUSE", "1") != "0":
        try:
            fused_ms = solver.step_timed_fused(nt)
        except lbm.LbmError:
            fused_ms = None
    if fused_ms is not None:
        kern, kbpc, kms = "fused_sweep", bpc["fused"], fused_ms
        step_bpc = bpc["fused"]
    else:
        _, hydro_ms = solver.step_timed(nt)
        kern, kbpc, kms = "hydro_sweep", bpc["hydro"], hydro_ms
        step_bpc = bpc["total"]
    solver.close()
    del solver
    torch.cuda.empty_cache()
    kgbs = kbpc * fluid / (kms * 1e-3) / 1e9
    traffic = load_traffic(kern, setup.name, storage, src_hash)
    return {
        "storage": storage, "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4),
        "mlups": round(fluid / (ms * 1e-3) / 1e6, 1),
        "coupled_gbs": round(step_bpc * fluid / (ms * 1e-3) / 1e9, 1), "bytes_per_cell": step_bpc,
        "roofline": {"bound": "hbm", "kernel": kern, "achieved": round(kgbs, 1), "peak": perf.HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(kgbs / perf.HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else traffic["bytes_per_launch"],
                     "bytes_per_cell": kbpc, "units_per_launch": fluid, "launch_ms": round(kms, 4)},
        "mass_drift_rel": (m1 - m0) / m0,
    }


def measure_straightforward(lbm, perf, setup, phi, u, ps, storage, steps, warmup):
    """The straightforward algorithm (six kernels per step, Sec. 4.2) on the
    same workload: coupled steps timed with HIP events on the solver stream,
    algorithmic bytes of its six passes, and the drift of sum(phi)."""
    import torch
    fluid = setup.nx * setup.nz * (setup.ny - 2 if setup.walls_y else setup.ny)
    solver = lbm.Solver(setup.physics(), storage=storage, device="cuda:0")
    solver.init_fields(phi, u, ps)
    stream = torch.cuda.current_stream(torch.device("cuda:0"))
    m0 = solver.reduce_mass()
    if warmup > 0:
        solver.step_straightforward(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    solver.step_straightforward(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    m1 = solver.reduce_mass()
    solver.close()
    del solver
    torch.cuda.empty_cache()
    bpc = perf.bytes_per_cell(storage)["straightforward"]
    return {"storage": storage, "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4),
            "mlups": round(fluid / (ms * 1e-3) / 1e6, 1), "bytes_per_cell": bpc,
            "achieved_gbs": round(bpc * fluid / (ms * 1e-3) / 1e9, 1), "mass_drift_rel": (m1 - m0) / m0}


LATTICE_VARIANTS = {
    "d3q15_d3q27": dict(lattice_phase=15, lattice_hydro=27, phase_mrt=False),
    "d3q15_d3q27_mrt": dict(lattice_phase=15, lattice_hydro=27, phase_mrt=True),
    "d3q19_d3q19": dict(lattice_phase=19, lattice_hydro=19, phase_mrt=False),
    "d3q19_d3q19_mrt": dict(lattice_phase=19, lattice_hydro=19, phase_mrt=True),
    "d3q27_d3q27": dict(lattice_phase=27, lattice_hydro=27, phase_mrt=False),
    "d3q15_d3q15": dict(lattice_phase=15, lattice_hydro=15, phase_mrt=False),
}


def measure_lattice(lbm, perf, setup, phi, u, ps, name, storage, steps, warmup, timed_steps):
    """One velocity-set variant (the stencil study of Sec. 5.1) on the same
    workload: coupled steps timed with HIP events on the solver stream and
    the fused kernel's mean launch time, against its algorithmic bytes."""
    import torch
    lat = LATTICE_VARIANTS[name]
    fluid = setup.nx * setup.nz * (setup.ny - 2 if setup.walls_y else setup.ny)
    solver = lbm.Solver(dict(setup.physics(), **lat), storage=storage, device="cuda:0")
    solver.init_fields(phi, u, ps)
    stream = torch.cuda.current_stream(torch.device("cuda:0"))
    m0 = solver.reduce_mass()
    if warmup > 0:
        solver.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    solver.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    m1 = solver.reduce_mass()
    fused_ms = solver.step_timed_fused(max(2, min(timed_steps, 4096)))
    solver.close()
    del solver
    torch.cuda.empty_cache()
    bpc = perf.bytes_per_cell(storage, lat["lattice_phase"], lat["lattice_hydro"])
    return {"storage": storage, "phase_set": lat["lattice_phase"], "hydro_set": lat["lattice_hydro"],
            "phase_mrt": lat["phase_mrt"], "ms_per_step": round(ms, 4),
            "mlups": round(fluid / (ms * 1e-3) / 1e6, 1), "fused_bytes_per_cell": bpc["fused"],
            "fused_ms": round(fused_ms, 4),
            "fused_gbs": round(bpc["fused"] * fluid / (fused_ms * 1e-3) / 1e9, 1),
            "mass_drift_rel": (m1 - m0) / m0}


def cpu_baseline(setup, phi, u, ps, target_s: float = 15.0):
    """Time the FP64 oracle on a 128 x ny x 128 slab of the same workload."""
    import numpy as np

    from oracle import oracle as orc
    nx = min(128, setup.nx)
    nz = min(128, setup.nz)
    phys = setup.physics()
    phys.update(nx=nx, nz=nz)
    o = orc.Oracle(orc.Params(**phys))
    o.init(np.ascontiguousarray(phi[:nz, :, :nx]), np.ascontiguousarray(u[:, :nz, :, :nx]),
           np.ascontiguousarray(ps[:nz, :, :nx]))
    fluid = nx * nz * (setup.ny - 2 if setup.walls_y else setup.ny)
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter()
    per = t1 - t0
    extra = max(0, min(9, int(target_s / max(per, 1e-3)) - 1))
    if extra:
        o.step(extra)
    t2 = time.perf_counter()
    steps = 1 + extra
    mlups = fluid * steps / (t2 - t0) / 1e6
    o.close()
    return {"value": mlups, "unit": "MLUPS", "cores": orc.num_threads(), "kind": "oracle",
            "cpu_model": host_cpu_model(),
            "sample": f"{steps} coupled steps of the FP64 oracle on a {nx}x{setup.ny}x{nz} slab of "
                      f"the {setup.name} fields ({fluid} fluid cells), {t2 - t0:.1f} s"}


def measure_network(shape=(8, 64, 96, 64), reps=5):
    """The surrogate network's MFMA convolutions on one batch of the
    training crop: the inference forward pass (decoder inputs read without
    forming them) and a forward + backward pass, timed with HIP events on
    the current stream, against the 2.5 PFLOP/s BF16 dense peak."""
    import torch

    from paper_2012_06144_amd import surrogate as S
    net = S.Net(seed=0)
    n, d, h, w = shape
    g = torch.Generator(device="cpu").manual_seed(1)
    x = (torch.randn((n, d, h, w, S.C_IN), generator=g) * 0.5).to(net.device, torch.bfloat16)
    stream = torch.cuda.current_stream(net.device)

    def timed(fn, k):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    def fwd_bwd():
        out = net.forward(x, keep=True)
        net.backward(torch.zeros(out.shape, device=net.device, dtype=torch.bfloat16))

    flop = S.flops_per_voxel() * n * d * h * w
    t_f = timed(lambda: net.forward(x, keep=False), reps)
    t_fb = timed(fwd_bwd, max(1, reps // 2))
    peak = 2500.0
    rec = {"shape": list(shape), "params": net.n_params(), "forward_ms": round(t_f, 4),
           "forward_tflops": round(flop / (t_f * 1e-3) / 1e12, 1),
           "roofline": {"bound": "mfma", "achieved": round(flop / (t_f * 1e-3) / 1e12, 1), "peak": peak,
                        "unit": "TFLOP/s", "frac": round(flop / (t_f * 1e-3) / 1e12 / peak, 4)},
           "forward_backward_ms": round(t_fb, 4),
           "forward_backward_tflops": round(3 * flop / (t_fb * 1e-3) / 1e12, 1)}
    del net, x
    torch.cuda.empty_cache()
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="bubble_swarm_512", choices=sorted(WORKLOAD_KEYS))
    ap.add_argument("--storage", default="f32", choices=["f64", "f32", "f16s", "bf16s"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timed-steps", type=int, default=50,
                    help="steps of the per-kernel event timing (roofline)")
    ap.add_argument("--lattices", default="f64,f32",
                    help="comma-separated storage formats (f64, f32) for which every built velocity-set variant "
                         "is measured on the same workload (empty: none)")
    ap.add_argument("--straightforward", default="f64,f32",
                    help="comma-separated storage formats (f64, f32) for which the straightforward six-kernel "
                         "algorithm is measured on the same workload (empty: none)")
    ap.add_argument("--no-network", action="store_true", help="skip the surrogate network's convolution timing")
    ap.add_argument("--other-storages", default="f64,f16s,bf16s",
                    help="comma-separated storage formats measured after the main one on the same workload "
                         "(empty: none)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU: the coupled step is built and measured on a single "
              f"MI355X (requested --gpus {args.gpus}, WORLD_SIZE {world}); multi-GPU domain "
              f"decomposition is not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2012_06144_amd import inputs, lbm, perf

    setup = inputs.WORKLOADS[WORKLOAD_KEYS[args.workload]]()
    log(f"[bench] workload {setup.name} {setup.nx}x{setup.ny}x{setup.nz} storage {args.storage}")
    t = time.perf_counter()
    phi, u, ps = inputs.build_fields(setup)
    log(f"[bench] inputs built in {time.perf_counter() - t:.1f}s")

    dev = torch.device("cuda:0")
    solver = lbm.Solver(setup.physics(), storage=args.storage, device="cuda:0")
    solver.init_fields(phi, u, ps)
    fluid = setup.nx * setup.nz * (setup.ny - 2 if setup.walls_y else setup.ny)
    stream = torch.cuda.current_stream(dev)

    mass0 = solver.reduce_mass()
    log(f"[bench] warmup {args.warmup} steps")
    if args.warmup > 0:
        solver.step(args.warmup)
    torch.cuda.synchronize()

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    log(f"[bench] timed {args.steps} steps")
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    solver.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1) / args.steps
    mass1 = solver.reduce_mass()
    mlups = fluid / (ms * 1e-3) / 1e6
    log(f"[bench] {ms:.3f} ms/step, {mlups:.0f} MLUPS (wall {wall:.2f}s)")

    # per-kernel durations (HIP events around each sweep on the solver stream)
    nt = max(1, min(args.timed_steps, 4096))
    phase_ms, hydro_ms = solver.step_timed(nt)
    bpc = perf.bytes_per_cell(args.storage)
    hydro_gbs = bpc["hydro"] * fluid / (hydro_ms * 1e-3) / 1e9
    phase_gbs = bpc["phase"] * fluid / (phase_ms * 1e-3) / 1e9
    log(f"[bench] phase {phase_ms:.3f} ms ({phase_gbs:.0f} GB/s), hydro {hydro_ms:.3f} ms "
        f"({hydro_gbs:.0f} GB/s)")
    # the timed steps ran the fused kernel (hydrodynamic sweep of one step with the phase
    # sweep of the next) unless the storage has none or LBM_FUSE=0: then it is the
    # dominant kernel, timed the same way
    fused_ms = None
    if os.environ.get("LBM_FUSE", "1") != "0":
        try:
            fused_ms = solver.step_timed_fused(max(2, nt))
        except lbm.LbmError:
            fused_ms = None
    if fused_ms is not None:
        rl_kernel, rl_bpc, rl_ms = "fused_sweep", bpc["fused"], fused_ms
    else:
        rl_kernel, rl_bpc, rl_ms = "hydro_sweep", bpc["hydro"], hydro_ms
    rl_gbs = rl_bpc * fluid / (rl_ms * 1e-3) / 1e9
    step_bpc = bpc["fused"] if fused_ms is not None else bpc["total"]
    coupled_gbs = step_bpc * fluid / (ms * 1e-3) / 1e9
    if fused_ms is not None:
        log(f"[bench] fused {fused_ms:.3f} ms ({rl_gbs:.0f} GB/s)")

    # STREAM copy bandwidth b_s (the paper's roofline denominator)
    nbytes = 4 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    lbm.lbm_stream_copy(a, b, nbytes, stream.cuda_stream)
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    reps = 10
    for _ in range(reps):
        lbm.lbm_stream_copy(a, b, nbytes, stream.cuda_stream)
    c1.record(stream)
    torch.cuda.synchronize()
    b_s = 2 * nbytes * reps / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del a, b
    log(f"[bench] STREAM copy b_s = {b_s:.0f} GB/s")

    src_hash = kernel_source_hash()
    traffic = load_traffic(rl_kernel, setup.name, args.storage, src_hash)
    traffic_val = None
    if traffic is not None:
        traffic_val = traffic["bytes_per_launch"]

    solver.close()
    del solver
    torch.cuda.empty_cache()
    others = {}
    for st in [x for x in args.other_storages.split(",") if x and x != args.storage]:
        log(f"[bench] storage {st}: warmup {args.warmup}, timed {args.steps} steps")
        rec = measure_storage(lbm, perf, setup, phi, u, ps, st, args.steps, args.warmup, args.timed_steps,
                              src_hash)
        log(f"[bench] storage {st}: {rec['ms_per_step']:.3f} ms/step, {rec['mlups']:.0f} MLUPS, "
            f"{rec['roofline']['kernel']} {rec['roofline']['achieved']:.0f} GB/s")
        others[st] = rec

    naive = {}
    for st in [x for x in args.straightforward.split(",") if x]:
        log(f"[bench] straightforward algorithm, storage {st}: warmup {args.warmup}, timed {args.steps} steps")
        rec = measure_straightforward(lbm, perf, setup, phi, u, ps, st, args.steps, args.warmup)
        improved = mlups if st == args.storage else others.get(st, {}).get("mlups")
        rec["improved_mlups"] = None if improved is None else round(improved, 1)
        rec["improved_over_straightforward"] = None if improved is None else round(improved / rec["mlups"], 3)
        log(f"[bench] straightforward {st}: {rec['ms_per_step']:.3f} ms/step, {rec['mlups']:.0f} MLUPS, "
            f"{rec['achieved_gbs']:.0f} GB/s algorithmic")
        naive[st] = rec

    lattices = {}
    for st in [x for x in args.lattices.split(",") if x]:
        for name in LATTICE_VARIANTS:
            log(f"[bench] lattice {name}, storage {st}: warmup {args.warmup}, timed {args.steps} steps")
            rec = measure_lattice(lbm, perf, setup, phi, u, ps, name, st, args.steps, args.warmup,
                                  args.timed_steps)
            log(f"[bench] lattice {name} {st}: {rec['ms_per_step']:.3f} ms/step, {rec['mlups']:.0f} MLUPS, "
                f"fused {rec['fused_gbs']:.0f} GB/s algorithmic")
            lattices[f"{name}_{st}"] = rec

    network = None
    if not args.no_network:
        log("[bench] surrogate network convolutions (batch 8 x 64 x 96 x 64)")
        network = measure_network()
        log(f"[bench] network forward {network['forward_ms']:.2f} ms ({network['forward_tflops']:.0f} TFLOP/s), "
            f"forward+backward {network['forward_backward_ms']:.2f} ms")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(setup, phi, u, ps)
        log(f"[bench] oracle {cpu['value']:.2f} MLUPS on {cpu['cores']} threads")

    line = {
        "metric": "coupled MLUPS + %HBM roofline; surrogate-vs-plain speedup at \u22641% rise-vel error",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16s": "f32 (f16 storage)",
                  "bf16s": "f32 (bf16 storage)"}[args.storage],
        "data": "synthetic",
        "config": {"workload": setup.name, "grid": [setup.nx, setup.ny, setup.nz],
                   "fluid_cells": fluid, "storage": args.storage,
                   "walls_y": bool(setup.walls_y), "bubbles": setup.n_bubbles or 1},
        "roofline": {"bound": "hbm", "kernel": rl_kernel,
                     "achieved": round(rl_gbs, 1), "peak": perf.HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(rl_gbs / perf.HBM_PEAK_GBS, 4), "traffic": traffic_val,
                     "bytes_per_cell": rl_bpc, "units_per_launch": fluid,
                     "launch_ms": round(rl_ms, 4)},
        "kernels": {"phase_ms": round(phase_ms, 4), "phase_gbs": round(phase_gbs, 1),
                    "hydro_ms": round(hydro_ms, 4), "hydro_gbs": round(hydro_gbs, 1),
                    "fused_ms": None if fused_ms is None else round(fused_ms, 4),
                    "fused_gbs": None if fused_ms is None else round(rl_gbs, 1)},
        "coupled_gbs": round(coupled_gbs, 1),
        "coupled_frac_hbm": round(coupled_gbs / perf.HBM_PEAK_GBS, 4),
        "stream_copy_gbs": round(b_s, 1),
        "coupled_frac_stream": round(coupled_gbs / b_s, 4),
        "bytes_per_cell": step_bpc,
        "mlups_all_cells": round(setup.cells / (ms * 1e-3) / 1e6, 1),
        "mass_drift_rel": (mass1 - mass0) / mass0,
        "paper_context": {"mlups": 550, "hardware": "Tesla P100", "precision": "f64",
                          "roofline_frac_of_stream": 0.78},
        "other_storages": others,
        "lattice_variants": lattices,
        "straightforward_algorithm": {"records": naive, "paper": {"straightforward_mlups": 211, "improved_mlups": 550,
                                                                "hardware": "Tesla P100", "precision": "f64"}},
        "cpu_baseline": cpu,
        "surrogate": load_surrogate_study(),
        "surrogate_network": network,
        "kernel_source_hash": src_hash,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
