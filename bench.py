"""Benchmark of the grid-integration hot path on one MI355X.

One step = gint_vlocal + gint_rho + gint_force_stress (Eq. 2-5), the three
calls a DFT code makes (rho comes first in a self-consistent step, V is built
from it, and the force uses that V).  The fused gint_rho_force_stress (rho
and the force from one pass, for callers that hold V and D together) is
timed once and reported beside the step, not in it.  Default
workload: the 868-atom twisted bilayer graphene slab (commensurate i = 8,
3.89 deg, 312 x 312 x 120 grid, 13 orbitals per C, rcut 8 Bohr).  Inputs are
synthetic and already resident in HBM when the timed region starts; the plan
(neighbour lists and work items) is built once per geometry, outside the
timed region, and its build time is reported separately.

The metric compares the mixed-precision form with the plain FP64 path on the
same workload: `value` is the throughput of the form named by --precision
(default fp16x3), and the line carries the FP64 path's throughput and the
speedup over it (--compare fp64, the default).  The errors of each form
against the FP64 oracle are measured by the GPU tests.

Throughput: W / t_step with W = sum_g n_orb(g)^2 (grid points x ordered
orbital pairs within rcut), counted exactly by the library.  Prints one JSON
line.  --config 3 runs the batch of 64 random C/H/O crystals in one plan;
--graph replays a captured HIP graph of the step; --autotune picks the tile
shape by timed trials first.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6    # MI355X dense FP64 (matrix and vector)
PEAK_FP16_TFLOPS = 2500.0  # MI355X dense FP16 / BF16 matrix
PRECISIONS = {"fp64": 0, "fp16x3": 1, "bf16x3": 2}
DTYPES = {0: "f64", 1: "f16x3 (f32 acc)", 2: "bf16x3 (f32 acc)"}
UNIT = "grid-pts*orbital-pairs/s"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(system, target_seconds: float = 15.0):
    """The FP64 oracle (as it stands) on a slab of the same workload's grid
    points: Vlocal + rho + force/stress restricted to a contiguous range of
    flat grid indices (whole n1-planes near the middle of the cell)."""
    from oracle import oracle as orc
    o = orc.Oracle(system)
    plane = int(system.grid[1]) * int(system.grid[2])
    n1 = int(system.grid[0])
    g0 = (n1 // 2) * plane
    # calibrate on one plane, then size the slab to the target time
    t = time.perf_counter()
    o.vlocal(g_range=(g0, g0 + plane))
    o.rho(g_range=(g0, g0 + plane))
    o.force_stress(g_range=(g0, g0 + plane))
    dt1 = time.perf_counter() - t
    nplanes = int(max(1, min(n1 // 2, round(target_seconds / max(dt1, 1e-3)))))
    g1 = g0 + nplanes * plane
    ws = o.work((g0, g1))
    t = time.perf_counter()
    o.vlocal(g_range=(g0, g1))
    o.rho(g_range=(g0, g1))
    o.force_stress(g_range=(g0, g1))
    dt = time.perf_counter() - t
    return {"value": ws / dt, "unit": UNIT, "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"{system.name}: Vlocal+rho+force/stress over grid planes n1={n1 // 2}.."
                      f"{n1 // 2 + nplanes - 1} ({nplanes} of {n1} planes, W_sample={ws:.4g}, {dt:.1f} s)"}


def workload_name(cfg, systems):
    s = systems[0]
    if len(systems) > 1:
        return (f"batch of {len(systems)} random C/H/O crystals ({min(x.natom for x in systems)}-"
                f"{max(x.natom for x in systems)} atoms, 13/5/13 orbitals, rcut 7/6/8 Bohr, grids "
                f"{min(int(x.grid[0]) for x in systems)}^3-{max(int(x.grid[0]) for x in systems)}^3) in one plan")
    if cfg == 1:
        return "jittered diamond, 8 C atoms, grid 32^3, 13 orbitals/atom, rcut 6 Bohr"
    return (f"twisted bilayer graphene ({s.natom} C atoms), grid {'x'.join(str(int(x)) for x in s.grid)}, "
            f"13 orbitals/atom, rcut 8 Bohr")


def run_form(G, torch, dev, systems, prec, args, bufs):
    """Plan, warm up and time one precision form; returns its measurements."""
    target = systems if len(systems) > 1 else systems[0]
    tune = None
    opts = dict(cluster_atoms=args.cluster_atoms, max_bigcells_per_item=args.max_bigcells)
    if args.autotune:
        chosen, tune = G.autotune(target, precision=prec, budget_seconds=args.tune_seconds)
        opts = dict(cluster_atoms=chosen["cluster_atoms"], max_bigcells_per_item=chosen["max_bigcells_per_item"])
        log(f"[bench] autotune {DTYPES[prec]}: {opts} {tune}")
    t = time.perf_counter()
    plan = G.Plan(target, precision=prec, **opts)
    plan_s = time.perf_counter() - t
    log(f"[bench] plan {DTYPES[prec]} {plan.info()} wall {plan_s:.2f} s")
    v, d, h, rho, ne, F, sig, E, Wt = (bufs[k] for k in ("v", "d", "h", "rho", "ne", "F", "sig", "E", "W"))
    G.gint_work_units(plan, Wt)
    torch.cuda.synchronize()
    W = float(Wt.cpu().sum())
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        G.gint_vlocal(plan, v, h)
        if ev is not None:
            ev[1].record(stream)
        G.gint_rho(plan, d, rho, ne)
        if ev is not None:
            ev[2].record(stream)
        G.gint_force_stress(plan, v, d, F, sig, E)
        if ev is not None:
            ev[3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the fused rho + force pass, once (reported, not part of the timed step)
    fev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    G.gint_rho_force_stress(plan, v, d, rho, F, sig, n_elec=ne, energy=E)
    fev[0].record(stream)
    G.gint_rho_force_stress(plan, v, d, rho, F, sig, n_elec=ne, energy=E)
    fev[1].record(stream)
    torch.cuda.synchronize()
    fused_ms = fev[0].elapsed_time(fev[1])
    # per-kernel durations: HIP events on the stream the library launches on
    if args.graph:
        graph = G.Graph(plan, v_loc=v, d_vals=d, h_vals=h, rho=rho, n_elec=ne, force=F, stress=sig, energy=E)
        graph.launch()
        torch.cuda.synchronize()
        kev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        step(kev)
        torch.cuda.synchronize()
        kern_ms = {"vlocal": kev[0].elapsed_time(kev[1]), "rho": kev[1].elapsed_time(kev[2]),
                   "force_stress": kev[2].elapsed_time(kev[3])}
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.launch()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        graph.close()
    else:
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
        t0 = time.perf_counter()
        for k in range(args.steps):
            step(evs[k])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        ms = {"vlocal": [], "rho": [], "force_stress": []}
        for e in evs:
            ms["vlocal"].append(e[0].elapsed_time(e[1]))
            ms["rho"].append(e[1].elapsed_time(e[2]))
            ms["force_stress"].append(e[2].elapsed_time(e[3]))
        kern_ms = {k: float(np.mean(x)) for k, x in ms.items()}
    log(f"[bench] {DTYPES[prec]} per-call ms {kern_ms} (fused rho+force {fused_ms:.2f} ms), "
        f"step {elapsed / args.steps * 1e3:.2f} ms")
    plan.close()
    return {"value": W * args.steps / elapsed, "ms_per_step": elapsed / args.steps * 1e3, "kernel_ms": kern_ms,
            "fused_rho_force_stress_ms": fused_ms, "W": W, "plan_seconds": plan_s, "options": opts, "autotune": tune}


PROFILE = os.path.join(ROOT, "profiles", "gint_tbg868_counters.md")
KERNEL_NAMES = {0: {"vlocal": "k_vlocal", "rho": "k_rho", "force_stress": "k_force<false>"},
                1: {"vlocal": "k_vlocal_mx<fp16>", "rho": "k_rho_mx<fp16>", "force_stress": "k_force_mx<fp16,false>"},
                2: {"vlocal": "k_vlocal_mx<bf16>", "rho": "k_rho_mx<bf16>", "force_stress": "k_force_mx<bf16,false>"}}


def sources_sha256(prec):
    """Hash of the kernel sources of a precision form (as recorded with the
    counter profile)."""
    import hashlib
    base = os.path.join(ROOT, "paper_2409_09399_amd", "csrc")
    main = "gint_kernels.hip" if prec == 0 else "gint_kernels_mixed.hip"
    h = hashlib.sha256()
    for f in (main, "gint_device.h", "gint_internal.h"):
        with open(os.path.join(base, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(cfg, prec, key):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary of the bilayer workload (FETCH_SIZE and WRITE_SIZE calibrated
    with a plain copy), or None when the workload differs, the kernel was not
    profiled, or its sources changed since the counters were taken."""
    import re
    if cfg != 2 or not os.path.exists(PROFILE):
        return None
    with open(PROFILE) as fh:
        m = re.search(r"<!-- traffic (\[.*\]) -->", fh.read())
    if not m:
        return None
    name, sha = KERNEL_NAMES[prec].get(key), sources_sha256(prec)
    for r in json.loads(m.group(1)):
        if r["kernel"] == name and r.get("sources_sha256") == sha:
            return r["read_bytes"] + r["write_bytes"]
    return None


def roofline(form, prec, cfg):
    # dominant kernel against its contraction roofline: 2 flops per unit of W
    km = form["kernel_ms"]
    dom = max(km, key=km.get)
    peak = PEAK_FP64_TFLOPS if prec == 0 else PEAK_FP16_TFLOPS
    achieved = 2.0 * form["W"] / (km[dom] * 1e-3) / 1e12
    return {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": profiled_traffic(cfg, prec, dom)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2, help="1 diamond, 2 bilayer (868 atoms), 3 batch of 64")
    ap.add_argument("--precision", choices=sorted(PRECISIONS), default="fp16x3")
    ap.add_argument("--compare", choices=sorted(PRECISIONS) + ["none"], default="fp64",
                    help="second form timed on the same workload (speedup reported against it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cluster-atoms", type=int, default=0)
    ap.add_argument("--max-bigcells", type=int, default=0)
    ap.add_argument("--graph", action="store_true", help="time replays of a captured HIP graph of the step")
    ap.add_argument("--autotune", action="store_true", help="choose the tile shape by timed trials first")
    ap.add_argument("--tune-seconds", type=float, default=2.0)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run one plain device-to-device copy of this many bytes (untimed), the "
                         "calibration kernel for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (--gpus {args.gpus} requested); "
              "multi-GPU sharding is a design note, not an implemented path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2409_09399_amd import gint as G
    from paper_2409_09399_amd import inputs as I

    dev = torch.device("cuda:0")
    t = time.perf_counter()
    cfg = I.make_config(args.config)
    systems = cfg if isinstance(cfg, list) else [cfg]
    natom = sum(x.natom for x in systems)
    ngrid = sum(x.ngrid for x in systems)
    nnz = sum(x.nnz for x in systems)
    n = len(systems)
    log(f"[bench] inputs {n} system(s), first {systems[0].name}: natom={natom} ngrid={ngrid} nnz={nnz} "
        f"({time.perf_counter() - t:.1f} s)")
    bufs = {"v": torch.tensor(np.concatenate([x.v for x in systems]), device=dev),
            "d": torch.tensor(np.concatenate([x.d for x in systems]), device=dev),
            "h": torch.empty(nnz, dtype=torch.float64, device=dev),
            "rho": torch.empty(ngrid, dtype=torch.float64, device=dev),
            "ne": torch.empty(n, dtype=torch.float64, device=dev),
            "F": torch.empty(3 * natom, dtype=torch.float64, device=dev),
            "sig": torch.empty(9 * n, dtype=torch.float64, device=dev),
            "E": torch.empty(n, dtype=torch.float64, device=dev),
            "W": torch.empty(n, dtype=torch.float64, device=dev)}

    if args.copy_bytes > 0:
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {src.numel() * 8} bytes done")
        del src, dst

    prec = PRECISIONS[args.precision]
    main_form = run_form(G, torch, dev, systems, prec, args, bufs)
    cmp_form = None
    if args.compare not in ("none", args.precision):
        cmp_prec = PRECISIONS[args.compare]
        c = run_form(G, torch, dev, systems, cmp_prec, args, bufs)
        cmp_form = {"precision": args.compare, "dtype": DTYPES[cmp_prec], "value": c["value"],
                    "ms_per_step": c["ms_per_step"], "kernel_ms": c["kernel_ms"],
                    "fused_rho_force_stress_ms": c["fused_rho_force_stress_ms"],
                    "roofline": roofline(c, cmp_prec, args.config), "plan_options": c["options"]}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline(systems[0], args.cpu_seconds)
        log(f"[bench] cpu baseline {cpu}")

    out = {
        "metric": "grid-pts*orbital-pairs/s for Vlocal+rho+force, mixed vs FP64 at stated error",
        "value": main_form["value"],
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_form["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[prec],
        "data": "synthetic",
        "config": {"workload": workload_name(args.config, systems), "precision": args.precision,
                   "W": main_form["W"], "natom": natom, "ngrid": ngrid, "nnz": nnz, "n_sys": n,
                   "graph": bool(args.graph), "plan_options": main_form["options"]},
        "kernel_ms": main_form["kernel_ms"],
        "fused_rho_force_stress_ms": main_form["fused_rho_force_stress_ms"],
        "plan_seconds": main_form["plan_seconds"],
        "roofline": roofline(main_form, prec, args.config),
        "compare": cmp_form,
        "speedup_vs_compare": (main_form["value"] / cmp_form["value"]) if cmp_form else None,
        "autotune": main_form["autotune"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
