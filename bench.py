"""Benchmark: DOF-stage updates/s of the IMEX ARK step on the flat-plate boundary layer.

Workload (default): 256x128 quads on [0,2]x[0,0.5], wall-normal stretching to
aspect ratio 1000, the 16 wall rows implicit HDG-MX, the rest explicit DG-IP,
degree 4, ARS(3,4,3); Re 1e4, Ma 0.3, Pr 0.72.  One step = one full pass of the
hot path: every explicit stage residual and ERK combination, every implicit
Newton stage (assembly, mixed elimination, LU + condensation, GMRES facet
solve, back-substitution) and the interface coupling.

value = N_DOF * s * steps / time, N_DOF = n_elem (k+1)^2 4, s = 3 stages.
Inputs are resident in device memory before the timed region starts.

Prints one JSON line.  Also reports:
  roofline      the dominant kernel's achieved rate against the MI355X peak
  cpu_baseline  the CPU oracle timed on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="boundary_layer")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (calibrates HBM traffic counters)")
    return ap.parse_args()


def cpu_baseline(seconds_budget: float = 25.0):
    """The oracle on a bounded sample of the boundary-layer workload: a 2x16 strip of the
    same mesh family (k=4, ARS(3,4,3), HDG-MX on the 2 wall rows = 1/8 implicit like the
    full mesh), one step, single thread."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:                       # pragma: no cover
        threadpool_limits = None
    from paper_2607_16044_amd import workloads
    from oracle.ark import IMEXSolver
    wl = workloads.boundary_layer(nx=2, ny=16, k=4, implicit_rows=2, Lx=2 * 2.0 / 256, height=None, steps=1,
                                  name="boundary_layer_sample")
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        s = IMEXSolver(wl)
        t0 = time.perf_counter()
        s.step()
        dt = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.unregister() if hasattr(ctx, "unregister") else None
    dof_stage = wl.n_dof * wl.stages
    return {"value": dof_stage / dt, "unit": "DOF-stage updates/s", "cores": 1, "kind": "oracle",
            "sample": f"boundary layer 2x16 strip (k=4, 2 implicit HDG-MX rows), 1 ARS(3,4,3) step, {dt:.1f} s"}


def assembly_flops(wl):
    """Dense element-Jacobian contraction flops per implicit element."""
    k = wl.degree
    nq = (3 * k + 2) // 2
    nn, nqv = (k + 1) ** 2, nq * nq
    nu, nf = 4 * nn, 16 * (k + 1)
    nqm = 5 * nn
    # volume and face sandwich products B^T J B for the blocks K, A12, A21 (+ C, D, E, A23, A32 on faces)
    vol = 2 * nqv * (nu * nu * 2 + nu * nqm * 2 + nqm * nu * 2)
    face = 2 * 4 * nq * (nu * nu + nu * nqm) + 2 * nq * (nu * nf + nf * nu + nf * nf + nqm * nf + nf * nqm)
    return vol + face


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; multi-GPU sharding is described in DESIGN.md "
                                   "and not built", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2607_16044_amd import binding, workloads
    if not os.path.exists(binding.LIB_PATH):
        from paper_2607_16044_amd import build
        build.build()
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = workloads.get(args.workload)
    prec = 0 if args.precision == "fp64" else 1
    eng = binding.Engine(wl, precision=prec)
    U = eng.initial_state()
    Uhat = eng.init_facets(U)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        eng.ark_step(wl.dt, U, Uhat)
    eng.reset_timers()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    newton = gmres = 0
    for _ in range(args.steps):
        st = eng.ark_step(wl.dt, U, Uhat)
        newton += st["newton_its"]
        gmres += st["gmres_its"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timers = eng.timers()
    phases = {k[:-3]: round(v / args.steps, 3) for k, v in timers.items() if k.endswith("_ms") and v > 0}
    n_dof = wl.n_dof
    s = wl.stages
    value = n_dof * s * args.steps / elapsed
    # dominant kernel: the element assembly (see the design doc for the algorithmic flop count)
    roof = None
    if timers["assemble_launches"] > 0:
        avg_ms = timers["assemble_ms"] / timers["assemble_launches"]
        flops = assembly_flops(wl) * eng.sizes["n_implicit"]
        achieved = flops / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma" if False else "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                "kernel": "hdg_assemble_kernel<4,true>", "avg_ms": avg_ms}
    out = {
        "metric": "DOF-stage updates/s, FP32+refine/batched vs plain FP64 GPU at <=1e-9 rel err",
        "value": value,
        "unit": "DOF-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "mesh": f"{wl.nx}x{wl.ny}", "degree": wl.degree, "n_dof": n_dof,
                   "implicit_elements": eng.sizes["n_implicit"], "tableau": wl.tableau, "stages": s,
                   "hdg": "MX" if wl.hdg_variant == workloads.HDG_MX else "IP", "precision": args.precision,
                   "newton_its_per_step": newton / args.steps, "gmres_its_per_step": gmres / args.steps},
        "roofline": roof,
        "phases_ms_per_step": phases,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
