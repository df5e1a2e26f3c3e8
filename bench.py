#!/usr/bin/env python3
"""Throughput of the porous-media lattice Boltzmann hot path on one MI355X.

Workload: D3Q27, FP32 storage and arithmetic, 256^3 periodic box, porosity from a seeded
Gaussian random field (correlation length 16 cells) mapped to phi in (0.3, 1), Kozeny-Carman
permeability with d = 2 cells, Forchheimer coefficient 0.55/sqrt(K), nu = 0.01, body force
1e-6 along x (synthetic inputs; see paper_2606_29619_amd/workloads.py).  A step is one full
update of every cell: moment pass, velocity correction, forcing-collide-stream pass.

Prints one JSON line: MLUPS (whole job), the roofline of the dominant kernel measured with HIP
events on the library's stream over the timed region, secondary rows timed the same way (the
shifted FP16/BF16 forms, the lagged single-pass scheme, FP64, and the 768x384x384 porous-sphere
duct), a bounded sample of the serving stream, and the FP64 CPU oracle timed on a bounded
sample of the same recipe with all host threads and with one.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0            # MI355X HBM3E, published
METRIC = "MLUPS & % HBM roofline (D3Q27); served MLUPS + p50/p99 time-to-steady"


def kernel_bytes_per_cell(Q, D, sp, s, m=0):
    """Algorithmic HBM bytes per cell of each kernel (values each kernel must move once), with
    sp bytes per population, s per static-field or moment value and m per solid-mask byte
    (1 when the run has solid cells, else 0):
    moments: read Q pops + eps, mu_D, mu_F (+ mask); write rho and v^(1) (D+1);
    velocity correction: read rho, v^(1), eps (+ mask); write v (D);
    collide-stream: read Q pops, rho, v, eps, mu_D, mu_F (+ mask); write Q pops."""
    return {
        "moments": Q * sp + (3 + (D + 1)) * s + m,
        "vcorrect": ((D + 1) + 1 + D) * s + m,
        "collide": 2 * Q * sp + ((D + 1) + 3) * s + m,
    }


def lagged_bytes_per_cell(Q, D, sp, s, m=0):
    """Single pass of the lagged scheme: read Q pops, 3 static fields (+ mask) and the previous
    step's rho, v^(1), v; write Q pops and the new rho, v^(1), v."""
    return 2 * Q * sp + (3 + 2 * (2 * D + 1)) * s + m


def method_bytes_per_cell(Q, D, sp, s, lagged=False, m=0):
    """Per-step minimum of the method.  Two-pass: pass one reads Q pops + 3 static fields
    (+ mask) and writes rho, v^(1); pass two reads Q pops, rho, v, 3 static fields (+ mask) and
    writes Q pops."""
    if lagged:
        return lagged_bytes_per_cell(Q, D, sp, s, m)
    return 3 * Q * sp + (3 + (D + 1) + (D + 1) + 3) * s + 2 * m


def source_hash():
    h = hashlib.sha256()
    for rel in ("paper_2606_29619_amd/csrc/lbm_device.hpp", "paper_2606_29619_amd/csrc/lbm_host.hpp",
                "paper_2606_29619_amd/csrc/lbm_launch.hpp", "paper_2606_29619_amd/csrc/lbm.hip"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, tag, src_hash, kind="box", n=256):
    """HBM bytes per launch from the committed rocprofv3 PMC summary of this row (the 256^3 box
    or the 768x384x384 sphere duct; tag: "f32", "f16_porous", "f32_lagged", ...), when it was
    taken on the current kernel source; otherwise None."""
    if kind == "box" and n == 256:
        name = f"pmc_d3q27_{tag}_256.json"
    elif kind == "sphere":
        name = f"pmc_d3q27_sphere_{tag}_768.json"
    else:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        pmc = json.load(fh)
    if pmc.get("source_hash") != src_hash or kernel not in pmc.get("kernels", {}):
        return None
    k = pmc["kernels"][kernel]
    return (k["fetch_kib"] * pmc["fetch_scale"] + k["write_kib"] * pmc["write_scale"]) * 1024.0


def cpu_baseline(budget_s=10.0, workload="box"):
    """The FP64 oracle, as it stands, on a bounded instance of the same recipe: the 64^3 box
    (seed 0), or the sphere duct at 1/8 scale (96 x 48 x 48, radius 12); timed with every
    thread the host gives the process (OpenMP default: OMP_NUM_THREADS, else the core count)
    and again with one thread, each for about budget_s of stepping."""
    import oracle
    from paper_2606_29619_amd import workloads
    if workload == "box":
        w = workloads.random_porosity_3d(n=64, seed=0, ell=16.0)
        what = "D3Q27 64^3 instance of the same random-porosity recipe (seed 0)"
    else:
        w = workloads.sphere_duct_3d(96, 48, 48, radius=12.0, bump_m=8, drive="pressure")
        what = "the sphere-duct recipe at 1/8 scale (96 x 48 x 48, radius 12, bump m = 8)"

    def timed(threads):
        print(f"[bench] cpu baseline: oracle on {threads or 'all'} thread(s), about "
              f"{budget_s:.0f} s", file=sys.stderr, flush=True)
        prev = oracle.set_threads(threads)
        used = oracle.set_threads(0) if threads == 0 else threads
        try:
            o = oracle.Oracle(oracle.OracleConfig(D=3, eps=w.eps, kappa=w.kappa, cf=w.forch,
                                                  mask=w.mask, nu_f=w.nu_f,
                                                  nu_eff_ref=w.nu_eff_ref, b=w.b))
            t0 = time.perf_counter()
            o.step(1)
            one = time.perf_counter() - t0
            k = max(1, int(budget_s / max(one, 1e-3)) - 1)
            t0 = time.perf_counter()
            o.step(k)
            dt = time.perf_counter() - t0
        finally:
            oracle.set_threads(prev)
        return w.cells * k / dt / 1e6, used, k, dt

    all_mlups, threads, k_all, dt_all = timed(0)
    one_mlups, _, k_one, dt_one = timed(1)
    return {"value": round(all_mlups, 4), "unit": "MLUPS", "cores": threads,
            "kind": "oracle", "nproc": os.cpu_count(),
            "value_1_core": round(one_mlups, 4),
            "sample": f"FP64 oracle, {what}: {k_all} timed steps on {threads} threads "
                      f"({dt_all:.1f} s) and {k_one} on one thread ({dt_one:.1f} s), each after "
                      f"1 warm-up step"}


def copy_bandwidth(nbytes=2 << 30, reps=10):
    """Practical HBM ceiling: a streaming copy of nbytes through torch's vectorised elementwise
    kernel (b = a + 0; read + write bytes per second; it moves about 20 % more than
    Tensor.copy_'s blit kernel), the best of reps, timed with events on the current stream."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.add(a, 0.0, out=b)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return round(2 * nbytes / best / 1e9, 1)


def serving_sample(n_requests, max_steps):
    """The first n_requests of the serving stream (seed 0) in FP64, FP32 and FP16-shifted
    storage: a closed batch measures the server's capacity (requests/s), then the same
    requests arrive as a Poisson process at 1.0x that rate.  Runs stop at steady state
    (relative L2 change of v over 100 steps below 1e-7), at the rounding floor of FP32/FP16
    storage (no new minimum of that change for 30 rounds: their rounding keeps it near 1e-4
    and 1e-3), or at max_steps (censored); the FP32/FP16 velocity fields are compared with
    the FP64 ones at retirement."""
    from paper_2606_29619_amd import serving, workloads
    stream = workloads.request_stream(n_requests, 0)
    out = {"sample": f"first {n_requests} requests of the 512-request stream (seed 0), "
                     f"step cap {max_steps}, tol 1e-7 per 100 steps, floor rule "
                     f"{serving.FLOOR_CHECKS} rounds for FP32/FP16; open run at 1.0x the "
                     f"closed-batch capacity of each storage form",
           "cells_total": int(sum(int(np.prod(q["shape"])) for q in stream))}
    # progress lines every 10 s of serving (a long quiet stretch reads as a hung run)
    res = serving.serve_storages(stream, ["f64", "f32", "f16"], 1e-7, max_steps, log=sys.stderr)
    for name, entry in res.items():
        c = entry["closed"]
        print(f"[bench] serving {name}: closed {c['served_MLUPS']} MLUPS, converged "
              f"{c['converged']}, at floor {c['at_floor']}, censored {c['censored']}",
              file=sys.stderr, flush=True)
    out.update({("f16_shifted" if k == "f16" else k): v for k, v in res.items()})
    return out


def make_workload(kind, n, steps):
    """The benchmark's inputs and a one-line description of them."""
    from paper_2606_29619_amd import workloads
    if kind == "box":
        w = workloads.random_porosity_3d(n=n, seed=0, ell=16.0, steps=steps)
        desc = (f"random-porosity D3Q27 {n}^3 periodic box, seed 0, correlation length 16, "
                f"phi in (0.3,1), Kozeny-Carman K (d=2), C_F=0.55/sqrt(K), nu=0.01, b=1e-6 x")
    else:
        w = workloads.sphere_duct_3d(bump_m=8, steps=steps, drive="pressure")
        desc = ("D3Q27 768x384x384 duct, solid walls on the y and z faces and solid x faces "
                "with pressure nodes at x = 1 and 766 (inlet/outlet pressure difference 1e-4, "
                "rho = 1 +- 1.5e-4, NEEM), porous sphere of radius 96 at (192, 192, 192): eps = "
                "1 - 0.5 B_8(r^2/R^2), 1/K = B_8/5e-3, C_F=0.55/sqrt(K), nu=0.052; MLUPS count "
                "every cell, solid walls included")
    return w, desc


def measure(w, desc, storage, shift, scheme, steps, warmup, src, kind="box", n=256,
            passes="auto"):
    """Create a solver for workload w, take `warmup` untimed steps, then time `steps` steps
    (wall clock around the whole region, HIP events around every kernel class on the library's
    stream).  Returns the result fields of one benchmark row."""
    import torch
    from paper_2606_29619_amd import capi
    st = {"f32": capi.LBM_F32, "f64": capi.LBM_F64, "f16": capi.LBM_F16_SHIFTED,
          "bf16": capi.LBM_BF16_SHIFTED}[storage]
    s_bytes = 8 if storage == "f64" else 4
    sp_bytes = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[storage]
    msk = 1 if w.mask is not None else 0
    lagged = scheme == "lagged"
    solver = capi.Solver.from_workload(
        w, storage=st,
        shift=capi.LBM_SHIFT_POROUS if shift == "porous" else capi.LBM_SHIFT_WEIGHTS,
        scheme=capi.LBM_SCHEME_LAGGED if lagged else capi.LBM_SCHEME_TWO_PASS,
        passes={"auto": capi.LBM_PASSES_AUTO, "separate": capi.LBM_PASSES_SEPARATE,
                "fused": capi.LBM_PASSES_FUSED}[passes])
    N = w.cells
    label = f"{kind} {storage} {scheme}"
    print(f"[bench] {label}: created, workspace {solver.nbytes / 2**30:.2f} GiB",
          file=sys.stderr, flush=True)
    solver.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms = solver.step_timed(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stt = solver.residual()
    mlups = N * steps / wall / 1e6
    print(f"[bench] {label}: {steps} steps in {wall:.3f} s ({mlups:.0f} MLUPS); mass "
          f"{stt.mass:.9e} vmax {stt.vmax:.3e}", file=sys.stderr, flush=True)
    assert stt.nonfinite == 0
    solver.close()
    del solver
    torch.cuda.empty_cache()
    Q, D = 27, 3
    # a lagged step with wet-node boundaries runs as separate passes (moment, correction and
    # collision kernels timed apart), whose bytes are those of the two-pass kernels
    bct = getattr(w, "bc_type", None)
    separate_lagged = lagged and bct is not None and bool((np.asarray(bct) > 0).any())
    if lagged and not separate_lagged:
        kb = {"fused": lagged_bytes_per_cell(Q, D, sp_bytes, s_bytes, msk)}
        avg_ms = {"fused": kms[2] / steps}
    else:
        kb = kernel_bytes_per_cell(Q, D, sp_bytes, s_bytes, msk)
        avg_ms = {"moments": kms[0] / steps, "vcorrect": kms[1] / steps,
                  "collide": kms[2] / steps}
        if kms[1] == 0.0:
            # the correction runs inside the collision pass (k_collide_vc): it reads the
            # (rho, v^(1)) records where the separate collision reads (rho, v), the same bytes
            del avg_ms["vcorrect"], kb["vcorrect"]
            avg_ms["collide_vc"] = avg_ms.pop("collide")
            kb["collide_vc"] = kb.pop("collide")
    dom = max(avg_ms, key=avg_ms.get)
    algo = kb[dom] * N
    achieved = algo / (avg_ms[dom] * 1e-3) / 1e9
    tag = storage if sp_bytes != 2 else f"{storage}_{shift}"
    if lagged:
        tag += "_lagged"
    traffic = traffic_from_profiles(dom, tag, src, kind, n)
    step_bytes = method_bytes_per_cell(Q, D, sp_bytes, s_bytes, lagged, msk)
    return {
        "value": round(mlups, 1),
        "ms_per_step": round(wall / steps * 1e3, 4),
        "dtype": "f64" if storage == "f64" else "f32",
        "config": {"workload": desc, "lattice": "D3Q27", "cells": N,
                   "scheme": ("lagged, separate passes (wet-node boundaries)" if separate_lagged
                              else scheme if lagged or "collide" in avg_ms
                              else "two-pass, velocity correction inside the collision pass"),
                   "storage": storage if sp_bytes != 2 else f"{storage} shifted ({shift})"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": None if traffic is None else round(traffic, 0),
                     "algorithmic_bytes_per_launch": algo},
        "step_hbm": {"method_bytes_per_cell": step_bytes,
                     "effective_GBps": round(mlups * 1e6 * step_bytes / 1e9, 1),
                     "frac_of_peak": round(mlups * 1e6 * step_bytes / 1e9 / HBM_PEAK_GBPS, 4)},
        "kernels": {k: {"avg_ms": round(avg_ms[k], 4), "bytes_per_cell": kb[k],
                        "achieved_GBps": round(kb[k] * N / (avg_ms[k] * 1e-3) / 1e9, 1)}
                    for k in avg_ms},
    }


# Rows timed after the headline, each under its own configuration: the other stored forms and
# schemes of the random-porosity box, and the sphere duct at scale.
SECONDARY = [("box", "f16", "porous", "two-pass"), ("box", "bf16", "porous", "two-pass"),
             ("box", "f32", "porous", "lagged"), ("box", "f16", "porous", "lagged"),
             ("box", "f64", "porous", "two-pass"), ("sphere", "f32", "porous", "two-pass")]


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", choices=["box", "sphere"], default="box",
                    help="box: random-porosity periodic box (headline); sphere: 768x384x384 "
                         "duct with walls on the y and z faces and a smooth porous sphere")
    ap.add_argument("--n", type=int, default=256, help="cells per side of the box")
    ap.add_argument("--storage", choices=["f32", "f64", "f16", "bf16"], default="f32",
                    help="population storage; f16/bf16 are the shifted 16-bit forms (FP32 math)")
    ap.add_argument("--shift", choices=["weights", "porous"], default="porous",
                    help="shift of the 16-bit forms")
    ap.add_argument("--scheme", choices=["two-pass", "lagged"], default="two-pass",
                    help="two-pass: the method as written (headline); lagged: single fused pass "
                         "with previous-step neighbour moments")
    ap.add_argument("--passes", choices=["auto", "separate", "fused"], default="auto",
                    help="two-pass step: fused corrects the velocity inside the collision pass "
                         "where the kernel supports the run, auto does so for FP32 storage, "
                         "separate keeps the correction kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the bounded serving-stream sample")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary rows (other stored forms, schemes, the duct)")
    ap.add_argument("--secondary-steps", type=int, default=None,
                    help="timed steps of each secondary row (default: --steps within 100..200)")
    ap.add_argument("--serve-requests", type=int, default=12)
    ap.add_argument("--serve-max-steps", type=int, default=30000)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed region, run one plain device copy of this many MiB "
                         "(counter calibration for profiling runs)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only: the hot path is a single-GPU kernel and this "
              f"build has no multi-GPU path (asked for --gpus {args.gpus}, WORLD_SIZE {world}).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    src = source_hash()
    w, desc = make_workload(args.workload, args.n, args.steps)
    row = measure(w, desc, args.storage, args.shift, args.scheme, args.steps, args.warmup, src,
                  args.workload, args.n, args.passes)
    del w
    line = {
        "metric": METRIC,
        "value": row["value"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": row["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": row["dtype"],
        "data": "synthetic",
        "config": row["config"],
        "roofline": row["roofline"],
        "step_hbm": row["step_hbm"],
        "kernels": row["kernels"],
        "source_hash": src,
    }
    copy = copy_bandwidth()
    line["roofline"]["copy_GBps"] = copy
    line["roofline"]["frac_of_copy"] = round(row["roofline"]["achieved"] / copy, 4)
    if args.copy_probe_mib:
        nb = args.copy_probe_mib * 2 ** 20
        a = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = {"read": nb, "write": nb}
        del a, b
    if not args.no_secondary:
        # at least 100 timed steps after 20 warm-up steps: a row of 20 steps reads several per
        # cent low (clocks and caches still settling after the row's creation)
        steps2 = args.secondary_steps or max(100, min(args.steps, 200))
        warm2 = 20
        rows, cache = [], {}
        for kind, storage, shift, scheme in SECONDARY:
            if (kind, storage, scheme) == (args.workload, args.storage, args.scheme):
                continue
            if kind not in cache:
                cache.clear()
                cache[kind] = make_workload(kind, args.n, steps2)
            wk, dk = cache[kind]
            r = measure(wk, dk, storage, shift, scheme, steps2, warm2, src, kind, args.n)
            rows.append(dict(r, steps=steps2, warmup=warm2))
        cache.clear()
        line["secondary"] = rows
    if not args.no_serving:
        line["serving"] = serving_sample(args.serve_requests, args.serve_max_steps)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(workload=args.workload)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
