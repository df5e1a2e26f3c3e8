"""Serving stream driver: seeded porous-media requests arrive as a Poisson process and are
served by the library's request server (admission by footprint, batched rounds, retirement).

Every request follows the stream recipe of ``workloads.request_stream``: D2Q9 with sides
uniform in [64, 1024] or D3Q27 with sides uniform in [32, 192] (even odds), a random porosity
field (correlation length 16) with phi_min uniform in [0.2, 0.6], Kozeny-Carman permeability,
nu uniform in [0.005, 0.05], body force 1e-6 along x, periodic box, run until the relative L2
change of v over 100 steps falls below 1e-7 (or a step cap, reported as censored).  FP32 and
the 16-bit forms cannot reach 1e-7: rounding keeps their state changing by about 1e-4 (FP32)
or 1e-3 (FP16) of v per 100 steps about the steady state, so their runs retire when the
residual stops falling (the server's floor rule), and their velocity accuracy is stated
against the same requests served in FP64.

This module only submits at the arrival times and reads results back; admission, batching and
retirement are the library's.

    python -m paper_2606_29619_amd.serving --requests 512 --storage f64,f32,f16 --max-steps 200000
"""
import argparse
import json
import sys
import time

import numpy as np


def make_request(q):
    """The workload of one stream entry (porous field drawn from the entry's own seed)."""
    from . import workloads
    if q["lattice"] == 9:
        _, ny, nx = q["shape"]
        return workloads.random_porosity_2d(nx=nx, ny=ny, seed=q["seed"], ell=16.0,
                                            phi_min=q["phi_min"], nu=q["nu"], b=1e-6)
    return workloads.random_porosity_3d(shape=q["shape"], seed=q["seed"], ell=16.0,
                                        phi_min=q["phi_min"], nu=q["nu"], b=1e-6)


def _pct(x, p):
    return float(np.percentile(np.asarray(x), p)) if len(x) else None


# Rounds without a new minimum of the residual after which a run whose storage cannot reach the
# tolerance retires at its rounding floor (FP32 and the 16-bit forms; FP64 runs do not need it).
FLOOR_CHECKS = 30


def serve(stream, storage, rate=None, tol=1e-7, max_steps=200000, check_every=100,
          pool_bytes=None, scheme=None, log=None, cache=None, floor_checks=None,
          keep_velocity=False):
    """Serve the stream.  rate: arrivals per second (None: every request arrives at t = 0,
    a closed batch).  cache: optional dict that keeps generated workloads between calls; the
    workloads are generated before the clock starts (submission, admission, stepping and
    retirement are timed).  floor_checks: the server's floor rule (default: off for FP64,
    FLOOR_CHECKS rounds otherwise).  Latencies are measured on this process's clock from each
    request's scheduled arrival to the moment the server reports it finished.  keep_velocity:
    keep each finished run's velocity field (numpy, FP64) in its result.  Returns a summary."""
    import torch
    from . import capi
    scheme = capi.LBM_SCHEME_TWO_PASS if scheme is None else scheme
    if floor_checks is None:
        floor_checks = 0 if storage == capi.LBM_F64 else FLOOR_CHECKS
    if pool_bytes is None:
        free, _total = torch.cuda.mem_get_info()
        pool_bytes = int(free * 0.8) & ~255
    srv = capi.Server(pool_bytes=pool_bytes, check_every=check_every)
    arrivals = [0.0 if rate is None else q["arrival_time"] / rate for q in stream]
    pending = list(range(len(stream)))
    ids = {}
    results = []
    # the synthetic inputs are the clients' work, not the server's: build them before the clock
    if cache is None:
        cache = {}
    for k in pending:
        if k not in cache:
            cache[k] = make_request(stream[k])
    t0 = time.perf_counter()
    next_log = 0.0
    while pending or srv.stats().active or srv.stats().queued:
        now = time.perf_counter() - t0
        while pending and arrivals[pending[0]] <= now:
            k = pending.pop(0)
            ids[srv.submit(cache[k], storage=storage, scheme=scheme, tol=tol,
                           max_steps=max_steps, floor_checks=floor_checks)] = k
        st = srv.stats()
        if st.active == 0 and st.queued == 0:
            if pending:
                time.sleep(max(0.0, min(0.05, arrivals[pending[0]] - now)))
            continue
        for rid in srv.progress(1):
            t_seen = time.perf_counter() - t0
            info = srv.info(rid)
            k = ids[rid]
            r = {"request": k, "state": info.state, "steps": info.steps, "cells": info.cells,
                 "residual": info.residual, "t_arrival": arrivals[k], "t_done": t_seen,
                 "wait_in_queue_s": info.t_admit - info.t_submit,
                 "time_in_system": t_seen - arrivals[k]}
            if keep_velocity and info.state != capi.LBM_REQ_FAILED:
                _, v = srv.solver(rid).moments(torch.float64)
                r["v"] = v.cpu().numpy()
            results.append(r)
            srv.release(rid)
        if log and now >= next_log:
            st = srv.stats()
            print(f"[serve] t={now:7.1f}s done {len(results)}/{len(stream)} active {st.active} "
                  f"queued {st.queued} pool {st.pool_used / 2**30:.1f} GiB", file=log, flush=True)
            next_log = now + 10.0
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    conv = [r for r in results if r["state"] == capi.LBM_REQ_CONVERGED]
    flo = [r for r in results if r["state"] == capi.LBM_REQ_FLOOR]
    cens = [r for r in results if r["state"] == capi.LBM_REQ_CENSORED]
    fail = [r for r in results if r["state"] == capi.LBM_REQ_FAILED]
    steady = conv + flo
    tts = [r["time_in_system"] for r in steady]
    tis = [r["time_in_system"] for r in results]
    return {
        "requests": len(stream), "converged": len(conv), "at_floor": len(flo),
        "censored": len(cens), "failed": len(fail), "wall_s": round(wall, 3),
        "served_MLUPS": round(st.cell_updates / wall / 1e6, 1),
        "cell_updates": st.cell_updates, "rounds": st.rounds,
        "p50_time_to_steady_s": _pct(tts, 50), "p99_time_to_steady_s": _pct(tts, 99),
        "p50_steps_to_steady": _pct([r["steps"] for r in steady], 50),
        "p50_residual_at_floor": _pct([r["residual"] for r in flo], 50),
        "p50_time_in_system_s": _pct(tis, 50), "p99_time_in_system_s": _pct(tis, 99),
        "pool_bytes": pool_bytes, "pool_peak_bytes": st.pool_peak,
        "arrival_rate_per_s": rate, "tol": tol, "max_steps": max_steps,
        "check_every": check_every, "floor_checks": floor_checks,
        "results": results,
    }


def velocity_accuracy(results, reference):
    """Per request, the relative L2 and Linf error of a served velocity field against the same
    request served in FP64 (results from serve(..., keep_velocity=True)); returns the median
    and the largest of each over the requests both runs finished."""
    ref = {r["request"]: r["v"] for r in reference if "v" in r}
    l2, linf = [], []
    for r in results:
        if "v" not in r or r["request"] not in ref:
            continue
        v, v0 = r["v"], ref[r["request"]]
        d = (v - v0).ravel()
        l2.append(float(np.linalg.norm(d) / np.linalg.norm(v0.ravel())))
        linf.append(float(np.abs(d).max() / np.abs(v0).max()))
    if not l2:
        return None
    return {"requests": len(l2), "p50_v_L2": _pct(l2, 50), "max_v_L2": max(l2),
            "p50_v_Linf": _pct(linf, 50), "max_v_Linf": max(linf)}


def serve_storages(stream, names, tol, max_steps, rate=None, open_run=True, pool=None,
                   log=None):
    """Serve the stream once per storage form in names ("f64", "f32", "f16", "bf16"): a closed
    batch (its capacity sets the arrival rate unless rate is given), then the same requests as
    a Poisson stream at that rate.  With "f64" among them, the closed FP64 results are the
    reference of the others' velocity accuracy.  Returns {name: {"closed", "open",
    "velocity_vs_f64"}} without the per-request fields."""
    import torch
    from . import capi
    codes = {"f32": capi.LBM_F32, "f16": capi.LBM_F16_SHIFTED, "bf16": capi.LBM_BF16_SHIFTED,
             "f64": capi.LBM_F64}
    order = sorted(names, key=lambda n: n != "f64")      # the FP64 reference first
    cache, out, ref = {}, {}, None
    brief = lambda d: {k: v for k, v in d.items() if k != "results"}
    for name in order:
        closed = serve(stream, codes[name], None, tol, max_steps, pool_bytes=pool, log=log,
                       cache=cache, keep_velocity="f64" in names)
        entry = {"closed": brief(closed)}
        if name == "f64":
            ref = closed["results"]
        elif ref is not None:
            entry["velocity_vs_f64"] = velocity_accuracy(closed["results"], ref)
        r = rate if rate is not None else closed["requests"] / closed["wall_s"]
        if open_run:
            entry["open"] = brief(serve(stream, codes[name], r, tol, max_steps, pool_bytes=pool,
                                        log=log, cache=cache))
            entry["open"]["arrival_rate_per_s"] = round(r, 4)
        out[name] = entry
        del closed
        torch.cuda.empty_cache()
    return out


def main():
    from . import workloads
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--storage", default="f64,f32,f16",
                    help="comma-separated storage forms among f64, f32, f16, bf16")
    ap.add_argument("--max-steps", type=int, default=200000)
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--rate", type=float, default=None,
                    help="arrivals per second; default: measure the closed-batch capacity "
                         "first and arrive at 1.0x that rate")
    ap.add_argument("--closed-only", action="store_true")
    ap.add_argument("--pool-gib", type=float, default=None,
                    help="device pool for the server (default: 80%% of free memory)")
    ap.add_argument("--out", default=None, help="write the summary here")
    args = ap.parse_args()
    stream = workloads.request_stream(args.requests, args.seed)
    pool = None if args.pool_gib is None else int(args.pool_gib * 2**30) & ~255
    out = {"sample": f"first {args.requests} requests of the stream (seed {args.seed}), step cap "
                     f"{args.max_steps}, tol {args.tol} per 100 steps, floor rule "
                     f"{FLOOR_CHECKS} rounds for FP32/16-bit storage",
           "storage": serve_storages(stream, args.storage.split(","), args.tol,
                                     args.max_steps, args.rate, not args.closed_only, pool,
                                     sys.stderr)}
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(out, fh, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
