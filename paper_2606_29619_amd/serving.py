"""Serving stream driver: seeded porous-media requests arrive as a Poisson process and are
served by the library's request server (admission by footprint, batched rounds, retirement).

Every request follows the stream recipe of ``workloads.request_stream``: D2Q9 with sides
uniform in [64, 1024] or D3Q27 with sides uniform in [32, 192] (even odds), a random porosity
field (correlation length 16) with phi_min uniform in [0.2, 0.6], Kozeny-Carman permeability,
nu uniform in [0.005, 0.05], body force 1e-6 along x, periodic box, run until the relative L2
change of v over 100 steps falls below 1e-7 (or a step cap, reported as censored).

This module only submits at the arrival times and reads results back; admission, batching and
retirement are the library's.

    python -m paper_2606_29619_amd.serving --requests 512 --storage f32 --max-steps 200000
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


def serve(stream, storage, rate=None, tol=1e-7, max_steps=200000, check_every=100,
          pool_bytes=None, scheme=None, log=None, cache=None):
    """Serve the stream.  rate: arrivals per second (None: every request arrives at t = 0,
    a closed batch).  cache: optional dict that keeps generated workloads between calls; the
    workloads are generated before the clock starts (submission, admission, stepping and
    retirement are timed).  Returns a summary dict."""
    import torch
    from . import capi
    scheme = capi.LBM_SCHEME_TWO_PASS if scheme is None else scheme
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
                           max_steps=max_steps)] = k
        st = srv.stats()
        if st.active == 0 and st.queued == 0:
            if pending:
                time.sleep(max(0.0, min(0.05, arrivals[pending[0]] - now)))
            continue
        for rid in srv.progress(1):
            info = srv.info(rid)
            results.append({"request": ids[rid], "state": info.state, "steps": info.steps,
                            "cells": info.cells, "residual": info.residual,
                            "t_submit": info.t_submit, "t_admit": info.t_admit,
                            "t_done": info.t_done,
                            "time_to_steady": info.t_done - info.t_submit})
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
    cens = [r for r in results if r["state"] == capi.LBM_REQ_CENSORED]
    fail = [r for r in results if r["state"] == capi.LBM_REQ_FAILED]
    tts = [r["time_to_steady"] for r in conv]
    tis = [r["time_to_steady"] for r in results]
    return {
        "requests": len(stream), "converged": len(conv), "censored": len(cens),
        "failed": len(fail), "wall_s": round(wall, 3),
        "served_MLUPS": round(st.cell_updates / wall / 1e6, 1),
        "cell_updates": st.cell_updates, "rounds": st.rounds,
        "p50_time_to_steady_s": _pct(tts, 50), "p99_time_to_steady_s": _pct(tts, 99),
        "p50_steps_to_steady": _pct([r["steps"] for r in conv], 50),
        "p50_time_in_system_s": _pct(tis, 50), "p99_time_in_system_s": _pct(tis, 99),
        "pool_bytes": pool_bytes, "pool_peak_bytes": st.pool_peak,
        "arrival_rate_per_s": rate, "tol": tol, "max_steps": max_steps,
        "check_every": check_every,
        "results": results,
    }


def main():
    from . import capi, workloads
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--storage", choices=["f32", "f16", "bf16", "f64"], default="f32")
    ap.add_argument("--max-steps", type=int, default=200000)
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--rate", type=float, default=None,
                    help="arrivals per second; default: measure the closed-batch capacity "
                         "first and arrive at 1.0x that rate")
    ap.add_argument("--closed-only", action="store_true")
    ap.add_argument("--pool-gib", type=float, default=None,
                    help="device pool for the server (default: 80%% of free memory)")
    ap.add_argument("--out", default=None, help="write the full summary (per request) here")
    args = ap.parse_args()
    storage = {"f32": capi.LBM_F32, "f16": capi.LBM_F16_SHIFTED, "bf16": capi.LBM_BF16_SHIFTED,
               "f64": capi.LBM_F64}[args.storage]
    stream = workloads.request_stream(args.requests, args.seed)
    out = {"storage": args.storage}
    rate = args.rate
    pool = None if args.pool_gib is None else int(args.pool_gib * 2**30) & ~255
    cache = {}
    if rate is None:
        closed = serve(stream, storage, None, args.tol, args.max_steps, pool_bytes=pool,
                       log=sys.stderr, cache=cache)
        rate = closed["requests"] / closed["wall_s"]
        out["closed"] = closed
    if not args.closed_only:
        out["open"] = serve(stream, storage, rate, args.tol, args.max_steps, pool_bytes=pool,
                            log=sys.stderr, cache=cache)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(out, fh, indent=1)
    brief = {k: {kk: vv for kk, vv in v.items() if kk != "results"} if isinstance(v, dict) else v
             for k, v in out.items()}
    print(json.dumps(brief), flush=True)


if __name__ == "__main__":
    main()
