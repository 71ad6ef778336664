"""Autotuner for batched queries: picks the build parameters (branching factor,
treelet size) and the launch shape (waves per CU) that answer a batched
collision workload fastest on the current GPU.

Every candidate must give answers identical to the first one: build
parameters and launch shape change how the work is done, never what the
answer is, so a candidate whose answers differ is reported as a failure.

    python -m paper_2012_05348_amd.autotune --out tuned.json

tunes the library's batched workload (a 20k-triangle link against 64
obstacles of 1k-200k triangles); `tune()` takes any meshes and poses.
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

import numpy as np

from . import (DOP18, EARLY_EXIT, Model, Obstacles, cbvh_collide_batch, workspace)

WAVES_ENV = "CBVH_WAVES_PER_CU"


def _time_batched(link, oset, Pd, od, n, steps, warmup):
    import torch
    ws = workspace(link, link, n, EARLY_EXIT, 0, Pd.device)
    hit = torch.empty(n, dtype=torch.uint8, device=Pd.device)
    st = torch.empty(n, dtype=torch.uint8, device=Pd.device)

    def step():
        cbvh_collide_batch(link.handle, link.dev, oset.handle, Pd, od, n, EARLY_EXIT, hit, st, ws.buf)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ms = []
    for _ in range(steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        step()
        b.record()
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    return float(np.median(ms)), hit.cpu().numpy(), bool((st == 0).all().item())


def tune(link_mesh, obstacle_meshes, poses, pose_obstacle, bv=DOP18, bits=16, leaf_size=4,
         branchings=(4, 8), treelet_bytes=(2048, 8192, 32768), waves_per_cu=(0, 8), steps=5, warmup=2,
         device="cuda", log=None):
    """Time every candidate; returns {"best": {...}, "results": [...]}.
    waves_per_cu 0 means as many as fit (the library's default)."""
    import torch
    n = len(poses)
    Pd = torch.from_numpy(np.ascontiguousarray(poses, dtype=np.float32)).to(device)
    od = torch.from_numpy(np.ascontiguousarray(pose_obstacle, dtype=np.uint32)).to(device)
    results, reference = [], None
    saved = os.environ.get(WAVES_ENV)
    try:
        for bf, tb in itertools.product(branchings, treelet_bytes):
            t0 = time.perf_counter()
            kw = dict(bv=bv, branching=bf, leaf_size=leaf_size, bits=bits, treelet_bytes=tb)
            link = Model.build(*link_mesh, **kw).to(device)
            oset = Obstacles([Model.build(V, T, **kw).to(device) for V, T in obstacle_meshes], device)
            build_s = time.perf_counter() - t0
            for wpc in waves_per_cu:
                if wpc:
                    os.environ[WAVES_ENV] = str(wpc)
                else:
                    os.environ.pop(WAVES_ENV, None)
                ms, hit, ok = _time_batched(link, oset, Pd, od, n, steps, warmup)
                if reference is None:
                    reference = hit
                same = bool(np.array_equal(hit, reference)) and ok
                r = {"branching": bf, "treelet_bytes": tb, "waves_per_cu": wpc, "ms": ms,
                     "poses_per_sec": n / (ms * 1e-3), "answers_equal": same, "build_s": build_s}
                results.append(r)
                if log:
                    log(f"autotune {r}")
    finally:
        if saved is None:
            os.environ.pop(WAVES_ENV, None)
        else:
            os.environ[WAVES_ENV] = saved
    good = [r for r in results if r["answers_equal"]]
    best = min(good, key=lambda r: r["ms"]) if good else None
    return {"best": best, "results": results, "all_answers_equal": len(good) == len(results)}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=None, help="write the results as JSON here")
    ap.add_argument("--quick", action="store_true", help="branching {4, 8} and the default treelet size only")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from synth import configs
    w = configs.BATCHED
    P, obj = w.raw_poses()
    meshes_ = [w.obstacle_mesh(i) for i in range(w.n_obstacles)]
    tbs = (8192,) if args.quick else (2048, 8192, 32768)
    res = tune(w.link_mesh(), meshes_, P, obj, bits=w.bits, leaf_size=w.leaf_size, treelet_bytes=tbs,
               log=lambda m: print(m, file=sys.stderr, flush=True))
    text = json.dumps(res, indent=1)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(json.dumps(res["best"]))


if __name__ == "__main__":
    main()
