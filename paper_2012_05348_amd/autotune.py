"""Autotuner for batched queries: picks the build parameters (branching factor,
treelet size) and the launch shape (waves per CU, waves per workgroup) that
answer a batched collision workload fastest on the current GPU.

Every candidate must give answers identical to the first one: build
parameters and launch shape change how the work is done, never what the
answer is, so a candidate whose answers differ is reported as a failure.

The pick is kept in a cache file (``save`` / ``load``; default
``$CBVH_TUNE_CACHE`` or ``~/.cache/cbvh/autotune.json``, one entry per GPU
name and workload) and applied with ``build_kwargs`` (model build
parameters) and ``launch_env`` (the launch knobs, environment variables the
library reads at every launch).

    python -m paper_2012_05348_amd.autotune --out tuned.json

tunes the library's batched workload (a 20k-triangle link against 64
obstacles of 1k-200k triangles) and stores the pick in the cache; `tune()`
takes any meshes and poses.
"""
from __future__ import annotations

import argparse
import contextlib
import itertools
import json
import os
import sys
import time

import numpy as np

from . import (DOP18, EARLY_EXIT, Model, Obstacles, cbvh_collide_batch, workspace)

WAVES_ENV = "CBVH_WAVES_PER_CU"
GROUP_ENV = "CBVH_WAVES_PER_GROUP"
HELPERS_ENV = "CBVH_MAX_HELPERS"
CACHE_ENV = "CBVH_TUNE_CACHE"
WHOLE_TREE = 1 << 30  # a treelet budget no model reaches: one treelet holds the whole tree


@contextlib.contextmanager
def launch_env(cfg):
    """Launch knobs of a tuned configuration ({"waves_per_cu", "waves_per_group",
    "helpers_per_cu", "max_helpers"}; 0 or missing = the library's default)
    set for the duration of the block; cfg None leaves the environment alone.

    helpers_per_cu: waves per CU that stay, once the pose queue is empty, to
    take handed-over work (the library's default: 1 for early-exit collision,
    2 for pair lists, 4 for distances); max_helpers: the same as a count of
    waves for the whole GPU (it wins over helpers_per_cu).  Waiting helpers
    hold their CU slots, so where several launches share the GPU fewer of
    them leave more room to the other launches' waves."""
    if cfg is None:
        yield
        return
    saved = {k: os.environ.get(k) for k in (WAVES_ENV, GROUP_ENV, HELPERS_ENV)}
    try:
        for key, env in (("waves_per_cu", WAVES_ENV), ("waves_per_group", GROUP_ENV)):
            v = int((cfg or {}).get(key) or 0)
            if v:
                os.environ[env] = str(v)
            else:
                os.environ.pop(env, None)
        hp = int((cfg or {}).get("helpers_per_cu") or 0)
        mh = int((cfg or {}).get("max_helpers") or 0)
        if mh:
            os.environ[HELPERS_ENV] = str(mh)
        elif hp:
            os.environ[HELPERS_ENV] = str(hp * _cu_count())
        else:
            os.environ.pop(HELPERS_ENV, None)
        yield
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _cu_count():
    """Compute units of the current GPU (the library counts helpers in waves)."""
    import torch
    return int(torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count)


def build_kwargs(cfg, default_branching=8):
    """Model build parameters of a tuned configuration."""
    return {"branching": int((cfg or {}).get("branching") or default_branching),
            "treelet_bytes": int((cfg or {}).get("treelet_bytes") or 0)}


def cache_path(path=None):
    return path or os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "cbvh",
                                                              "autotune.json")


def _gpu_name():
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"


def save(workload, best, path=None):
    """Store the pick for (this GPU, workload) in the cache file."""
    p = cache_path(path)
    data = {}
    if os.path.exists(p):
        with open(p) as f:
            data = json.load(f)
    data[f"{_gpu_name()}|{workload}"] = best
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1)
    os.replace(tmp, p)
    return p


def load(workload, path=None):
    """The stored pick for (this GPU, workload), or None."""
    p = cache_path(path)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        return json.load(f).get(f"{_gpu_name()}|{workload}")


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
         branchings=(4, 8), treelet_bytes=(2048, 8192, 32768, WHOLE_TREE), waves_per_cu=(0, 8),
         waves_per_group=(1, 2, 4), steps=5, warmup=2, device="cuda", log=None):
    """Time every candidate; returns {"best": {...}, "results": [...]}.
    waves_per_cu 0 means as many as fit (the library's default)."""
    import torch
    n = len(poses)
    Pd = torch.from_numpy(np.ascontiguousarray(poses, dtype=np.float32)).to(device)
    od = torch.from_numpy(np.ascontiguousarray(pose_obstacle, dtype=np.uint32)).to(device)
    results, reference = [], None
    for bf, tb in itertools.product(branchings, treelet_bytes):
        t0 = time.perf_counter()
        kw = dict(bv=bv, branching=bf, leaf_size=leaf_size, bits=bits, treelet_bytes=tb)
        link = Model.build(*link_mesh, **kw).to(device)
        oset = Obstacles([Model.build(V, T, **kw).to(device) for V, T in obstacle_meshes], device)
        build_s = time.perf_counter() - t0
        for wpc, wpg in itertools.product(waves_per_cu, waves_per_group):
            cfg = {"branching": bf, "treelet_bytes": tb, "waves_per_cu": wpc, "waves_per_group": wpg}
            with launch_env(cfg):
                ms, hit, ok = _time_batched(link, oset, Pd, od, n, steps, warmup)
            if reference is None:
                reference = hit
            same = bool(np.array_equal(hit, reference)) and ok
            r = dict(cfg, ms=ms, poses_per_sec=n / (ms * 1e-3), answers_equal=same, build_s=build_s)
            results.append(r)
            if log:
                log(f"autotune {r}")
    good = [r for r in results if r["answers_equal"]]
    best = min(good, key=lambda r: r["ms"]) if good else None
    return {"best": best, "results": results, "all_answers_equal": len(good) == len(results)}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=None, help="write the results as JSON here")
    ap.add_argument("--quick", action="store_true", help="branching {4, 8} and the default treelet size only")
    ap.add_argument("--cache", default=None, help="cache file for the pick (default: $CBVH_TUNE_CACHE or "
                                                  "~/.cache/cbvh/autotune.json)")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from synth import configs
    w = configs.BATCHED
    P, obj = w.raw_poses()
    meshes_ = [w.obstacle_mesh(i) for i in range(w.n_obstacles)]
    tbs = (8192,) if args.quick else (2048, 8192, 32768, WHOLE_TREE)
    res = tune(w.link_mesh(), meshes_, P, obj, bits=w.bits, leaf_size=w.leaf_size, treelet_bytes=tbs,
               log=lambda m: print(m, file=sys.stderr, flush=True))
    text = json.dumps(res, indent=1)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    if res["best"]:
        print("stored in", save(w.name, res["best"], args.cache), file=sys.stderr)
    print(json.dumps(res["best"]))


if __name__ == "__main__":
    main()
