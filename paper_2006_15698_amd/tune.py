"""Autotuner for the per-degree tile (elements per workgroup) of the batched
multi-mesh kernels.

For every degree p = 1..5 and every tile size the library was built with
(dg_batch_tile_options), a batch of identical meshes of that degree is timed
over a few graph-replayed LSERK45 steps on the current GPU; the fastest tile
per degree is stored in tuned_tiles.json next to this file, keyed by the
device name.  Batch() loads it by default.

    python -m paper_2006_15698_amd.tune [--meshes 16] [--n 16] [--steps 4]
"""

import argparse
import json
import math
import os

import torch

from . import dg

HERE = os.path.dirname(os.path.abspath(__file__))
TUNED_PATH = os.path.join(HERE, "tuned_tiles.json")


def _uniform_state(n, p, count):
    """A smooth periodic state of every mesh; every tile is timed on the
    same state (the stage time depends a little on the data values)."""
    N = p + 1
    ar = torch.arange(n, dtype=torch.float64)
    x = (ar.view(1, 1, n, 1, 1, 1) + 0.5) / n
    base = torch.ones(n, n, n, N, N, N, dtype=torch.float64)
    rho = base * (1.0 + 0.1 * torch.sin(2 * math.pi * x))
    st = torch.stack([rho, 0.1 * rho, 0.0 * rho, 0.0 * rho, base / 0.4 + 0.005 * rho])
    return [st] * count


def time_tile(p, epb, meshes=16, n=16, steps=4, reps=3):
    b = dg.Batch([(n, n, n)] * meshes, [p] * meshes, [(1.0, 1.0, 1.0)] * meshes, tiles={p: epb})
    Q = b.pack(_uniform_state(n, p, meshes))
    res = torch.zeros_like(Q)
    b.set_dt([1e-5] * meshes)
    b.step(Q, res, nsteps=1, graph=True)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.step(Q, res, nsteps=steps, graph=True)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / steps)
    return best


def tune(meshes=16, n=16, steps=4, path=TUNED_PATH, verbose=True):
    dev = torch.cuda.get_device_name(0)
    tiles, times = {}, {}
    for p in range(1, 6):
        opts = dg.dg_batch_tile_options(p)
        t = {e: time_tile(p, e, meshes, n, steps) for e in opts}
        times[p] = t
        tiles[p] = min(t, key=t.get)
        if verbose:
            print(f"p={p}: " + ", ".join(f"epb {e}: {v:.3f} ms/step" for e, v in t.items())
                  + f" -> {tiles[p]}", flush=True)
    rec = {}
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
    rec[dev] = {"tiles": {str(k): v for k, v in tiles.items()},
                "ms_per_step": {str(k): {str(e): v for e, v in t.items()} for k, t in times.items()},
                "workload": f"{meshes} meshes of {n}^3 elements per degree, {steps} graph steps, "
                            f"the default launch form (one launch per degree)"}
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    return tiles


def load_tiles(path=TUNED_PATH):
    """Tuned {degree: tile} for the current device, or None."""
    try:
        with open(path) as f:
            rec = json.load(f)
        ent = rec.get(torch.cuda.get_device_name(0))
        if not ent:
            return None
        return {int(k): int(v) for k, v in ent["tiles"].items()}
    except (OSError, ValueError, KeyError, RuntimeError, AssertionError):
        return None


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--meshes", type=int, default=16)
    ap.add_argument("--n", type=int, default=16)
    ap.add_argument("--steps", type=int, default=4)
    a = ap.parse_args()
    print(tune(a.meshes, a.n, a.steps))
