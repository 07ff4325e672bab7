"""Autotuner for the batched persistent launches.

For a batch (list of X extents and PSF extents) it builds one plan per
candidate tuning -- output planes per tile (2 or 4), persistent work-groups
per CU (1 or 2) and tile order (by volume, interleaved, costliest volume
first) -- times one forward plus one transpose launch of each with HIP events
on the launch stream, and keeps the fastest.  Results persist in a JSON table
keyed by the batch's shapes, which plan_for() reads."""
import hashlib
import json
import os

import torch

from .batched import BatchPlan

DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_table.json")
CANDIDATES = [(mg, wpc, order, 1) for mg in (4, 2) for wpc in (2, 1) for order in (0, 1, 2)]


def signature(shapes, psf_shapes):
    key = ";".join("%s/%s" % (tuple(s), tuple(h)) for s, h in zip(shapes, psf_shapes))
    return hashlib.sha1(key.encode()).hexdigest()


def load_table(table=None):
    path = table or DEFAULT_TABLE
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_entry(sig, entry, table=None):
    path = table or DEFAULT_TABLE
    data = load_table(path)
    data[sig] = entry
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_plan(plan, xs, hs, reps=2):
    s = torch.cuda.current_stream()
    ys = plan.conv_full(xs, hs)
    plan.conv_adjoint(ys, hs, xs=[torch.empty_like(x) for x in xs])
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        plan.conv_full(xs, hs, ys=ys)
        plan.conv_adjoint(ys, hs)
        e1.record(s)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune(shapes, psf_shapes, candidates=CANDIDATES, reps=2, table=None, seed=0):
    """Time every candidate on random data of the batch's shapes; store and
    return (best tuning, {tuning: ms})."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    xs = [torch.rand(s, device="cuda", generator=g) for s in shapes]
    hs = [torch.rand(h, device="cuda", generator=g) for h in psf_shapes]
    times = {}
    for cand in candidates:
        plan = BatchPlan(shapes, psf_shapes, tuning=cand)
        times[cand] = time_plan(plan, xs, hs, reps)
        plan.close()
    best = min(times, key=times.get)
    save_entry(signature(shapes, psf_shapes),
               {"tuning": list(best), "ms": {",".join(map(str, k)): round(v, 4) for k, v in times.items()}},
               table)
    return best, times


def best_tuning(shapes, psf_shapes, table=None):
    entry = load_table(table).get(signature(shapes, psf_shapes))
    if entry:
        return tuple(entry["tuning"])
    return tune(shapes, psf_shapes, table=table)[0]
