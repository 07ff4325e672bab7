"""Autotuner for the library's kernel forms and tile shapes.

Single-volume problems (tune_conv): for each operator (forward, transpose)
it times every kernel form that can run the problem -- the small-PSF
streaming kernel, the 4x4x1 matrix-core tile with 8 or 16 x-blocks per
instruction (32x32 or 16x64 outputs per group of waves), the 32x32x16 bf16
tile with 2, 3 or 4 blocks per wave, and the general vector-ALU kernel for
small tap counts -- with HIP events on the launch stream, installs the
fastest through ndc_tile_override (every later conv_full_nd,
conv_adjoint_nd, deconv_iterate and rl_iterate of that problem uses it) and
records it in the JSON table, which apply_table() installs again in a new
process.

Batches (tune): one plan per candidate tuning -- output planes per tile (2
or 4), persistent work-groups per CU (1 or 2) and tile order (by volume,
interleaved, costliest volume first), or each volume's own kernels on the
plan's streams -- timed on two steps of the batched deconvolution, the only
call the tuning shapes (the batched operators run each volume's own kernel
whatever it is); the fastest is stored keyed by the batch's shapes, which
plan_for() reads."""
import hashlib
import json
import os

import torch

from . import _native
from .batched import BatchPlan

DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_table.json")
# the persistent tile's shapes, and (0, ...) the volumes' own kernels on the plan's streams
CANDIDATES = [(mg, wpc, order, 1) for mg in (4, 2) for wpc in (2, 1) for order in (0, 1, 2)] + [(0, 1, 0, 1)]


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


def time_plan(plan, ys, hs, xs, reps=2, iters=2):
    """Best of `reps` timings of `iters` batched deconvolution steps from the
    same start (after one call that captures the plan's graph)."""
    s = torch.cuda.current_stream()
    plan.deconv(ys, hs, [x.clone() for x in xs], iters)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        x1 = [x.clone() for x in xs]
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        plan.deconv(ys, hs, x1, iters)
        e1.record(s)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune(shapes, psf_shapes, candidates=CANDIDATES, reps=2, table=None, seed=0, forms=True):
    """Time every candidate on random data of the batch's shapes; store and
    return (best tuning, {tuning: ms}).  With forms=True each distinct
    volume problem first gets its kernel forms tuned and stored (tune_conv):
    the batched operators, and the deconvolution on the volumes' own
    kernels, run the form installed for each volume."""
    if forms:
        for shape, psf in sorted({(tuple(int(v) for v in a), tuple(int(v) for v in b))
                                  for a, b in zip(shapes, psf_shapes)}):
            tune_conv(shape, psf, table=table, seed=seed)
    g = torch.Generator(device="cuda").manual_seed(seed)
    xt = [torch.rand(s, device="cuda", generator=g) for s in shapes]
    hs = [torch.rand(h, device="cuda", generator=g) for h in psf_shapes]
    hs = [h / h.sum() for h in hs]
    xs = [torch.rand(s, device="cuda", generator=g) for s in shapes]
    times = {}
    ys = None
    for cand in candidates:
        plan = BatchPlan(shapes, psf_shapes, tuning=cand)
        if ys is None:
            ys = plan.conv_full(xt, hs)
        times[cand] = time_plan(plan, ys, hs, xs, reps)
        plan.close()
    best = min(times, key=times.get)
    save_entry(signature(shapes, psf_shapes),
               {"tuning": list(best), "ms": {",".join(map(str, k)): round(v, 4) for k, v in times.items()}},
               table)
    return best, times


def install_batch_forms(shapes, psf_shapes, table=None):
    """Install the stored kernel forms of a batch's volumes (entries that
    tune_conv wrote); returns how many operator choices were installed."""
    entries = load_table(table)
    count = 0
    for shape, psf in {(tuple(int(v) for v in a), tuple(int(v) for v in b)) for a, b in zip(shapes, psf_shapes)}:
        e = entries.get(conv_signature(shape, psf, "fp32", torch.float32))
        for op in OPS if e else ():
            try:
                set_form(shape, psf, op, e[op]["form"][0], e[op]["form"][1])
                count += 1
            except _native.NdcError:
                pass
    return count


def best_tuning(shapes, psf_shapes, table=None):
    entry = load_table(table).get(signature(shapes, psf_shapes))
    if entry:
        return tuple(entry["tuning"])
    return tune(shapes, psf_shapes, table=table)[0]


# ---------------------------------------------------------------- single volume
FORMS = {"valu": _native.NDC_FORM_VALU, "small": _native.NDC_FORM_SMALL, "mfma4": _native.NDC_FORM_MFMA4,
         "mfma32": _native.NDC_FORM_MFMA32, "slot": _native.NDC_FORM_SLOT}
FORM_NAMES = {v: k for k, v in FORMS.items()}
PRECISION_CODES = {"fp32": 0, "fp64": 0, "native": 0, "bf16": 1, "split_bf16": 2}
OPS = ("forward", "transpose")
VALU_MAX_TAPS = 729  # the general kernel is a candidate up to 9^3 taps


def conv_candidates(precision, taps):
    if PRECISION_CODES[precision] == 0:
        c = [("small", 0), ("mfma4", 8), ("mfma4", 16), ("slot", 0)]
    elif precision == "bf16":
        c = [("mfma4", 8), ("mfma32", 2), ("mfma32", 3), ("mfma32", 4), ("slot", 0)]
    else:
        c = [("mfma4", 8), ("mfma32", 2), ("mfma32", 3)]
    if taps <= VALU_MAX_TAPS:
        c.append(("valu", 0))
    return c


def conv_signature(shape, psf_shape, precision, dtype):
    return "conv:%s/%s/%s/%s" % (tuple(int(v) for v in shape), tuple(int(v) for v in psf_shape), precision,
                                 "f64" if dtype == torch.float64 else "f32")


def _problem(shape, psf_shape, precision, dtype):
    p = [(int(e) - 1) // 2 for e in psf_shape]
    return (len(shape), _native.i64_array(shape), _native.i64_array(p), 1 if dtype == torch.float64 else 0,
            PRECISION_CODES[precision])


def set_form(shape, psf_shape, op, form, param=0, precision="fp32", dtype=torch.float32):
    """Install (form, param) for one operator of one problem; form "auto"
    removes the override.  Raises NdcError if the form cannot run it."""
    n, m, p, dt, pr = _problem(shape, psf_shape, precision, dtype)
    code = _native.NDC_FORM_AUTO if form == "auto" else FORMS[form]
    _native.check(_native.lib.ndc_tile_override(n, m, p, dt, pr, OPS.index(op), code, int(param)),
                  "ndc_tile_override")


def current_form(shape, psf_shape, op, precision="fp32", dtype=torch.float32):
    import ctypes
    n, m, p, dt, pr = _problem(shape, psf_shape, precision, dtype)
    out = (ctypes.c_int * 2)()
    _native.check(_native.lib.ndc_tile_choice(n, m, p, dt, pr, OPS.index(op), out), "ndc_tile_choice")
    return FORM_NAMES[out[0]], int(out[1])


def _time_op(nd, op, x, h, y, r, g, precision, reps):
    s = torch.cuda.current_stream()
    run = (lambda: nd.conv_full_nd(x, h, Y=y, precision=precision)) if op == "forward" else \
        (lambda: nd.conv_adjoint_nd(r, h, X=g, precision=precision))
    run()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        run()
        e1.record(s)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune_conv(shape, psf_shape, precision="fp32", dtype=torch.float32, reps=3, table=None, seed=0, save=True,
              x=None, h=None, r=None):
    """Time every candidate form of both operators of one problem, install
    the fastest of each and (save=True) store them.  x (X-shaped), h (the
    PSF) and r (Y-shaped, the transpose's input) are the data to time on:
    the matrix-core tiles' speed depends on the values (their bit patterns
    change the units' power draw and so the clock), so a workload's own
    operands give its own ranking; missing ones are drawn uniformly at
    random.  Returns {op: ((form, param), {"form/param": ms})}."""
    import paper_1711_11224_amd as nd
    gen = torch.Generator(device="cuda").manual_seed(seed)
    shape, psf_shape = [int(v) for v in shape], [int(v) for v in psf_shape]
    yshape = [a + b - 1 for a, b in zip(shape, psf_shape)]
    x = x if x is not None else torch.rand(shape, device="cuda", generator=gen, dtype=dtype)
    h = h if h is not None else torch.rand(psf_shape, device="cuda", generator=gen, dtype=dtype)
    y = torch.empty(yshape, device="cuda", dtype=dtype)
    r = r if r is not None else torch.rand(yshape, device="cuda", generator=gen, dtype=dtype)
    g = torch.empty(shape, device="cuda", dtype=dtype)
    taps = 1
    for v in psf_shape:
        taps *= v
    result = {}
    for op in OPS:
        times = {}
        for form, param in conv_candidates(precision, taps):
            try:
                set_form(shape, psf_shape, op, form, param, precision, dtype)
            except _native.NdcError:
                continue  # this form cannot run the problem
            times[(form, param)] = _time_op(nd, op, x, h, y, r, g, precision, reps)
        best = min(times, key=times.get)
        set_form(shape, psf_shape, op, best[0], best[1], precision, dtype)
        result[op] = (best, {"%s/%d" % k: round(v, 4) for k, v in times.items()})
    if save:
        save_entry(conv_signature(shape, psf_shape, precision, dtype),
                   {"shape": shape, "psf_shape": psf_shape, "precision": precision,
                    "dtype": "f64" if dtype == torch.float64 else "f32",
                    **{op: {"form": list(result[op][0]), "ms": result[op][1]} for op in OPS}}, table)
    return result


def apply_table(table=None):
    """Install every single-volume entry of the table; returns how many
    operator choices were installed (entries whose form cannot run are
    skipped)."""
    count = 0
    for key, e in load_table(table).items():
        if not key.startswith("conv:"):
            continue
        dtype = torch.float64 if e.get("dtype") == "f64" else torch.float32
        for op in OPS:
            form, param = e[op]["form"]
            try:
                set_form(e["shape"], e["psf_shape"], op, form, param, e["precision"], dtype)
                count += 1
            except _native.NdcError:
                pass
    return count
