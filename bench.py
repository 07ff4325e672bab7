"""Benchmark of the deconvolution hot path on one MI355X.

Workload: a synthetic 128x512x512 (z, y, x) microscopy-like volume (8000
points, 400 filaments), Gaussian PSF 63x31x31 (sigma_z 9, sigma_xy 3),
Y = X (x) H plus Poisson (peak 500) and N(0, 2^2) read noise, FP32, lambda 0.

One step = one projected-gradient iteration: transpose of the residual with
the fused gradient/projection epilogue, forward convolution of the trial with
the fused residual/objective epilogue, the device-side acceptance decision
and the commit.  Algorithmic work per step: 2 N K multiply-adds (N = 33.5M
voxels, K = 60543 taps), zero-padding products not counted.

Prints one JSON line: the metric and value (multiply-adds per second of whole
steps), the roofline of the dominant kernel (its launch time, TFLOP/s against
the FP32 matrix peak and its HBM bytes from rocprofv3 counters), each precision
form, the CPU oracle's rate on a bounded sample with each form's error on it,
and the other workloads (step rules, 2-D, small PSFs, differentiable, batched).
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3, "bf16": 2500.0, "split_bf16": 2500.0 / 3.0, "hbm": 8000.0}
# the files the FP32 matrix-core tile is compiled from (its HBM counters stay
# valid while these are unchanged)
TILE_SOURCES = ["paper_1711_11224_amd/csrc/conv_mfma.hip", "paper_1711_11224_amd/csrc/mfma_tile.h",
                "paper_1711_11224_amd/csrc/ndc_device.h", "paper_1711_11224_amd/csrc/ndc_internal.h",
                "include/ndconv.h"]


EXTRA_LEGS = ("step_rules", "richardson_lucy", "paper_2d", "small_psf", "differentiable", "refinement", "batched")
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "hbm_traffic_conv_128x512x512_psf63x31x31.json")
TILE_KERNEL = "void ndc::conv_mfma_kernel<31, 0, 8>"


def tile_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for p in TILE_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()


def kernel_key_name(name):
    """rocprofv3's demangled name without the argument list and anonymous
    namespaces: 'void ndc::conv_mfma_kernel<31, 0, 8>'."""
    name = name.replace("(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(name):  # cut at the '(' that opens the argument list
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0 and i > 0:
            return name[:i]
    return name


def read_counter_csv(path, counter):
    """Per-dispatch values of one counter from a rocprofv3 --pmc CSV:
    [(kernel name, grid size, value summed over the dispatch's rows,
    duration in ns)]."""
    import csv
    per = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            key = row["Dispatch_Id"]
            name, grid = kernel_key_name(row["Kernel_Name"]), int(row["Grid_Size"])
            dur = int(row["End_Timestamp"]) - int(row["Start_Timestamp"]) if row.get("End_Timestamp") else 0
            v = per.get(key, (name, grid, 0.0, dur))
            per[key] = (name, grid, v[2] + float(row["Counter_Value"]), dur)
    return list(per.values())


def write_traffic_record(fetch_csv, write_csv):
    """The FP32 tile's HBM bytes per launch from the FETCH_SIZE and WRITE_SIZE
    passes (KiB per dispatch), each scaled by what the same counter reads for
    the 1 GiB calibration copy (the largest copyBuffer dispatch), keyed by the
    hash of the tile's sources so that bench.py drops them once those change."""
    rec = {"csrc_sha256": tile_sources_sha256(), "kernels": {}}
    for csv_path, counter, key in ((fetch_csv, "FETCH_SIZE", "fetch"), (write_csv, "WRITE_SIZE", "write")):
        rows = read_counter_csv(csv_path, counter)
        copies = [v for n, g, v, t in rows if "copyBuffer" in n]
        if not copies:
            raise SystemExit("no calibration copy in %s (run with --copy-calibration 1024)" % csv_path)
        scale = 1048576.0 / max(copies)
        rec["%s_scale" % key] = scale
        # launches that did the work: a deconvolution call's trial slots after
        # the run has stopped return at once (under a fifth of the longest)
        longest = {}
        for n, g, v, t in rows:
            longest[(n, g)] = max(longest.get((n, g), 0), t)
        acc = {}
        for n, g, v, t in rows:
            if n == TILE_KERNEL and t >= 0.2 * longest[(n, g)]:
                acc.setdefault("%s/%d" % (n, g), []).append(v)
        for k, vals in acc.items():
            kib = float(np.mean(vals))
            d = rec["kernels"].setdefault(k, {})
            d["%s_kib" % key] = kib
            d["read_bytes" if key == "fetch" else "write_bytes"] = kib * 1024.0 * scale
    with open(TRAFFIC_RECORD, "w") as f:
        json.dump(rec, f, indent=1)
    log("wrote", TRAFFIC_RECORD)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def make_inputs(nd, torch, cfg, dev):
    import synth
    t = time.time()
    x_true = synth.make_objects(cfg)
    h = synth.psf_for(cfg).astype(np.float32)
    xg = torch.from_numpy(x_true.astype(np.float32)).to(dev)
    hg = torch.from_numpy(h).to(dev)
    blurred = nd.conv_full_nd(xg, hg).cpu().numpy()
    y = synth.add_noise(blurred, cfg).astype(np.float32)
    x0 = synth.flat_start(y, h, cfg.shape).astype(np.float32)
    log("inputs ready in %.1fs" % (time.time() - t))
    return (torch.from_numpy(y).to(dev), hg, torch.from_numpy(x0).to(dev))


def time_pairs(nd, torch, x, h, precision, reps):
    """Average duration of each operator launch, HIP events on the stream the
    library launches on (torch's current stream)."""
    s = torch.cuda.current_stream()
    y = nd.conv_full_nd(x, h, precision=precision)
    g = nd.conv_adjoint_nd(y, h, precision=precision)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b, c in ev:
        a.record(s)
        nd.conv_full_nd(x, h, Y=y, precision=precision)
        b.record(s)
        nd.conv_adjoint_nd(y, h, X=g, precision=precision)
        c.record(s)
    torch.cuda.synchronize()
    fwd = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    adj = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    return fwd, adj


def measured_traffic(kernel_key, forward=True):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    record (written by --traffic-record), or None when the kernel's sources
    (TILE_SOURCES) changed since the counters were taken.
    Both operators may run the same kernel instantiation; the forward launch
    is the one with the larger grid (its output extent m+2p exceeds m)."""
    try:
        rec = json.load(open(TRAFFIC_RECORD))
    except (OSError, ValueError):
        return None
    k = sorted((int(key.split("/")[1]), v) for key, v in rec.get("kernels", {}).items()
               if key.split("/")[0] == kernel_key)
    if rec.get("csrc_sha256") != tile_sources_sha256() or not k or len(k) > 2:
        return None
    k = k[-1][1] if forward else k[0][1]
    return int(k["read_bytes"] + k["write_bytes"])


def bench_differentiable(nd, torch, reps=3):
    """Differentiable workload (X 64x256x256, PSF 41x21x21): one forward and
    the hand-written backward (dX by the transpose, dH by the PSF-gradient
    kernel), 3 N K multiply-adds per pass."""
    import synth
    from paper_1711_11224_amd.autograd import conv_full_ad
    cfg = synth.CONFIGS["c5_diff"]
    g = torch.Generator(device="cuda").manual_seed(4)
    x = torch.rand(cfg.shape, device="cuda", generator=g).requires_grad_(True)
    h = torch.tensor(synth.psf_for(cfg), dtype=torch.float32, device="cuda").requires_grad_(True)
    gy = torch.randn([a + b - 1 for a, b in zip(cfg.shape, cfg.psf_shape)], device="cuda", generator=g)
    N, K = int(np.prod(cfg.shape)), int(np.prod(cfg.psf_shape))

    def one():
        x.grad = None
        h.grad = None
        conv_full_ad(x, h).backward(gy)

    one()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        one()
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    # the PSF-gradient kernel alone
    y = nd.conv_full_nd(x.detach(), h.detach())
    e0.record(s)
    for _ in range(reps):
        nd.conv_dH_nd(x.detach(), gy, cfg.psf_shape)
    e1.record(s)
    torch.cuda.synchronize()
    dh_ms = e0.elapsed_time(e1) / reps
    # the plain FP32 operators on the same tensors (forward + transpose, no autograd)
    fwd_ms, adj_ms = time_pairs(nd, torch, x.detach(), h.detach(), "fp32", reps)
    del y
    return {"workload": "X 64x256x256, PSF 41x21x21, FP32", "forward_backward_ms": round(ms, 3),
            "gmacs": round(3.0 * N * K / (ms * 1e-3) / 1e9, 1), "dH_ms": round(dh_ms, 3),
            "dH_gmacs": round(N * K / (dh_ms * 1e-3) / 1e9, 1),
            "plain_forward_plus_transpose_ms": round(fwd_ms + adj_ms, 3)}


def bench_joint_refinement(nd, torch, steps=20, sigma_steps=60):
    """Differentiable workload end to end: Y = X (x) H(6, 2.5, 2.5) plus
    noise (the library's forward), then `steps` joint X / sigma steps from
    the flat start and the guess (5, 2, 2) (JointRefiner: one forward, the
    dX / dH backward, a projected X step and an Adam step on log sigma), and
    `sigma_steps` sigma-only steps with X known, where sigma is identifiable."""
    import synth
    from paper_1711_11224_amd.autograd import GaussianPSF, JointRefiner, conv_full_ad
    cfg = synth.CONFIGS["c5_diff"]
    xt = torch.tensor(synth.make_objects(cfg), dtype=torch.float32, device="cuda")
    h = torch.tensor(synth.psf_for(cfg), dtype=torch.float32, device="cuda")
    b = nd.conv_full_nd(xt, h).cpu().numpy()
    y = torch.from_numpy(synth.add_noise(b, cfg).astype(np.float32)).cuda()
    xt = xt * float(cfg.peak_photons / b.max())  # the object in Y's photon units
    guess = tuple(cfg.extra["guess_sigmas"])
    x0 = torch.from_numpy(synth.flat_start(y.cpu().numpy(), synth.psf_for(cfg), cfg.shape).astype(np.float32)).cuda()
    model = GaussianPSF(cfg.psf_shape, guess)
    ref = JointRefiner(y, x0, model, lr=0.02)
    first = float(ref.step())  # warm-up
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        last = ref.step()
    e1.record(s)
    torch.cuda.synchronize()
    joint_ms = e0.elapsed_time(e1) / steps
    sig_joint = [round(float(v), 3) for v in model.sigmas().detach().cpu()]
    m2 = GaussianPSF(cfg.psf_shape, guess)
    opt = torch.optim.Adam(m2.parameters(), lr=0.03)
    for _ in range(sigma_steps):
        opt.zero_grad()
        loss = 0.5 * ((conv_full_ad(xt, m2()) - y) ** 2).sum()
        loss.backward()
        opt.step()
    sig_known = m2.sigmas().detach().cpu().numpy()
    true = np.array(cfg.sigmas)
    err0 = float(np.abs(np.array(guess) - true).max())
    N, K = int(np.prod(cfg.shape)), int(np.prod(cfg.psf_shape))
    return {"joint_steps": steps, "joint_ms_per_step": round(joint_ms, 3),
            "joint_gmacs": round(3.0 * N * K / (joint_ms * 1e-3) / 1e9, 1),
            "joint_loss_first_last": [first, float(last)], "joint_sigmas": sig_joint,
            "known_x_sigma_steps": sigma_steps, "known_x_sigmas": [round(float(v), 3) for v in sig_known],
            "known_x_sigma_error_first_last": [round(err0, 3), round(float(np.abs(sig_known - true).max()), 4)],
            "true_sigmas": list(cfg.sigmas), "guess_sigmas": list(guess)}


def bench_batched(nd, torch, steps=None, table=None):
    """Batched workload: 64 volumes of 32^3 .. 96x160x160, each with its own
    Gaussian PSF of odd extents 9..31, FP32, one hipGraph-captured step per
    iteration, tuning from the autotuner's table; one call runs the
    workload's own iteration count (50) unless `steps` is given."""
    import synth
    from paper_1711_11224_amd.batched import plan_for
    cfgs = synth.batched_configs(64)
    steps = steps or cfgs[0].iters
    shapes, psfs = [c.shape for c in cfgs], [c.psf_shape for c in cfgs]
    t = time.time()
    plan = plan_for(shapes, psfs, tuning="auto", table=table)
    tune_s = time.time() - t
    ys, hs, xs = [], [], []
    for c in cfgs:
        xt = torch.tensor(synth.make_objects(c), dtype=torch.float32, device="cuda")
        h = torch.tensor(synth.psf_for(c), dtype=torch.float32, device="cuda")
        y = synth.add_noise(nd.conv_full_nd(xt, h).cpu().numpy(), c).astype(np.float32)
        ys.append(torch.from_numpy(y).cuda())
        hs.append(h)
        xs.append(torch.from_numpy(synth.flat_start(y, synth.psf_for(c), c.shape).astype(np.float32)).cuda())
    macs = 2.0 * sum(int(np.prod(c.shape)) * int(np.prod(c.psf_shape)) for c in cfgs)
    plan.deconv(ys, hs, xs, 1)  # warm-up (captures the graph)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    _, stats, info = plan.deconv(ys, hs, xs, steps)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    done = int(info[:, 0].min())
    pair_ms = time_plan_pair(plan, torch, xs, hs)
    plan.close()
    # the plain FP32 path on the same volumes: one single-volume call per volume
    x1 = [x.clone() for x in xs]
    for v in range(len(cfgs)):  # warm-up (plans, workspaces)
        nd.deconv_iterate(ys[v], hs[v], x1[v], 1)
    torch.cuda.synchronize()
    x1 = [x.clone() for x in xs]
    e0.record(s)
    for v in range(len(cfgs)):
        nd.deconv_iterate(ys[v], hs[v], x1[v], steps)
    e1.record(s)
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1)
    y1 = [nd.conv_full_nd(xs[v], hs[v]) for v in range(len(cfgs))]
    g1 = [nd.conv_adjoint_nd(y1[v], hs[v]) for v in range(len(cfgs))]
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(3):
        for v in range(len(cfgs)):
            nd.conv_full_nd(xs[v], hs[v], Y=y1[v])
            nd.conv_adjoint_nd(y1[v], hs[v], X=g1[v])
    e1.record(s)
    torch.cuda.synchronize()
    seq_pair_ms = e0.elapsed_time(e1) / 3
    return {"workload": "64 volumes 32^3..96x160x160, PSFs 9..31 per axis, FP32", "tuning": list(plan.tuning),
            "tune_or_lookup_s": round(tune_s, 2), "steps": steps, "steps_accepted_min": done,
            "ms_per_step": round(ms / steps, 3), "iters_per_s": round(steps / (ms * 1e-3), 2),
            "gmacs": round(macs * done / (ms * 1e-3) / 1e9, 1),
            "conv_pair_ms": round(pair_ms, 3), "conv_pair_gmacs": round(macs / (pair_ms * 1e-3) / 1e9, 1),
            "single_volume_calls": {"ms_per_step": round(seq_ms / steps, 3),
                                    "conv_pair_ms": round(seq_pair_ms, 3),
                                    "step_speedup_of_batched": round(seq_ms / ms, 2),
                                    "pair_speedup_of_batched": round(seq_pair_ms / pair_ms, 2)}}


def time_plan_pair(plan, torch, xs, hs, reps=3):
    ys = plan.conv_full(xs, hs)
    gs = plan.conv_adjoint(ys, hs)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        plan.conv_full(xs, hs, ys=ys)
        plan.conv_adjoint(ys, hs, xs=gs)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def deconv_rate(nd, torch, y, h, x0, precision, steps):
    """Deconvolution iterations per second in one precision form: one call of
    `steps` iterations from X^0 (after a 1-step warm-up call), HIP events on
    the launching stream; the objective reached is reported beside it."""
    if steps <= 0:
        return {}
    nbytes = nd.deconv_workspace_bytes(list(x0.shape), list(h.shape), torch.float32, precision)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=x0.device)
    nd.deconv_iterate(y, h, x0.clone(), 1, precision=precision, ws=ws)
    x = x0.clone()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    _, st, info = nd.deconv_iterate(y, h, x, steps, precision=precision, ws=ws)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    done = int(info.cpu()[0])
    f = st.cpu().numpy()[: done + 1, 0]
    del ws
    return {"deconv_steps": done, "iters_per_s": round(done / (ms * 1e-3), 3),
            "ms_per_iter": round(ms / max(done, 1), 3), "f_after_steps": float(f[-1])}


def bench_rl(nd, torch, y, h, x0, steps=10):
    """Richardson-Lucy on the metric workload (Y clipped at 0: the method
    needs non-negative data), `steps` iterations in one call: one forward
    and one transpose per iteration, 2 N K multiply-adds."""
    yp = torch.clamp(y, min=0)
    nd.rl_iterate(yp, h, x0.clone(), 1)
    x = x0.clone()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    _, st, info = nd.rl_iterate(yp, h, x, steps)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    d = st.cpu().numpy()
    N, K = x0.numel(), h.numel()
    return {"steps": steps, "ms_per_iter": round(ms / steps, 3), "iters_per_s": round(steps / (ms * 1e-3), 3),
            "gmacs": round(2.0 * N * K * steps / (ms * 1e-3) / 1e9, 1),
            "divergence_first_last": [float(d[0]), float(d[-1])]}


def bench_step_rules(nd, torch, y, h, x0, ws, steps=10, fixed_max=60):
    """First-trial rules of the projected-gradient iteration on the metric
    workload: time per step, objective after `steps` steps, and how many steps
    the fixed first trial needs to reach that objective."""
    def run(rule, n):
        x = x0.clone()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        _, st, info = nd.deconv_iterate(y, h, x, n, ws=ws, rule=rule)
        e1.record(s)
        torch.cuda.synchronize()
        done = int(info.cpu()[0])
        return e0.elapsed_time(e1), st.cpu().numpy()[: done + 1, 0], done
    ms_f, f_fixed, done_f = run("fixed", fixed_max)
    out = {"steps": steps, "fixed": {"ms_per_step": round(ms_f / max(done_f, 1), 3),
                                     "f_after_steps": float(f_fixed[min(steps, done_f)])}}
    # the Laplacian (Tikhonov-Miller) term: extra small-PSF convolutions per step
    x = x0.clone()
    nbytes = nd.deconv_workspace_bytes_ex(list(x0.shape), list(h.shape), torch.float32, "native", 1)
    ws_tm = torch.empty(nbytes, dtype=torch.uint8, device=x0.device)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    _, st, info = nd.deconv_iterate(y, h, x, steps, ws=ws_tm, mu=1e-3)
    e1.record()
    torch.cuda.synchronize()
    out["fixed_laplacian_mu1e-3"] = {"ms_per_step": round(e0.elapsed_time(e1) / max(int(info.cpu()[0]), 1), 3),
                                     "workspace_GB": round(nbytes / 1e9, 3)}
    del ws_tm
    for rule in ("cauchy", "bb"):
        ms, f, done = run(rule, steps)
        target = f[-1]
        reach = [k for k in range(len(f_fixed)) if f_fixed[k] <= target]
        out[rule] = {"ms_per_step": round(ms / max(done, 1), 3), "f_after_steps": float(target),
                     "steps_done": done,
                     "fixed_steps_to_match": reach[0] if reach else ">%d" % fixed_max}
    return out


def bench_paper_2d(nd, torch, iters=100):
    """The paper's two 2-D experiment shapes on synthetic stand-ins (a 512x512
    crossing-lines phantom with a 9x9 PSF, noise std 5; a 225x225 8-bit image
    with a 5x5 PSF, noise std 20 and 5): `iters` iterations from the blurred
    start max(crop(Y), 0) with each first-trial rule; time per iteration and
    SNR = 10 log10(||X||^2/||X_est - X||^2) before and after."""
    import synth
    out = {}
    for name, w in synth.PAPER_2D.items():
        x = w["object"]()
        h = synth.gaussian_psf(w["psf"], w["sigma"])
        b = nd.conv_full(torch.from_numpy(x.astype(np.float32)).cuda(),
                         torch.from_numpy(h.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
        p = [(e - 1) // 2 for e in w["psf"]]
        for std in w["noise"]:
            y = synth.gaussian_noise(b, std, seed=11)
            x0 = np.maximum(y[p[0]:p[0] + x.shape[0], p[1]:p[1] + x.shape[1]], 0.0)
            yg = torch.from_numpy(y.astype(np.float32)).cuda()
            hg = torch.from_numpy(h.astype(np.float32)).cuda()
            snr = lambda e: round(float(10 * np.log10(np.sum(x * x) / np.sum((np.asarray(e, np.float64) - x) ** 2))), 3)
            rec = {"shape": list(x.shape), "psf": list(w["psf"]), "noise_std": std, "snr_blurred_db": snr(x0)}
            for rule in ("fixed", "bb"):
                xg = torch.from_numpy(x0.astype(np.float32)).cuda()
                nd.deconv_iterate(yg, hg, xg.clone(), 2, rule=rule)  # warm-up
                torch.cuda.synchronize()
                s = torch.cuda.current_stream()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s)
                _, st, info = nd.deconv_iterate(yg, hg, xg, iters, rule=rule)
                e1.record(s)
                torch.cuda.synchronize()
                rec[rule] = {"ms_per_iter": round(e0.elapsed_time(e1) / iters, 4),
                             "snr_db": snr(xg.cpu().numpy()), "iters_done": int(info.cpu()[0])}
            # Richardson-Lucy (the paper's comparison method) on max(Y, 0), from the flat start
            yp = torch.clamp(yg, min=0)
            xr = torch.from_numpy(synth.flat_start(np.maximum(y, 0), h, x.shape).astype(np.float32)).cuda()
            nd.rl_iterate(yp, hg, xr.clone(), 2)  # warm-up
            torch.cuda.synchronize()
            e0.record(s)
            _, st, info = nd.rl_iterate(yp, hg, xr, iters)
            e1.record(s)
            torch.cuda.synchronize()
            rec["rl"] = {"ms_per_iter": round(e0.elapsed_time(e1) / iters, 4), "snr_db": snr(xr.cpu().numpy()),
                         "iters_done": int(info.cpu()[0])}
            out["%s_std%g" % (name, std)] = rec
    return out


def bench_small_psf(nd, torch, reps=5):
    """Small-PSF sweep on the metric volume (128x512x512), Gaussian PSFs 3^3,
    5^3, 7^3, reported as algorithmic GB/s (4 (N + N_Y) bytes per operator:
    read one side, write the other) against 8 TB/s, and as 2 N K FLOP per
    operator against the 157.3 TFLOP/s FP32 vector peak; `bound` names the
    larger of the two floors (HBM at 3^3, the vector ALUs from 5^3 on)."""
    import synth
    m = synth.CONFIGS["c3_metric"].shape
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.rand(m, device="cuda", generator=g)
    out = {}
    for k, sig in synth.SWEEP_PSFS.items():
        h = torch.tensor(synth.gaussian_psf((k, k, k), sig), dtype=torch.float32, device="cuda")
        fwd, adj = time_pairs(nd, torch, x, h, "fp32", reps)
        N = int(np.prod(m))
        NY = int(np.prod([a + k - 1 for a in m]))
        by = 4.0 * (N + NY)
        out["%d^3" % k] = {"forward_ms": round(fwd, 4), "transpose_ms": round(adj, 4),
                           "forward_GBps": round(by / (fwd * 1e-3) / 1e9, 1),
                           "transpose_GBps": round(by / (adj * 1e-3) / 1e9, 1),
                           "forward_hbm_frac": round(by / (fwd * 1e-3) / 8e12, 3),
                           "transpose_hbm_frac": round(by / (adj * 1e-3) / 8e12, 3),
                           # the slower operator bounds a step, as in the main roofline
                           "hbm_frac": round(by / (max(fwd, adj) * 1e-3) / 8e12, 3),
                           "gmacs": round(2.0 * N * k ** 3 / ((fwd + adj) * 1e-3) / 1e9, 1),
                           "bound": "hbm" if by / 8e12 >= 2.0 * N * k ** 3 / 157.3e12 else "alu",
                           "alu_frac": round(2.0 * N * k ** 3 / 157.3e12 / (max(fwd, adj) * 1e-3), 3)}
    return out


def cpu_baseline(cfg, nd=None, torch=None, target_s=15.0):
    """The FP64 oracle, as it stands, on a bounded random sample of forward
    and transpose outputs of the same workload (each output is a full
    K-tap sum).  With the library at hand, the same sampled outputs of the
    GPU operators in each precision are compared with the oracle's (relative
    L2 error; inputs are FP32 values on both sides)."""
    import oracle
    import synth
    rng = np.random.default_rng(99)
    m, ks = cfg.shape, cfg.psf_shape
    p = [(k - 1) // 2 for k in ks]
    x = rng.random(m).astype(np.float32).astype(np.float64)
    h = synth.psf_for(cfg).astype(np.float32).astype(np.float64)
    r = rng.standard_normal([a + 2 * b for a, b in zip(m, p)]).astype(np.float32).astype(np.float64)
    K = int(np.prod(ks))
    nthreads = oracle.threads()
    # interior forward outputs (every tap in range) and any transpose output
    def interior(cnt):
        idx = [rng.integers(2 * q, a, size=cnt) for a, q in zip(m, p)]
        return np.ravel_multi_index(idx, [a + 2 * b for a, b in zip(m, p)])
    n = 64
    while True:
        t0 = time.time()
        i_f, i_a = interior(n), rng.integers(0, int(np.prod(m)), size=n)
        y_f = oracle.conv_full_at(x, h, i_f)
        g_a = oracle.conv_adjoint_at(r, h, i_a)
        dt = time.time() - t0
        if dt >= target_s or n >= 1 << 22:
            break
        n = int(n * min(8.0, max(2.0, 1.2 * target_s / max(dt, 1e-3))))
    macs = 2.0 * n * K
    out = {"value": macs / dt / 1e9, "unit": "GMAC/s", "cores": nthreads, "kind": "oracle",
           "sample": "%d forward + %d transpose outputs of the 128x512x512 / 63x31x31 workload, %d taps each, "
                     "FP64 (%.1f s on %s)" % (n, n, K, dt, cpu_model())}
    if nd is not None:
        def rel(a, b):
            return float(np.linalg.norm(a - b) / np.linalg.norm(b))
        xt = torch.from_numpy(x.astype(np.float32)).cuda()
        ht = torch.from_numpy(h.astype(np.float32)).cuda()
        rt = torch.from_numpy(r.astype(np.float32)).cuda()
        tf, ta = torch.from_numpy(i_f).cuda(), torch.from_numpy(i_a).cuda()
        acc = {}
        for pr in ("fp32", "bf16", "split_bf16"):
            yg = nd.conv_full_nd(xt, ht, precision=pr).view(-1)[tf].double().cpu().numpy()
            gg = nd.conv_adjoint_nd(rt, ht, precision=pr).view(-1)[ta].double().cpu().numpy()
            acc[pr] = {"forward": float("%.3g" % rel(yg, y_f)), "transpose": float("%.3g" % rel(gg, g_a))}
        out["accuracy_vs_oracle"] = acc
        out["accuracy_sample"] = "the same %d forward and %d transpose outputs, relative L2 error" % (n, n)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100,
                    help="timed iterations, in one call (the metric workload runs 100)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "split_bf16"])
    ap.add_argument("--pair-reps", type=int, default=5)
    ap.add_argument("--precision-steps", type=int, default=10,
                    help="deconvolution iterations timed in each precision form (0: operators only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precisions", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the differentiable and batched workloads")
    ap.add_argument("--tuning-table", default=None, help="autotuner table (default: the package's)")
    ap.add_argument("--retune", action="store_true",
                    help="time every kernel form of the workload's two operators in each precision and store the "
                         "fastest in the tuning table (otherwise the table's choices are installed)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of MIB MiB (scales HBM counters)")
    ap.add_argument("--legs", default=",".join(EXTRA_LEGS),
                    help="comma-separated extra legs to run (default: all of %s)" % ",".join(EXTRA_LEGS))
    ap.add_argument("--traffic-record", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the FP32 tile's HBM-traffic record from two rocprofv3 --pmc counter files "
                         "(FETCH_SIZE and WRITE_SIZE passes with --copy-calibration 1024) and exit")
    args = ap.parse_args()
    if args.traffic_record:
        write_traffic_record(*args.traffic_record)
        return
    legs = set(l for l in args.legs.split(",") if l)
    unknown = legs - set(EXTRA_LEGS)
    if unknown:
        ap.error("unknown legs: %s" % ",".join(sorted(unknown)))
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the hot path here is single-GPU (no collectives); "
              "sharding over several GPUs is not built", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1711_11224_amd as nd
    import synth

    dev = torch.device("cuda:0")
    cfg = synth.CONFIGS["c3_metric"]
    N = int(np.prod(cfg.shape))
    K = int(np.prod(cfg.psf_shape))
    from paper_1711_11224_amd import autotune
    y, h, x0 = make_inputs(nd, torch, cfg, dev)
    if args.retune:
        # the workload's own operands: X^0 for the forward, its residual for the transpose
        r0 = nd.conv_full_nd(x0, h) - y
        for pr in ("fp32", "bf16", "split_bf16"):
            res = autotune.tune_conv(cfg.shape, cfg.psf_shape, pr, table=args.tuning_table, x=x0, h=h, r=r0)
            log("tuned %s:" % pr, {op: res[op][0] for op in res}, {op: res[op][1] for op in res})
        del r0
    else:
        log("kernel forms installed from the tuning table:", autotune.apply_table(args.tuning_table))
    tile_forms = {pr: {op: list(autotune.current_form(cfg.shape, cfg.psf_shape, op, pr)) for op in autotune.OPS}
                  for pr in ("fp32", "bf16", "split_bf16")}
    if args.copy_calibration > 0:
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read, %d bytes written" % (nb, nb))
        del src, dst
    prec = args.precision

    # untimed warm-up steps, then exactly `steps` timed steps
    x = x0.clone()
    nbytes = nd.deconv_workspace_bytes(cfg.shape, cfg.psf_shape, torch.float32, prec)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    if args.warmup > 0:
        nd.deconv_iterate(y, h, x, args.warmup, precision=prec, ws=ws)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_host = time.perf_counter()
    e0.record(s)
    _, stats, info = nd.deconv_iterate(y, h, x, args.steps, precision=prec, ws=ws)
    e1.record(s)
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t_host
    ms = e0.elapsed_time(e1)
    done, status = [int(v) for v in info.cpu().tolist()]
    if done != args.steps:
        log("warning: %d of %d steps accepted (status %d)" % (done, args.steps, status))
    f = stats.cpu().numpy()[: done + 1, 0]
    log("deconv: %d steps in %.1f ms (host %.1f ms), f %.6g -> %.6g" % (args.steps, ms, t_host * 1e3, f[0], f[-1]))
    macs = 2.0 * N * K * done
    value = macs / (ms * 1e-3) / 1e9

    # per-kernel launch durations of the two operators (same kernels as the steps)
    fwd_ms, adj_ms = time_pairs(nd, torch, x, h, prec, args.pair_reps)
    pair_gmacs = 2.0 * N * K / ((fwd_ms + adj_ms) * 1e-3) / 1e9
    log("pair %s: forward %.2f ms, transpose %.2f ms, %.0f GMAC/s" % (prec, fwd_ms, adj_ms, pair_gmacs))
    dom_ms = max(fwd_ms, adj_ms)
    achieved = 2.0 * N * K / (dom_ms * 1e-3) / 1e12
    peak = PEAK[prec]
    roofline = {"bound": "mfma" if os.environ.get("NDC_BOUND", "mfma") == "mfma" else "alu",
                "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": None,
                "traffic_unit": "bytes per launch",
                "kernel": "forward" if fwd_ms >= adj_ms else "transpose",
                "kernel_ms": round(dom_ms, 3)}

    if prec == "fp32":
        # both operators run the 32 x 32 tile instantiation for this workload
        roofline["traffic"] = measured_traffic(TILE_KERNEL, fwd_ms >= adj_ms)

    precisions = {}
    if not args.no_precisions:
        for pr in ("fp32", "bf16", "split_bf16"):
            fm, am = time_pairs(nd, torch, x, h, pr, 3)
            slow = 2.0 * N * K / (max(fm, am) * 1e-3) / 1e12  # TFLOP/s of the slower operator
            precisions[pr] = {"forward_ms": round(fm, 3), "transpose_ms": round(am, 3),
                              "gmacs": round(2.0 * N * K / ((fm + am) * 1e-3) / 1e9, 1),
                              "tflops_slower_op": round(slow, 1), "peak": PEAK[pr],
                              "frac": round(slow / PEAK[pr], 4)}
            precisions[pr].update(deconv_rate(nd, torch, y, h, x0, pr, args.precision_steps))
            if "fp32" in precisions:
                precisions[pr]["pair_speedup_vs_fp32"] = round(
                    (precisions["fp32"]["forward_ms"] + precisions["fp32"]["transpose_ms"]) / (fm + am), 2)
            log("pair %s: %.2f + %.2f ms" % (pr, fm, am))

    out = {
        "metric": "GMAC/s of 3-D full conv+adjoint and deconv iterations/s at 512²×128, PSF 31²×63",
        "value": round(value, 1), "unit": "GMAC/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms / max(1, args.steps), 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp32": "f32", "bf16": "bf16", "split_bf16": "bf16x3"}[prec],
        "data": "synthetic",
        "config": {"workload": "3-D deconvolution, X 128x512x512 (z,y,x), PSF 63x31x31, FP32 storage, lambda 0",
                   "precision": prec, "steps_accepted": done, "iters_per_s": round(done / (ms * 1e-3), 3),
                   "conv_pair_gmacs": round(pair_gmacs, 1), "macs_per_step": 2 * N * K},
        "roofline": roofline,
        "precisions": precisions,
        "tile_forms": tile_forms,
    }
    if not args.no_extra:
        if "step_rules" in legs:
            out["step_rules"] = bench_step_rules(nd, torch, y, h, x0, ws)
            log("step rules:", out["step_rules"])
        if "richardson_lucy" in legs:
            out["richardson_lucy"] = bench_rl(nd, torch, y, h, x0)
            log("richardson-lucy:", out["richardson_lucy"])
        if "paper_2d" in legs:
            out["paper_2d"] = bench_paper_2d(nd, torch)
            log("paper 2-D shapes:", out["paper_2d"])
        if "small_psf" in legs:
            out["small_psf"] = bench_small_psf(nd, torch)
            log("small psf:", out["small_psf"])
        if "differentiable" in legs:
            out["differentiable"] = bench_differentiable(nd, torch)
            log("differentiable:", out["differentiable"])
        if "refinement" in legs:
            out.setdefault("differentiable", {})["refinement"] = bench_joint_refinement(nd, torch)
            log("refinement:", out["differentiable"]["refinement"])
        if "batched" in legs:
            out["batched"] = bench_batched(nd, torch, table=args.tuning_table)
            log("batched:", out["batched"])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, nd, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
