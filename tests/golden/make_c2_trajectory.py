"""Write tests/golden/c2_deconv_trajectory.json: the FP64 oracle's
projected-gradient trajectory on the 3-D FP32 workload (X 64x128x128,
PSF 31x15x15, sigma_z 5, sigma_xy 2, Poisson peak 500 + read noise 2,
seed 1, 100 iterations, lambda 0, flat flux-matching start).

Calls only oracle/ and synth/.  Inputs are rounded to float32 first, as the
GPU run receives them.  Stored: f_k and delta_k for every step, X after the
last step at 4096 seeded voxels, and checksums of Y and X^0 so a test can
confirm it rebuilt the same inputs."""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def inputs():
    cfg = synth.CONFIGS["c2_3d_f32"]
    x_true = synth.make_objects(cfg)
    h = synth.psf_for(cfg).astype(np.float32)
    y = synth.add_noise(oracle.conv_full(x_true, h.astype(np.float64)), cfg).astype(np.float32)
    x0 = synth.flat_start(y, h, cfg.shape).astype(np.float32)
    return cfg, y, h, x0


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    cfg, y, h, x0 = inputs()
    t = time.time()
    x, stats, done, status = oracle.deconv(y.astype(np.float64), h.astype(np.float64), x0.astype(np.float64),
                                           cfg.iters)
    rng = np.random.default_rng(2024)
    idx = rng.choice(x.size, 4096, replace=False)
    out = {"config": cfg.name, "iters": cfg.iters, "done": int(done), "status": int(status),
           "y_sha256": sha(y), "x0_sha256": sha(x0), "h_sha256": sha(h),
           "f": stats[:, 0].tolist(), "delta": stats[1:, 1].tolist(), "rejections": stats[1:, 2].tolist(),
           "sample_idx": idx.tolist(), "x_samples": x.ravel()[idx].tolist(),
           "x_norm": float(np.linalg.norm(x)), "oracle_seconds": time.time() - t}
    with open(os.path.join(ROOT, "tests", "golden", "c2_deconv_trajectory.json"), "w") as f:
        json.dump(out, f)
    print("done", done, status, time.time() - t)


if __name__ == "__main__":
    main()
