"""Device-code resources of the kernels on the measured paths (CPU: hipcc
cross-compiles for gfx950 with the library's own flags and reports each
kernel's registers and scratch).  A kernel that keeps a helper as a real
function call, or spills inside its instruction loop, shows up as scratch
memory per lane; the small-PSF kernel once lost inlining that way and ran
4x slower.  Limits: none for the FP32 matrix-core tile and the row-slot
tiles, a few words for the small-PSF kernel (its finished-plane buffer)."""
import concurrent.futures as cf
import importlib.util
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1711_11224_amd")


def _build_module():
    spec = importlib.util.spec_from_file_location("ndc_build_flags", os.path.join(PKG, "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


CASES = {"conv_small_f32_k13.hip": 32,  # 3^3: the HBM-bound small PSF
         "conv_small_f32_k5.hip": 32,
         "conv_mfma.hip": 0,             # the FP32 tile of the metric workload
         "conv_slot.hip": 0}             # bf16 row-slot tile


def _scratch(b, hipcc, src, tmp):
    cmd = [hipcc] + b.CXXFLAGS + b.FILE_FLAGS.get(src, []) + [
        "--cuda-device-only", "-Rpass-analysis=kernel-resource-usage", "-c", os.path.join(b.CSRC, src), "-o",
        os.path.join(tmp, src + ".o")]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-2000:]
    names = re.findall(r"Function Name: (\S+)", r.stderr)
    scratch = [int(v) for v in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", r.stderr)]
    assert names and len(names) == len(scratch)
    return max(zip(scratch, names))


@pytest.mark.slow
def test_kernel_scratch_per_lane():
    """The sources compile in parallel (about two minutes on 8 cores)."""
    b = _build_module()
    hipcc = b._hipcc()
    if os.path.sep in hipcc and not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as tmp, cf.ThreadPoolExecutor(len(CASES)) as ex:
        worst = dict(zip(CASES, ex.map(lambda s: _scratch(b, hipcc, s, tmp), CASES)))
    for src, limit in CASES.items():
        assert worst[src][0] <= limit, "%s: %s keeps %d bytes of scratch per lane (limit %d)" % (
            src, worst[src][1], worst[src][0], limit)
