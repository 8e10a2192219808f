"""The register DFT building blocks of the k-mesh transforms, the pair
transform and the grid FFT (dft_small.hpp: radix-2 splits, butterflies for
lengths 2 and 4, symmetric pairs for 3 and 5, direct sums otherwise),
compiled for the host and checked against numpy's FFT for every length the
kernels instantiate (1-16), both signs in FP64 and the forward FP32 lines."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("dft") / "dft_host_check")
    cmd = [HIPCC, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
           "-I", os.path.join(ROOT, "paper_2601_16379_amd", "csrc"),
           os.path.join(HERE, "dft_host_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def _run(exe, cases):
    text = "".join("%d %d %d %s\n" % (len(x), s, b, " ".join("%.17g %.17g" % (v.real, v.imag) for v in x))
                   for x, s, b in cases)
    r = subprocess.run([exe], input=text, capture_output=True, text=True)
    assert r.returncode == 0
    out = []
    for line in r.stdout.strip().splitlines():
        v = np.array([float(t) for t in line.split()])
        out.append(v[0::2] + 1j * v[1::2])
    return out


def test_line_dfts_against_numpy(driver):
    rng = np.random.default_rng(11)
    cases = []
    for m in range(1, 17):
        for rep in range(20):
            x = rng.standard_normal(m) + 1j * rng.standard_normal(m)
            cases += [(x, -1, 64), (x, 1, 64), (x.astype(np.complex64).astype(np.complex128), -1, 32)]
    got = _run(driver, cases)
    assert len(got) == len(cases)
    worst = {}
    for (x, s, b), y in zip(cases, got):
        m = len(x)
        ref = np.fft.fft(x) if s < 0 else m * np.fft.ifft(x)
        scale = np.sqrt(m) * np.max(np.abs(x))
        err = np.max(np.abs(y - ref)) / scale
        key = (m, s, b)
        worst[key] = max(worst.get(key, 0.0), err)
        # FP64: a few ulps per level of the splits; FP32: a few FP32 ulps
        assert err < (1e-15 * (2 + m) if b == 64 else 1e-6 * (2 + m)), (m, s, b, err)
    print({k: "%.1e" % v for k, v in sorted(worst.items()) if k[0] in (3, 5, 6, 8, 10, 16)})
