"""The FP64 exponential of the cell kernels (exp64 in csrc/cellmodels.hpp),
built for the host from the same source and checked against e^x computed to
40 digits: within an ulp over the arguments the models give it (voltages
over a few mV, up to about +-100) and over the whole finite range, exact at
0, inf past ln(DBL_MAX), 0 below the subnormals, subnormal results within
one subnormal step, NaN kept."""
import os
import shutil
import subprocess

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def exp64(tmp_path_factory):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("no hipcc")
    d = tmp_path_factory.mktemp("exp64")
    exe = str(d / "exp64_check")
    subprocess.run([HIPCC, "--cuda-host-only", "-x", "hip", "-O2", "-std=c++17",
                    "-I", os.path.join(ROOT, "paper_2112_12854_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "exp64_check.cpp"), "-o", exe], check=True)

    def run(x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        src, dst = str(d / "x.bin"), str(d / "y.bin")
        x.tofile(src)
        subprocess.run([exe, src, dst], check=True)
        return np.fromfile(dst, dtype=np.float64)
    return run


def ulp_error(x, y):
    mp.mp.dps = 40
    err = np.empty(x.size)
    for i, (a, b) in enumerate(zip(x.tolist(), y.tolist())):
        e = mp.exp(mp.mpf(a))
        err[i] = float(abs(mp.mpf(b) - e) / mp.mpf(np.spacing(float(e))))
    return err


def test_model_range_within_an_ulp(exp64):
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.uniform(-100, 100, 20000), rng.uniform(-1, 1, 5000),
                        rng.uniform(-1e-3, 1e-3, 2000),
                        np.arange(-200, 201) * np.log(2) / 2,        # ends of the reduced range
                        np.nextafter(np.arange(-200, 201) * np.log(2) / 2, np.inf)])
    err = ulp_error(x, exp64(x))
    assert err.max() < 1.0, (err.max(), x[np.argmax(err)])
    assert np.mean(err) < 0.3


def test_full_range_within_an_ulp(exp64):
    rng = np.random.default_rng(12)
    x = rng.uniform(-708.0, 709.7, 20000)
    err = ulp_error(x, exp64(x))
    assert err.max() < 1.0, (err.max(), x[np.argmax(err)])


def test_ends_and_special_values(exp64):
    x = np.array([0.0, -0.0, 709.783, 710.0, 1e5, -746.0, -1e5, np.nan, 709.7, -708.3])
    y = exp64(x)
    assert y[0] == 1.0 and y[1] == 1.0
    assert np.isinf(y[2]) and np.isinf(y[3]) and np.isinf(y[4]) and y[4] > 0
    assert y[5] == 0.0 and y[6] == 0.0
    assert np.isnan(y[7])
    assert np.isfinite(y[8]) and y[8] > 1.6e308   # just below ln(DBL_MAX) = 709.7827
    assert ulp_error(x[8:], y[8:]).max() < 1.0
    # subnormal results: within one step of the subnormal grid
    xs = np.linspace(-744.0, -709.0, 2001)
    ys = exp64(xs)
    mp.mp.dps = 40
    for a, b in zip(xs.tolist(), ys.tolist()):
        assert abs(mp.mpf(b) - mp.exp(mp.mpf(a))) <= mp.mpf(2.0) ** -1074


def test_monotone(exp64):
    x = np.sort(np.random.default_rng(13).uniform(-90, 60, 50000))
    assert np.all(np.diff(exp64(x)) >= 0)
