"""The FP64 exponential and logarithm of the cell kernels (exp64 and log64
in csrc/cellmodels.hpp), built for the host from the same source and checked
against e^x and ln x computed to 40 digits.  exp64: within an ulp over the
arguments the models give it (voltages over a few mV, up to about +-100) and
over the whole finite range, exact at 0, inf past ln(DBL_MAX), 0 below the
subnormals, subnormal results within one subnormal step, NaN kept.  log64:
within an ulp over the concentration ratios of the Nernst potentials and
over the positive normal and subnormal numbers, exact at 1 and at powers of
two up to the rounding of k ln2, monotone, NaN for 0, negative, infinite
and NaN arguments."""
import os
import shutil
import subprocess

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def check_exe(tmp_path_factory):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("no hipcc")
    d = tmp_path_factory.mktemp("fp64_math")
    exe = str(d / "fp64_math_check")
    subprocess.run([HIPCC, "--cuda-host-only", "-x", "hip", "-O2", "-std=c++17",
                    "-I", os.path.join(ROOT, "paper_2112_12854_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "fp64_math_check.cpp"), "-o", exe],
                   check=True)
    return d, exe


def runner(check_exe, fn):
    d, exe = check_exe

    def run(x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        src, dst = str(d / "x.bin"), str(d / "y.bin")
        x.tofile(src)
        subprocess.run([exe, fn, src, dst], check=True)
        return np.fromfile(dst, dtype=np.float64)
    return run


@pytest.fixture(scope="module")
def exp64(check_exe):
    return runner(check_exe, "exp")


@pytest.fixture(scope="module")
def log64(check_exe):
    return runner(check_exe, "log")


def ulp_error(x, y, f=None):
    mp.mp.dps = 40
    f = f or mp.exp
    err = np.empty(x.size)
    for i, (a, b) in enumerate(zip(x.tolist(), y.tolist())):
        e = f(mp.mpf(a))
        err[i] = float(abs(mp.mpf(b) - e) / mp.mpf(np.spacing(abs(float(e)))))
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


def test_log_model_range_within_an_ulp(log64):
    rng = np.random.default_rng(21)
    # ratios of the Nernst potentials (Na, K, Ca, K+Na; also the CRN and
    # Stewart values) and a dense sweep around 1, where ln x is small
    x = np.concatenate([10.0 ** rng.uniform(-2, 5.5, 20000), rng.uniform(0.5, 2.0, 5000),
                        1.0 + rng.uniform(-1e-3, 1e-3, 2000),
                        np.sqrt(0.5) * (1 + rng.uniform(-1e-12, 1e-12, 500))])
    err = ulp_error(x, log64(x), mp.log)
    assert err.max() < 1.0, (err.max(), x[np.argmax(err)])
    assert np.mean(err) < 0.3


def test_log_full_range_and_special_values(log64):
    rng = np.random.default_rng(22)
    x = np.concatenate([2.0 ** rng.uniform(-1070, 1023, 20000), np.array([np.nextafter(0, 1)])])
    err = ulp_error(x, log64(x), mp.log)
    assert err.max() < 1.0, (err.max(), x[np.argmax(err)])
    y = log64(np.array([1.0, 2.0, 0.5, 1024.0, 0.0, -0.0, -1.0, np.inf, np.nan]))
    assert y[0] == 0.0
    assert abs(y[1] - np.log(2.0)) <= np.spacing(np.log(2.0))
    assert y[2] == -y[1] and abs(y[3] - 10 * y[1]) <= 8 * np.spacing(y[3])
    assert np.all(np.isnan(y[4:]))


def test_log_monotone(log64):
    x = np.sort(10.0 ** np.random.default_rng(23).uniform(-6, 6, 50000))
    assert np.all(np.diff(log64(x)) >= 0)
