"""The library's host code (mesh preparation, Purkinje graph and junction
regions, coarse aggregates, the server's admission rule) built on the CPU
with AddressSanitizer and UndefinedBehaviorSanitizer and checked against the
oracle by tests/host/host_check.cpp: the fused stencil applied on the CPU
equals the oracle's operator to 1e-12 of max |L| in every cell order, with
and without the 2D medium split off; substep counts and junction regions
equal the oracle's; admission keeps budget, slots and arrival order;
malformed meshes are refused."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2112_12854_amd", "csrc")
ORACLE = os.path.join(ROOT, "oracle")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=undefined"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                    reason="no host compiler")
def test_host_code_under_sanitizers(tmp_path):
    objs = []
    for src in ("orc_tissue.c", "orc_tp06.c", "orc_crn.c", "orc_stewart.c"):
        obj = str(tmp_path / (src + ".o"))
        subprocess.run(["gcc", "-std=c99", "-fopenmp", "-ffp-contract=off", "-D_DEFAULT_SOURCE"] + SAN +
                       ["-c", os.path.join(ORACLE, src), "-o", obj], check=True)
        objs.append(obj)
    exe = str(tmp_path / "host_check")
    subprocess.run(["g++", "-std=c++17", "-pthread"] + SAN +
                   [os.path.join(ROOT, "tests", "host", "host_check.cpp")] +
                   [os.path.join(CSRC, s) for s in ("prep.cpp", "purkinje.cpp", "coarse.cpp")] +
                   objs + ["-fopenmp", "-lm", "-o", exe], check=True)
    env = dict(os.environ, OMP_NUM_THREADS="1", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=900)
    print(r.stdout[-4000:])
    print(r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-2000:]
    assert "host checks passed" in r.stdout
    assert "FAIL" not in r.stdout
