"""The C-ABI library loads and exports every symbol include/ep.h declares;
host-only entry points behave as documented (no device compute here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ep.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(ep_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def eplib():
    from paper_2112_12854_amd import ep
    return ep


def test_header_declares_boundary():
    names = declared_functions()
    for must in ("ep_create", "ep_set_mesh", "ep_set_conductivity", "ep_set_models",
                 "ep_add_stimulus", "ep_init", "ep_step", "ep_sync", "ep_get_vm",
                 "ep_get_activation", "ep_get_apd90", "ep_get_mean_vm_trace",
                 "ep_get_state", "ep_set_state", "ep_footprint"):
        assert must in names


def test_library_exports_every_declared_symbol(eplib):
    L = C.CDLL(eplib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # the binding wraps every declared entry point under the same name
    assert sorted(eplib.exported_symbols()) == declared_functions()


def test_no_device_gives_edevice_not_fallback(eplib):
    """Without a usable HIP device the library refuses to run (no CPU path)."""
    import subprocess, sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import ctypes as C\n"
            "from paper_2112_12854_amd import ep\n"
            "L = ep.lib(); o = ep.ep_options(); L.ep_default_options(C.byref(o))\n"
            "h = C.c_void_p(); print(L.ep_create(C.byref(o), C.byref(h)))\n") % ROOT
    env = dict(os.environ, HIP_VISIBLE_DEVICES="-1", ROCR_VISIBLE_DEVICES="-1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.stdout.strip() == str(eplib.EP_EDEVICE), (r.stdout, r.stderr)


def test_bad_options_rejected(eplib):
    L = eplib.lib()
    o = eplib.ep_options()
    L.ep_default_options(C.byref(o))
    assert o.chi == 140.0 and o.cm == 0.01 and o.dt == 0.02 and o.repol_frac == 0.9
    o.dt = -1.0
    h = C.c_void_p()
    assert L.ep_create(C.byref(o), C.byref(h)) == eplib.EP_EINVAL


def test_state_slot_format_matches_oracle(eplib, oracle_lib):
    """The per-cell state exchange format (slot order per model) is the same
    on both sides; each side lists it from its own model code."""
    for m in range(6):
        assert eplib.model_n_slots(m) == oracle_lib.n_slots(m)
        assert eplib.model_slot_names(m) == oracle_lib.slot_names(m)
    assert eplib.model_n_slots(9) == 0
