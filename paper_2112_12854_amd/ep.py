"""Python binding of libep.so (include/ep.h): argument marshalling only.

Every step of the monodomain path runs in the HIP library; this module only
converts arrays and forwards calls under the C names.  PyTorch, when used,
only supplies device memory (its caching allocator, through the library's
allocator callbacks) and the stream the library runs on.  There is no CPU
fallback: if the library or a HIP device is missing, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libep.so")

EP_OK, EP_EINVAL, EP_ENOMEM, EP_EDEVICE, EP_ESTATE, EP_ENUMERIC, EP_EBUSY = 0, -1, -2, -3, -4, -5, -6
EP_FP64, EP_FP32_MIXED = 0, 1
EP_SCHEME_FE, EP_SCHEME_AB2, EP_SCHEME_RL2_AB2 = 0, 1, 2
EP_ORDER_RCM, EP_ORDER_MORTON, EP_ORDER_INPUT = 0, 1, 2
EP_TP06_ENDO, EP_TP06_MID, EP_TP06_EPI, EP_CRN, EP_STEWART, EP_PASSIVE = range(6)
EP_MAX_SLOTS = 21
STATUS_NAMES = {0: "EP_OK", -1: "EP_EINVAL", -2: "EP_ENOMEM", -3: "EP_EDEVICE",
                -4: "EP_ESTATE", -5: "EP_ENUMERIC", -6: "EP_EBUSY"}

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class ep_options(C.Structure):
    _fields_ = [("prec", C.c_int), ("device", C.c_int), ("stream", C.c_void_p),
                ("dt", C.c_double), ("chi", C.c_double), ("cm", C.c_double),
                ("at_threshold", C.c_double), ("repol_frac", C.c_double),
                ("trace_every", C.c_int32), ("dev_alloc", ALLOC_FN),
                ("dev_free", FREE_FN), ("alloc_ctx", C.c_void_p)]


class ep_stimulus(C.Structure):
    _fields_ = [("n_ids", C.c_int64), ("ids", C.POINTER(C.c_int32)), ("t0", C.c_double),
                ("dur", C.c_double), ("amp", C.c_double), ("period", C.c_double),
                ("count", C.c_int32), ("domain", C.c_int32)]


class ep_pmj(C.Structure):
    _fields_ = [("node", C.c_int32), ("two_way", C.c_int32), ("radius", C.c_double),
                ("delay_ortho", C.c_double), ("delay_anti", C.c_double), ("amp", C.c_double),
                ("dur", C.c_double)]


class ep_cell_junction(C.Structure):
    _fields_ = [("cell", C.c_int32), ("two_way", C.c_int32), ("radius", C.c_double),
                ("delay_ortho", C.c_double), ("delay_anti", C.c_double), ("amp", C.c_double),
                ("dur", C.c_double)]


class ep_purkinje(C.Structure):
    _fields_ = [("n", C.c_int64), ("xyz", C.POINTER(C.c_double)), ("n_edges", C.c_int64),
                ("edges", C.POINTER(C.c_int32)), ("edge_scale", C.POINTER(C.c_double)),
                ("sigma", C.c_double), ("model", C.c_int32), ("n_sub", C.c_int32),
                ("n_pmj", C.c_int32), ("pmj", C.POINTER(ep_pmj))]


class ep_request(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("xyz", C.POINTER(C.c_double)),
                ("n_tets", C.c_int64), ("tet_nodes", C.POINTER(C.c_int32)),
                ("fibre", C.POINTER(C.c_double)), ("sigma_l", C.c_double),
                ("sigma_t", C.c_double), ("scale", C.POINTER(C.c_double)),
                ("model", C.POINTER(C.c_uint8)), ("n_stimuli", C.c_int32),
                ("stimuli", C.POINTER(ep_stimulus)), ("ionic_scale", C.c_double * 4),
                ("n_steps", C.c_int64), ("purkinje", C.POINTER(ep_purkinje)),
                ("n_cell_junctions", C.c_int32), ("cell_junctions", C.POINTER(ep_cell_junction)),
                ("medium_substeps", C.c_int32)]


class ep_result(C.Structure):
    _fields_ = [("id", C.c_int64), ("status", C.c_int), ("n_tets", C.c_int64),
                ("steps", C.c_int64), ("footprint", C.c_size_t), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("t_ready", C.c_double)]


class ep_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("running", C.c_int64),
                ("queued", C.c_int64), ("cell_steps", C.c_double),
                ("bytes_in_use", C.c_size_t), ("bytes_budget", C.c_size_t),
                ("graph_launches", C.c_int64), ("table_updates", C.c_int64),
                ("steps_per_graph", C.c_int32), ("xcd_remap", C.c_int32),
                ("autotune_runs", C.c_int64), ("tuned_ms_per_step", C.c_double),
                ("tile_cells", C.c_int32), ("pad", C.c_int32)]


class EPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)

# name -> (restype, argtypes)
_SIGS = {
    "ep_default_options": (None, [C.POINTER(ep_options)]),
    "ep_create": (C.c_int, [C.POINTER(ep_options), C.POINTER(C.c_void_p)]),
    "ep_destroy": (None, [C.c_void_p]),
    "ep_set_mesh": (C.c_int, [C.c_void_p, C.c_int64, _dp, C.c_int64, _ip]),
    "ep_set_conductivity": (C.c_int, [C.c_void_p, _dp, C.c_double, C.c_double, _dp]),
    "ep_set_models": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint8)]),
    "ep_set_ionic_scale": (C.c_int, [C.c_void_p, C.c_char_p, C.c_double]),
    "ep_add_stimulus": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, _ip, C.c_double,
                                  C.c_double, C.c_double, C.c_double, C.c_int32]),
    "ep_set_purkinje": (C.c_int, [C.c_void_p, C.c_int64, _dp, C.c_int64, _ip, C.c_double,
                                  C.c_int32, C.c_int32]),
    "ep_set_purkinje_scale": (C.c_int, [C.c_void_p, C.c_int64, _dp]),
    "ep_set_time_scheme": (C.c_int, [C.c_void_p, C.c_int32]),
    "ep_set_cell_order": (C.c_int, [C.c_void_p, C.c_int32]),
    "ep_set_medium_substeps": (C.c_int, [C.c_void_p, C.c_int32]),
    "ep_get_medium_substeps": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "ep_add_cell_junction": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double,
                                       C.c_int32, C.c_double, C.c_double]),
    "ep_add_pmj": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double,
                             C.c_int32, C.c_double, C.c_double]),
    "ep_get_purkinje_vm": (C.c_int, [C.c_void_p, _dp, C.c_int64]),
    "ep_get_purkinje_activation": (C.c_int, [C.c_void_p, _dp, C.c_int64]),
    "ep_get_purkinje_substeps": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "ep_set_bidomain": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_int32, C.c_double,
                                  C.c_int32]),
    "ep_get_phi_e": (C.c_int, [C.c_void_p, _dp, C.c_int64]),
    "ep_get_bidomain_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                        _dp]),
    "ep_init": (C.c_int, [C.c_void_p]),
    "ep_footprint": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "ep_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "ep_sync": (C.c_int, [C.c_void_p]),
    "ep_get_vm": (C.c_int, [C.c_void_p, _dp, C.c_int64]),
    "ep_get_activation": (C.c_int, [C.c_void_p, _dp, C.c_int64]),
    "ep_get_apd90": (C.c_int, [C.c_void_p, _dp, C.c_int64]),
    "ep_get_mean_vm_trace": (C.c_int, [C.c_void_p, _dp, _dp, C.c_int64,
                                       C.POINTER(C.c_int64)]),
    "ep_get_time": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), _dp]),
    "ep_apply_diffusion": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "ep_apply_diffusion_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "ep_get_states": (C.c_int, [C.c_void_p, _dp, C.c_int64, C.c_int32]),
    "ep_set_states": (C.c_int, [C.c_void_p, _dp, C.c_int64, C.c_int32]),
    "ep_model_n_slots": (C.c_int, [C.c_int]),
    "ep_model_slot_name": (C.c_char_p, [C.c_int, C.c_int]),
    "ep_state_size": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "ep_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "ep_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "ep_set_launch": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]),
    "ep_set_tile_size": (C.c_int, [C.c_void_p, C.c_int32]),
    "ep_get_launch": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                C.POINTER(C.c_int32)]),
    "ep_autotune": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_int32),
                              C.POINTER(C.c_int32), _dp]),
    "ep_profile_steps": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, _dp, _dp, _dp]),
    "ep_algorithmic_bytes": (C.c_int, [C.c_void_p, _dp, _dp, _dp]),
    "ep_last_error": (C.c_char_p, [C.c_void_p]),
    "ep_server_create": (C.c_int, [C.POINTER(ep_options), C.c_size_t, C.c_int32,
                                   C.POINTER(C.c_void_p)]),
    "ep_server_submit": (C.c_int, [C.c_void_p, C.POINTER(ep_request), C.POINTER(C.c_int64)]),
    "ep_server_poll": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(ep_result)]),
    "ep_server_wait": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(ep_result)]),
    "ep_server_get_vm": (C.c_int, [C.c_void_p, C.c_int64, _dp, C.c_int64]),
    "ep_server_get_activation": (C.c_int, [C.c_void_p, C.c_int64, _dp, C.c_int64]),
    "ep_server_get_apd90": (C.c_int, [C.c_void_p, C.c_int64, _dp, C.c_int64]),
    "ep_server_get_purkinje_vm": (C.c_int, [C.c_void_p, C.c_int64, _dp, C.c_int64]),
    "ep_server_get_purkinje_activation": (C.c_int, [C.c_void_p, C.c_int64, _dp, C.c_int64]),
    "ep_server_release": (C.c_int, [C.c_void_p, C.c_int64]),
    "ep_server_get_stats": (C.c_int, [C.c_void_p, C.POINTER(ep_server_stats)]),
    "ep_server_set_launch": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "ep_server_autotune": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32]),
    "ep_server_set_time_scheme": (C.c_int, [C.c_void_p, C.c_int32]),
    "ep_server_hold": (C.c_int, [C.c_void_p, C.c_int32]),
    "ep_server_destroy": (None, [C.c_void_p]),
    "ep_server_last_error": (C.c_char_p, [C.c_void_p]),
}


def lib():
    """Load libep.so; raises if it was not built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "paper_2112_12854_amd/build.py (or __graft_entry__.build())")
        # One HIP runtime per process: PyTorch ships its own, so load it
        # first (when installed); the library then binds to that runtime and
        # PyTorch's streams and caching allocator can be handed to it.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(st, h=None):
    if st != EP_OK:
        msg = lib().ep_last_error(h).decode() if h else ""
        raise EPError(st, msg)


def _d(a):
    return a.ctypes.data_as(_dp)


class _TorchAllocator:
    """Device memory from PyTorch's caching allocator."""

    def __init__(self, device: int):
        import torch
        self.torch = torch
        self.device = device
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            return int(self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device))
        except Exception:
            return None

    def _free(self, ptr, ctx):
        self.torch.cuda.caching_allocator_delete(ptr)


class Sim:
    """One simulation object: create, upload a workload, init, step, read.

    `w` is a paper_2112_12854_amd.meshgen.Workload.  `allocator` is "torch"
    (PyTorch caching allocator and a PyTorch side stream) or "hip" (the
    library's hipMalloc and its own stream)."""

    def __init__(self, w, prec: int = EP_FP64, device: int = 0,
                 allocator: str = "hip", trace_every: int = 50,
                 launch=None, cell_order=None):
        L = lib()
        o = ep_options()
        L.ep_default_options(C.byref(o))
        o.prec, o.device = prec, device
        o.dt, o.chi, o.cm = w.dt, w.chi, w.cm
        o.trace_every = trace_every
        self._alloc = None
        self._stream = None
        if allocator == "torch":
            import torch
            self._alloc = _TorchAllocator(device)
            o.dev_alloc, o.dev_free = self._alloc.alloc_cb, self._alloc.free_cb
            self._stream = torch.cuda.Stream(device=device)
            o.stream = C.c_void_p(self._stream.cuda_stream)
        h = C.c_void_p()
        _check(L.ep_create(C.byref(o), C.byref(h)))
        self.h = h
        self.n = w.n_tets
        self.prec = prec
        xyz = np.ascontiguousarray(w.xyz, np.float64)
        tets = np.ascontiguousarray(w.tets, np.int32)
        _check(L.ep_set_mesh(h, w.n_nodes, _d(xyz), w.n_tets, tets.ctypes.data_as(_ip)), h)
        fib = np.ascontiguousarray(w.fibre, np.float64)
        sc = None if w.scale is None else np.ascontiguousarray(w.scale, np.float64)
        _check(L.ep_set_conductivity(h, _d(fib), w.sigma_l, w.sigma_t,
                                     None if sc is None else _d(sc)), h)
        mdl = np.ascontiguousarray(w.model, np.uint8)
        _check(L.ep_set_models(h, mdl.ctypes.data_as(C.POINTER(C.c_uint8))), h)
        for k, v in (w.ionic_scale or {}).items():
            _check(L.ep_set_ionic_scale(h, k.encode(), float(v)), h)
        pk = getattr(w, "purkinje", None)
        self.n_purkinje = 0
        if pk is not None:
            pxyz = np.ascontiguousarray(pk.xyz, np.float64)
            pe = np.ascontiguousarray(pk.edges, np.int32)
            _check(L.ep_set_purkinje(h, pxyz.shape[0], _d(pxyz), pe.shape[0],
                                     pe.ctypes.data_as(_ip), pk.sigma, pk.model, pk.n_sub), h)
            if pk.edge_scale is not None:
                es = np.ascontiguousarray(pk.edge_scale, np.float64)
                _check(L.ep_set_purkinje_scale(h, es.size, _d(es)), h)
            self.n_purkinje = pxyz.shape[0]
            for node in pk.pmj_nodes:
                _check(L.ep_add_pmj(h, int(node), pk.pmj_radius, pk.delay_ortho, pk.delay_anti,
                                    int(pk.two_way), pk.pmj_amp, pk.pmj_dur), h)
        for cj in getattr(w, "cell_junctions", []):
            _check(L.ep_add_cell_junction(h, int(cj.cell), cj.radius, cj.delay_ortho, cj.delay_anti,
                                          int(cj.two_way), cj.amp, cj.dur), h)
        for st in w.stimuli:
            ids = np.ascontiguousarray(st.ids, np.int32)
            _check(L.ep_add_stimulus(h, st.domain, ids.size, ids.ctypes.data_as(_ip),
                                     st.t0, st.dur, st.amp, st.period, st.count), h)
        if getattr(w, "time_scheme", 0):
            _check(L.ep_set_time_scheme(h, int(w.time_scheme)), h)
        bd = getattr(w, "bidomain", None)
        self.bidomain = bd is not None
        if bd is not None:
            _check(L.ep_set_bidomain(h, bd.sigma_el, bd.sigma_et, bd.restart, bd.tol,
                                     bd.max_iter), h)
        if launch is not None:
            self.set_launch(*launch)
        if cell_order is not None:
            _check(L.ep_set_cell_order(h, int(cell_order)), h)
        if getattr(w, "medium_substeps", None) is not None:
            _check(L.ep_set_medium_substeps(h, int(w.medium_substeps)), h)
        _check(L.ep_init(h), h)
        self.device = device

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().ep_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- stepping
    def step(self, n: int):
        _check(lib().ep_step(self.h, int(n)), self.h)

    def sync(self):
        _check(lib().ep_sync(self.h), self.h)

    def set_launch(self, block=256, steps_per_graph=50, xcd_remap=1):
        """block: cells per cell tile 64/128/256 (0 keeps); steps_per_graph: 0 = no graphs."""
        _check(lib().ep_set_launch(self.h, block, steps_per_graph, xcd_remap), self.h)

    def set_tile_size(self, cells: int = 256):
        _check(lib().ep_set_tile_size(self.h, int(cells)), self.h)

    def launch(self) -> dict:
        """The schedule and cell tile size in effect."""
        a, c, d = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().ep_get_launch(self.h, C.byref(a), C.byref(c), C.byref(d)), self.h)
        return {"tile_cells": a.value, "steps_per_graph": c.value, "xcd_remap": d.value}

    def medium_substeps(self) -> int:
        """Substeps per step of the 2D medium (1: it steps with the tets)."""
        n = C.c_int32()
        _check(lib().ep_get_medium_substeps(self.h, C.byref(n)), self.h)
        return n.value

    def apply_diffusion(self, v, entry: str = "ep_apply_diffusion"):
        """The simulation's diffusion operator applied to the cell potentials
        v ([n_tets], caller order): L in mV/ms as a host array.  v and L pass
        through device tensors; `entry` names the C entry point to call."""
        import torch
        dev = torch.device("cuda", self.device)
        vt = torch.as_tensor(np.ascontiguousarray(v, np.float64)).to(dev)
        Lt = torch.full_like(vt, float("nan"))
        torch.cuda.synchronize(dev)
        _check(getattr(lib(), entry)(self.h, C.c_void_p(vt.data_ptr()),
                                     C.c_void_p(Lt.data_ptr()), vt.numel()), self.h)
        torch.cuda.synchronize(dev)
        return Lt.cpu().numpy()

    # ---- readouts
    def _vec(self, fn):
        out = np.empty(self.n)
        _check(fn(self.h, _d(out), self.n), self.h)
        return out

    def vm(self):
        return self._vec(lib().ep_get_vm)

    def activation(self):
        return self._vec(lib().ep_get_activation)

    def apd90(self):
        return self._vec(lib().ep_get_apd90)

    def _pvec(self, fn):
        out = np.empty(self.n_purkinje)
        _check(fn(self.h, _d(out), self.n_purkinje), self.h)
        return out

    def purkinje_vm(self):
        return self._pvec(lib().ep_get_purkinje_vm)

    def purkinje_activation(self):
        return self._pvec(lib().ep_get_purkinje_activation)

    def phi_e(self):
        return self._vec(lib().ep_get_phi_e)

    def bidomain_stats(self):
        """(Arnoldi steps of the last solve, total, last relative residual)"""
        a, b, r = C.c_int64(), C.c_int64(), C.c_double()
        _check(lib().ep_get_bidomain_stats(self.h, C.byref(a), C.byref(b), C.byref(r)), self.h)
        return a.value, b.value, r.value

    def purkinje_n_sub(self) -> int:
        n = C.c_int32()
        _check(lib().ep_get_purkinje_substeps(self.h, C.byref(n)), self.h)
        return n.value

    def mean_vm_trace(self, cap: int = 1 << 16):
        t, v = np.empty(cap), np.empty(cap)
        n = C.c_int64()
        _check(lib().ep_get_mean_vm_trace(self.h, _d(t), _d(v), cap, C.byref(n)), self.h)
        return t[:n.value].copy(), v[:n.value].copy()

    def time(self):
        s, t = C.c_int64(), C.c_double()
        _check(lib().ep_get_time(self.h, C.byref(s), C.byref(t)), self.h)
        return s.value, t.value

    def states(self):
        out = np.empty((EP_MAX_SLOTS, self.n))
        _check(lib().ep_get_states(self.h, _d(out), self.n, EP_MAX_SLOTS), self.h)
        return out

    def set_states(self, st):
        st = np.ascontiguousarray(st, np.float64)
        _check(lib().ep_set_states(self.h, _d(st), self.n, EP_MAX_SLOTS), self.h)

    def footprint(self) -> int:
        b = C.c_size_t()
        _check(lib().ep_footprint(self.h, C.byref(b)), self.h)
        return b.value

    def checkpoint(self) -> bytes:
        n = C.c_size_t()
        _check(lib().ep_state_size(self.h, C.byref(n)), self.h)
        buf = C.create_string_buffer(n.value)
        _check(lib().ep_get_state(self.h, buf, n.value), self.h)
        return buf.raw

    def restore(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().ep_set_state(self.h, buf, len(blob)), self.h)

    def autotune(self, trial_steps: int = 100) -> dict:
        """Pick the fastest launch schedule on this simulation (the trial
        steps advance it); returns the choice and its ms per step."""
        k, r, ms = C.c_int32(), C.c_int32(), C.c_double()
        _check(lib().ep_autotune(self.h, int(trial_steps), C.byref(k), C.byref(r),
                                 C.byref(ms)), self.h)
        out = self.launch()
        out["ms_per_step"] = ms.value
        return out

    def profile_steps(self, n: int, per_step: bool = False, every: int = 1):
        """n steps, those of steps 0, every, 2 every, ... event-timed: (cell
        kernel ms, node gather ms) averages over the timed steps, and with
        per_step the device time of every timed step (ms)."""
        a, b = C.c_double(), C.c_double()
        st = np.empty((int(n) + int(every) - 1) // int(every)) if per_step and every > 0 else None
        _check(lib().ep_profile_steps(self.h, int(n), int(every), C.byref(a), C.byref(b),
                                      None if st is None else _d(st)), self.h)
        return (a.value, b.value, st) if per_step else (a.value, b.value)

    def algorithmic_bytes(self, with_diffusion: bool = False):
        """(node gather, cell kernel[, one apply_diffusion call]) bytes per step."""
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        _check(lib().ep_algorithmic_bytes(self.h, C.byref(a), C.byref(b), C.byref(c)), self.h)
        return (a.value, b.value, c.value) if with_diffusion else (a.value, b.value)


def model_n_slots(model: int) -> int:
    return lib().ep_model_n_slots(model)


def model_slot_names(model: int):
    return [lib().ep_model_slot_name(model, i).decode() for i in range(model_n_slots(model))]


def _result_dict(r: ep_result) -> dict:
    return dict(id=r.id, status=r.status, n_tets=r.n_tets, steps=r.steps,
                footprint=r.footprint, t_submit=r.t_submit, t_ready=r.t_ready,
                t_admit=r.t_admit, t_done=r.t_done, latency=r.t_done - r.t_submit)


class Server:
    """Continuous-batching server (ep_server_*): submit workloads, wait, read."""

    def __init__(self, prec: int = EP_FP32_MIXED, dt: float = 0.02, hbm_budget: int = 0,
                 max_slots: int = 64, device: int = 0, trace_every: int = 50,
                 allocator: str = "hip", steps_per_graph: int = 50, chi=140.0, cm=0.01,
                 time_scheme: int = 0):
        L = lib()
        o = ep_options()
        L.ep_default_options(C.byref(o))
        o.prec, o.device, o.dt, o.chi, o.cm = prec, device, dt, chi, cm
        o.trace_every = trace_every
        self._alloc = None
        self._stream = None
        if allocator == "torch":
            import torch
            self._alloc = _TorchAllocator(device)
            o.dev_alloc, o.dev_free = self._alloc.alloc_cb, self._alloc.free_cb
            self._stream = torch.cuda.Stream(device=device)
            o.stream = C.c_void_p(self._stream.cuda_stream)
        h = C.c_void_p()
        _check(L.ep_server_create(C.byref(o), int(hbm_budget), int(max_slots), C.byref(h)))
        self.h = h
        self.n_of = {}
        self.np_of = {}
        _check(L.ep_server_set_launch(h, steps_per_graph, 1))
        if time_scheme:
            _check(L.ep_server_set_time_scheme(h, int(time_scheme)))

    def _err(self):
        return lib().ep_server_last_error(self.h).decode()

    def _chk(self, st):
        if st != EP_OK:
            raise EPError(st, self._err())

    def submit(self, w, n_steps: int) -> int:
        xyz = np.ascontiguousarray(w.xyz, np.float64)
        tets = np.ascontiguousarray(w.tets, np.int32)
        fib = np.ascontiguousarray(w.fibre, np.float64)
        sc = None if w.scale is None else np.ascontiguousarray(w.scale, np.float64)
        mdl = np.ascontiguousarray(w.model, np.uint8)
        ids = [np.ascontiguousarray(st.ids, np.int32) for st in w.stimuli]
        stims = (ep_stimulus * max(1, len(w.stimuli)))()
        for k, st in enumerate(w.stimuli):
            stims[k] = ep_stimulus(ids[k].size, ids[k].ctypes.data_as(_ip), st.t0, st.dur,
                                   st.amp, st.period, st.count, st.domain)
        rq = ep_request()
        rq.n_nodes, rq.xyz = w.n_nodes, _d(xyz)
        rq.n_tets, rq.tet_nodes = w.n_tets, tets.ctypes.data_as(_ip)
        rq.fibre, rq.sigma_l, rq.sigma_t = _d(fib), w.sigma_l, w.sigma_t
        rq.scale = None if sc is None else _d(sc)
        rq.model = mdl.ctypes.data_as(C.POINTER(C.c_uint8))
        rq.n_stimuli, rq.stimuli = len(w.stimuli), stims
        gs = w.ionic_scale or {}
        for i, k in enumerate(("GKr", "GKs", "GCaL", "GNa")):
            rq.ionic_scale[i] = float(gs.get(k, 1.0))
        rq.n_steps = int(n_steps)
        pk = getattr(w, "purkinje", None)
        keep = []
        if pk is not None:
            pxyz = np.ascontiguousarray(pk.xyz, np.float64)
            pe = np.ascontiguousarray(pk.edges, np.int32)
            es = None if pk.edge_scale is None else np.ascontiguousarray(pk.edge_scale, np.float64)
            jn = (ep_pmj * max(1, len(pk.pmj_nodes)))()
            for k, node in enumerate(pk.pmj_nodes):
                jn[k] = ep_pmj(int(node), int(pk.two_way), pk.pmj_radius, pk.delay_ortho,
                               pk.delay_anti, pk.pmj_amp, pk.pmj_dur)
            g = ep_purkinje(pxyz.shape[0], _d(pxyz), pe.shape[0], pe.ctypes.data_as(_ip),
                            None if es is None else _d(es), pk.sigma, pk.model, pk.n_sub,
                            len(pk.pmj_nodes), jn)
            keep = [pxyz, pe, es, jn, g]
            rq.purkinje = C.pointer(g)
        cjs = list(getattr(w, "cell_junctions", []))
        if cjs:
            arr = (ep_cell_junction * len(cjs))()
            for k, cj in enumerate(cjs):
                arr[k] = ep_cell_junction(int(cj.cell), int(cj.two_way), cj.radius, cj.delay_ortho,
                                          cj.delay_anti, cj.amp, cj.dur)
            rq.n_cell_junctions, rq.cell_junctions = len(cjs), arr
            keep.append(arr)
        ms = getattr(w, "medium_substeps", None)
        if ms is not None:
            rq.medium_substeps = -1 if ms <= 0 else int(ms)
        rid = C.c_int64()
        self._chk(lib().ep_server_submit(self.h, C.byref(rq), C.byref(rid)))
        del keep
        self.n_of[rid.value] = w.n_tets
        self.np_of[rid.value] = 0 if pk is None else int(np.asarray(pk.xyz).shape[0])
        return rid.value

    def poll(self, rid: int):
        r = ep_result()
        st = lib().ep_server_poll(self.h, rid, C.byref(r))
        if st == EP_EBUSY:
            return None
        self._chk(st)
        return _result_dict(r)

    def wait(self, rid: int) -> dict:
        r = ep_result()
        self._chk(lib().ep_server_wait(self.h, rid, C.byref(r)))
        return _result_dict(r)

    def _vec(self, fn, rid, graph=False):
        out = np.empty(self.np_of[rid] if graph else self.n_of[rid])
        st = fn(self.h, rid, _d(out), out.size)
        if st not in (EP_OK, EP_ENUMERIC):
            self._chk(st)
        return out

    def vm(self, rid):
        return self._vec(lib().ep_server_get_vm, rid)

    def activation(self, rid):
        return self._vec(lib().ep_server_get_activation, rid)

    def apd90(self, rid):
        return self._vec(lib().ep_server_get_apd90, rid)

    def purkinje_vm(self, rid):
        return self._vec(lib().ep_server_get_purkinje_vm, rid, graph=True)

    def purkinje_activation(self, rid):
        return self._vec(lib().ep_server_get_purkinje_activation, rid, graph=True)

    def release(self, rid):
        self._chk(lib().ep_server_release(self.h, rid))

    def set_launch(self, steps_per_graph: int = 50, xcd_remap: int = 1):
        self._chk(lib().ep_server_set_launch(self.h, int(steps_per_graph), int(xcd_remap)))

    def hold(self, on: bool = True):
        """Admit and upload requests without stepping them (batch start)."""
        self._chk(lib().ep_server_hold(self.h, int(bool(on))))

    def autotune(self, trial_steps: int = 50, retune: bool = False):
        """Tune the schedule on the batch live when the driver next steps."""
        self._chk(lib().ep_server_autotune(self.h, int(trial_steps), int(bool(retune))))

    def stats(self) -> dict:
        s = ep_server_stats()
        self._chk(lib().ep_server_get_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in ep_server_stats._fields_}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().ep_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
