"""ctypes view of the CPU FP64 oracle (oracle/liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline call this to check and time the HIP library.  The product package
never imports it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
MAX_SLOTS = 21
TP06_ENDO, TP06_MID, TP06_EPI, CRN, STEWART, PASSIVE = range(6)

_lib = None
_lib_path = LIB_PATH
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_up = C.POINTER(C.c_uint8)


def use_native():
    """Build the -march=native copy of the oracle on this host and load it
    instead of the portable one (the timing copy; call before any other use)."""
    global _lib_path
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    from . import build as _b
    _lib_path = _b.build(native=True)
    return _lib_path


def build_flags() -> list[str]:
    """Compiler flags of the loaded copy."""
    from . import build as _b
    return ["gcc"] + _b.flags(native=_lib_path != LIB_PATH)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_lib_path):
            from . import build as _b
            _b.build()
        L = C.CDLL(_lib_path)
        L.orc_model_n_slots.argtypes = [C.c_int]
        L.orc_model_slot_name.argtypes = [C.c_int, C.c_int]
        L.orc_model_slot_name.restype = C.c_char_p
        L.orc_model_init.argtypes = [C.c_int, _dp]
        L.orc_model_step.argtypes = [C.c_int, _dp, C.c_double, C.c_double, _dp]
        L.orc_model_step.restype = C.c_double
        L.orc_create.argtypes = [C.c_int64, _dp, C.c_int64, _ip, _dp, C.c_double,
                                 C.c_double, _dp, _up, C.c_double, C.c_double,
                                 C.c_double]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_ionic_scale.argtypes = [C.c_void_p, _dp]
        L.orc_add_stimulus.argtypes = [C.c_void_p, C.c_int64, _ip, C.c_double,
                                       C.c_double, C.c_double, C.c_double, C.c_int32]
        L.orc_set_detection.argtypes = [C.c_void_p, C.c_double, C.c_double]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_get_step.argtypes = [C.c_void_p]
        L.orc_get_step.restype = C.c_int64
        L.orc_set_step.argtypes = [C.c_void_p, C.c_int64]
        for name in ("orc_get_vm", "orc_get_activation", "orc_get_apd90",
                     "orc_get_states", "orc_set_states", "orc_get_detect_state",
                     "orc_set_detect_state"):
            getattr(L, name).argtypes = [C.c_void_p, _dp]
        L.orc_mean_vm.argtypes = [C.c_void_p]
        L.orc_mean_vm.restype = C.c_double
        L.orc_geometry.argtypes = [C.c_void_p, _dp, _dp, _ip]
        for name in ("orc_node_values", "orc_cell_gradients", "orc_apply_diffusion"):
            getattr(L, name).argtypes = [C.c_void_p, _dp, _dp]
        L.orc_detect_waveform.argtypes = [_dp, C.c_int64, C.c_double, C.c_double,
                                          C.c_double, _dp, _dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_purkinje.argtypes = [C.c_void_p, C.c_int64, _dp, C.c_int64, _ip, _dp,
                                       C.c_double, C.c_int, C.c_int32]
        L.orc_add_pmj.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_double,
                                  C.c_double, C.c_int, C.c_double, C.c_double]
        L.orc_add_cell_junction.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_double,
                                            C.c_double, C.c_int, C.c_double, C.c_double]
        L.orc_add_purkinje_stimulus.argtypes = [C.c_void_p, C.c_int64, _ip, C.c_double,
                                                C.c_double, C.c_double, C.c_double, C.c_int32]
        L.orc_set_time_scheme.argtypes = [C.c_void_p, C.c_int]
        L.orc_set_medium_substeps.argtypes = [C.c_void_p, C.c_int32]
        L.orc_medium_substeps.argtypes = [C.c_void_p]
        L.orc_medium_substeps.restype = C.c_int32
        L.orc_purkinje_n_sub.argtypes = [C.c_void_p]
        L.orc_purkinje_n_sub.restype = C.c_int32
        L.orc_get_purkinje_vm.argtypes = [C.c_void_p, _dp]
        L.orc_get_purkinje_activation.argtypes = [C.c_void_p, _dp]
        L.orc_get_pmj_region.argtypes = [C.c_void_p, C.c_int, _ip, C.c_int64]
        L.orc_get_pmj_region.restype = C.c_int64
        L.orc_set_bidomain.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, C.c_double,
                                       C.c_int]
        L.orc_get_phi_e.argtypes = [C.c_void_p, _dp]
        L.orc_bidomain_iterations.argtypes = [C.c_void_p, C.POINTER(C.c_int64), _dp]
        L.orc_bidomain_iterations.restype = C.c_int64
        L.orc_apply_flux.argtypes = [C.c_void_p, _dp, C.c_double, C.c_double, _dp]
        L.orc_gmres.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_double, C.c_int,
                                C.c_double, C.c_int, _dp]
        L.orc_gmres.restype = C.c_int64
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def n_slots(model: int) -> int:
    return lib().orc_model_n_slots(model)


def slot_names(model: int) -> list[str]:
    return [lib().orc_model_slot_name(model, i).decode() for i in range(n_slots(model))]


def model_init(model: int) -> np.ndarray:
    y = np.zeros(MAX_SLOTS)
    lib().orc_model_init(model, _d(y))
    return y[:n_slots(model)].copy()


def model_step(model: int, y: np.ndarray, dt: float, istim: float = 0.0,
               gscale=None) -> float:
    """Advance one cell one step in place (V not updated); returns I_ion."""
    buf = np.zeros(MAX_SLOTS)
    buf[:y.size] = y
    gs = None if gscale is None else np.ascontiguousarray(gscale, dtype=np.float64)
    r = lib().orc_model_step(model, _d(buf), dt, istim, None if gs is None else _d(gs))
    y[:] = buf[:y.size]
    return r


def single_cell(model: int, t_end: float, dt: float, stim_amp: float = -52.0,
                stim_dur: float = 1.0, stim_t0: float = 0.0, gscale=None):
    """Single-cell trace (no diffusion): returns (t, V) sampled every step."""
    y = model_init(model)
    n = int(round(t_end / dt))
    n0, nd = int(round(stim_t0 / dt)), int(round(stim_dur / dt))
    vs = np.empty(n + 1)
    vs[0] = y[0]
    for i in range(n):
        ist = stim_amp if n0 <= i < n0 + nd else 0.0
        iion = model_step(model, y, dt, ist, gscale)
        y[0] = y[0] + dt * (-iion - ist)
        vs[i + 1] = y[0]
    return np.arange(n + 1) * dt, vs


def detect_waveform(v: np.ndarray, dt: float, threshold: float = 0.0,
                    repol_frac: float = 0.9):
    v = np.ascontiguousarray(v, dtype=np.float64)
    ta, apd = C.c_double(), C.c_double()
    lib().orc_detect_waveform(_d(v), v.size, dt, threshold, repol_frac,
                              C.byref(ta), C.byref(apd))
    return ta.value, apd.value


class Sim:
    """Oracle tissue simulation of a meshgen.Workload (or explicit arrays)."""

    def __init__(self, w, model=None):
        self.w = w
        L = lib()
        self.nc, self.nn = w.n_tets, w.n_nodes
        self._xyz = np.ascontiguousarray(w.xyz, dtype=np.float64)
        self._tets = np.ascontiguousarray(w.tets, dtype=np.int32)
        self._fib = np.ascontiguousarray(w.fibre, dtype=np.float64)
        self._model = np.ascontiguousarray(w.model if model is None else model,
                                           dtype=np.uint8)
        self._scale = None if w.scale is None else np.ascontiguousarray(w.scale, np.float64)
        self.h = L.orc_create(self.nn, _d(self._xyz), self.nc,
                              self._tets.ctypes.data_as(_ip), _d(self._fib),
                              w.sigma_l, w.sigma_t,
                              None if self._scale is None else _d(self._scale),
                              self._model.ctypes.data_as(_up), w.dt, w.chi, w.cm)
        pk = getattr(w, "purkinje", None)
        self.np = 0
        if pk is not None:
            pxyz = np.ascontiguousarray(pk.xyz, np.float64)
            pe = np.ascontiguousarray(pk.edges, np.int32)
            self._escale = (None if pk.edge_scale is None
                            else np.ascontiguousarray(pk.edge_scale, np.float64))
            r = L.orc_set_purkinje(self.h, pxyz.shape[0], _d(pxyz), pe.shape[0],
                                   pe.ctypes.data_as(_ip),
                                   None if self._escale is None else _d(self._escale),
                                   pk.sigma, pk.model, pk.n_sub)
            assert r == 0
            self.np = pxyz.shape[0]
            for node in pk.pmj_nodes:
                L.orc_add_pmj(self.h, int(node), pk.pmj_radius, pk.delay_ortho,
                              pk.delay_anti, int(pk.two_way), pk.pmj_amp, pk.pmj_dur)
        for cj in getattr(w, "cell_junctions", []):
            assert L.orc_add_cell_junction(self.h, int(cj.cell), cj.radius, cj.delay_ortho,
                                           cj.delay_anti, int(cj.two_way), cj.amp, cj.dur) >= 0
        for st in w.stimuli:
            ids = np.ascontiguousarray(st.ids, dtype=np.int32)
            fn = L.orc_add_stimulus if st.domain == 0 else L.orc_add_purkinje_stimulus
            fn(self.h, ids.size, ids.ctypes.data_as(_ip), st.t0, st.dur, st.amp,
               st.period, st.count)
        if w.ionic_scale:
            gs = np.array([w.ionic_scale.get(k, 1.0) for k in ("GKr", "GKs", "GCaL", "GNa")])
            L.orc_set_ionic_scale(self.h, _d(gs))
        if getattr(w, "time_scheme", 0):
            assert L.orc_set_time_scheme(self.h, int(w.time_scheme)) == 0
        if getattr(w, "medium_substeps", None) is not None:
            assert L.orc_set_medium_substeps(self.h, int(w.medium_substeps)) == 0
        bd = getattr(w, "bidomain", None)
        if bd is not None:
            assert L.orc_set_bidomain(self.h, bd.sigma_el, bd.sigma_et, bd.restart, bd.tol,
                                      bd.max_iter) == 0

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def step(self, n: int):
        lib().orc_step(self.h, int(n))

    @property
    def step_index(self) -> int:
        return lib().orc_get_step(self.h)

    def set_step(self, n: int):
        lib().orc_set_step(self.h, int(n))

    def _vec(self, fn):
        out = np.empty(self.nc)
        fn(self.h, _d(out))
        return out

    def vm(self):
        return self._vec(lib().orc_get_vm)

    def activation(self):
        return self._vec(lib().orc_get_activation)

    def apd90(self):
        return self._vec(lib().orc_get_apd90)

    def purkinje_vm(self):
        out = np.empty(self.np)
        lib().orc_get_purkinje_vm(self.h, _d(out))
        return out

    def purkinje_activation(self):
        out = np.empty(self.np)
        lib().orc_get_purkinje_activation(self.h, _d(out))
        return out

    def medium_substeps(self) -> int:
        """Substeps per step of the 2D medium (1: it steps with the tissue)."""
        return lib().orc_medium_substeps(self.h)

    def purkinje_n_sub(self) -> int:
        return lib().orc_purkinje_n_sub(self.h)

    def pmj_region(self, k: int):
        out = np.empty(self.nc, np.int32)
        n = lib().orc_get_pmj_region(self.h, k, out.ctypes.data_as(_ip), out.size)
        return out[:n].copy()

    def phi_e(self):
        out = np.empty(self.nc)
        lib().orc_get_phi_e(self.h, _d(out))
        return out

    def bidomain_iterations(self):
        """(Arnoldi steps of the last solve, total, last relative residual)"""
        tot, rr = C.c_int64(), C.c_double()
        last = lib().orc_bidomain_iterations(self.h, C.byref(tot), C.byref(rr))
        return last, tot.value, rr.value

    def apply_flux(self, x, sl, st):
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.empty(self.nc)
        lib().orc_apply_flux(self.h, _d(x), sl, st, _d(out))
        return out

    def gmres(self, b, x0, sl, st, restart=30, tol=1e-10, max_iter=10000):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.array(x0, dtype=np.float64)
        rr = C.c_double()
        it = lib().orc_gmres(self.h, _d(b), _d(x), sl, st, restart, tol, max_iter, C.byref(rr))
        return x, it, rr.value

    def mean_vm(self) -> float:
        return lib().orc_mean_vm(self.h)

    def states(self) -> np.ndarray:
        out = np.empty((MAX_SLOTS, self.nc))
        lib().orc_get_states(self.h, _d(out))
        return out

    def set_states(self, st: np.ndarray):
        st = np.ascontiguousarray(st, dtype=np.float64)
        assert st.shape == (MAX_SLOTS, self.nc)
        lib().orc_set_states(self.h, _d(st))

    def detection(self) -> np.ndarray:
        """(4, n_tets): status, activation time, running max of V, repolarisation time."""
        out = np.empty((4, self.nc))
        lib().orc_get_detect_state(self.h, _d(out))
        return out

    def set_detection(self, d: np.ndarray):
        d = np.ascontiguousarray(d, dtype=np.float64)
        assert d.shape == (4, self.nc)
        lib().orc_set_detect_state(self.h, _d(d))

    def geometry(self):
        vol = np.empty(self.nc)
        S = np.empty((self.nc, 4, 3))
        nbr = np.empty((self.nc, 4), dtype=np.int32)
        lib().orc_geometry(self.h, _d(vol), _d(S), nbr.ctypes.data_as(_ip))
        return vol, S, nbr

    def node_values(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64)
        out = np.empty(self.nn)
        lib().orc_node_values(self.h, _d(v), _d(out))
        return out

    def gradients(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64)
        out = np.empty((self.nc, 3))
        lib().orc_cell_gradients(self.h, _d(v), _d(out))
        return out

    def apply_diffusion(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64)
        out = np.empty(self.nc)
        lib().orc_apply_diffusion(self.h, _d(v), _d(out))
        return out


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int):
    lib().orc_set_num_threads(int(n))
