"""Python binding of the gfx950 TTCF library (include/ttcf.h).

Argument marshalling only: every computation runs in the HIP kernels of libttcf.so. The
library is loaded from this package directory; if it is missing, importing this module
raises, because there is no other implementation to fall back to. PyTorch supplies the HIP
stream and, when ``use_torch_allocator()`` is called, the device allocator.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libttcf.so")

TTCF_OK, TTCF_EINVAL, TTCF_ENOMEM, TTCF_EDEVICE, TTCF_ESTATE, TTCF_EUNSTABLE = 0, -1, -2, -3, -4, -5
TTCF_ESCRATCH = -6
STATIC_SCRATCH_BYTES = 1 << 20
TTCF_WCA, TTCF_LJ = 0, 1
TTCF_PREC_FP64, TTCF_PREC_FP32_FORCES = 0, 1
TTCF_DAUGHTER_GIK, TTCF_DAUGHTER_NH = 0, 1
TTCF_OBS_PXY = 0
TTCF_OBS_WALL_STRESS = 1
TTCF_OBS_VPROFILE = 2
TTCF_OBS_N1, TTCF_OBS_N2, TTCF_OBS_ENERGY, TTCF_OBS_SLAB_PX = 3, 4, 5, 6
TTCF_OBS_JX = 7
TTCF_OBS_PEF_N1 = 8
TTCF_OBS_MIX_J = 9
TTCF_OBS_MIX_N1 = 10
TTCF_OBS_MIX_PXY = 11
TTCF_BULK_SLABS = 8
OBS_COLS = 3 + TTCF_BULK_SLABS  # columns of ttcf_export_observables
TTCF_CV_ESTIMATE = 1
TTCF_CV_CALIBRATE = 2


class TTCFError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        super().__init__(f"{where} failed with {code}: {detail}")
        self.code = code


class System(C.Structure):
    """ttcf_system of include/ttcf.h."""
    _fields_ = [("n_atoms", C.c_int32), ("potential", C.c_int32), ("box", C.c_double * 3),
                ("temperature", C.c_double), ("dt", C.c_double), ("r_cut", C.c_double),
                ("c_attr", C.c_double), ("u_shift", C.c_double), ("nh_tau", C.c_double),
                ("precision", C.c_int32), ("block_threads", C.c_int32),
                ("daughter_thermostat", C.c_int32)]


class Shape(C.Structure):
    _fields_ = [("variant", C.c_int32), ("threads", C.c_int32), ("kmax", C.c_int32),
                ("skin", C.c_double), ("ms_per_step", C.c_double), ("candidates", C.c_int32)]


class GraphDesc(C.Structure):
    _fields_ = [("mother", C.c_int32), ("n_replicas", C.c_int32),
                ("kicks", C.POINTER(C.c_double)), ("decorrelate_steps", C.c_int64),
                ("states_per_replica", C.c_int32), ("steps_between", C.c_int64),
                ("mapping_mask", C.c_uint32), ("gamma_dot", C.POINTER(C.c_double)),
                ("n_gamma", C.c_int32), ("n_steps", C.c_int32), ("max_replays", C.c_int32)]


class Channel(C.Structure):
    """ttcf_channel of include/ttcf.h."""
    _fields_ = [("n_fluid", C.c_int32), ("n_wall", C.c_int32), ("n_bins", C.c_int32),
                ("kmax", C.c_int32), ("lx", C.c_double), ("lz", C.c_double),
                ("y_extent", C.c_double), ("r_cut", C.c_double), ("c_ff", C.c_double),
                ("c_wf", C.c_double), ("k_spring", C.c_double), ("temperature", C.c_double),
                ("dt", C.c_double), ("nh_tau", C.c_double), ("bin_lo", C.c_double),
                ("bin_hi", C.c_double), ("skin", C.c_double)]


def make_channel(geom, skin: float = 0.0, kmax: int = 0) -> Channel:
    """From a ttcf_inputs.ChannelSystem."""
    return Channel(int(geom.n_fluid), int(geom.n_wall), int(geom.n_bins), int(kmax),
                   float(geom.lx), float(geom.lz), float(geom.y_extent), float(geom.rc),
                   float(geom.c_ff), float(geom.c_wf), float(geom.k_spring),
                   float(geom.temperature), float(geom.dt), float(geom.nh_tau),
                   float(geom.bin_lo), float(geom.bin_hi), float(skin))


def make_system(n_atoms: int, box, temperature: float = 0.722, dt: float = 0.0025,
                r_cut: float = 2.0 ** (1.0 / 6.0), c_attr: float = 1.0, u_shift: float | None = None,
                nh_tau: float = 0.25, precision: int = TTCF_PREC_FP32_FORCES,
                block_threads: int = 0, potential: int = TTCF_WCA,
                thermostat: int = TTCF_DAUGHTER_GIK) -> System:
    if np.isscalar(box):
        box = (float(box),) * 3
    if u_shift is None:
        u_shift = float("nan")  # the library's shift: phi(r_cut) = 0
    s = System()
    s.n_atoms = int(n_atoms)
    s.potential = int(potential)
    for a in range(3):
        s.box[a] = float(box[a])
    s.temperature = float(temperature)
    s.dt = float(dt)
    s.r_cut = float(r_cut)
    s.c_attr = float(c_attr)
    s.u_shift = float(u_shift)
    s.nh_tau = float(nh_tau)
    s.precision = int(precision)
    s.block_threads = int(block_threads)
    s.daughter_thermostat = int(thermostat)
    return s


_lib = None
_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p)
_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_keep = []


def lib():
    """The loaded libttcf.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU implementation of this library)")
    # torch ships a HIP runtime of its own: load it first, so that this library binds to the
    # same runtime (a second copy loaded earlier leaves torch's device discovery broken)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    D, I, L64, V = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.c_void_p
    S = C.POINTER(System)
    P = C.POINTER(C.c_void_p)
    F = C.POINTER(C.c_float)
    CH = C.POINTER(Channel)
    sig = {
        "ttcf_set_allocator": [_ALLOC, _FREE, V],
        "ttcf_init_mother": [P, S, D, D, C.c_int64, C.c_double, C.c_int64, V, I],
        "ttcf_spawn_daughters": [V, C.c_int32, C.c_int32, C.c_int64, C.c_uint32, D, C.c_int32,
                                 C.c_int32, L64],
        "ttcf_step": [V, C.c_int32],
        "ttcf_accumulate": [V, L64],
        "ttcf_response": [V, C.c_int32, C.c_double, C.c_int32, D, D, D, D, L64],
        "ttcf_sample_states": [V, C.c_int32, C.c_int32, C.c_int64],
        "ttcf_import_states": [V, C.c_int32, C.c_int32, D, D],
        "ttcf_export_states": [V, C.c_int32, C.c_int32, D, D],
        "ttcf_import_states_zeta": [V, C.c_int32, C.c_int32, D],
        "ttcf_acf": [V, D, C.c_int64, C.c_int32, C.c_double, D, I, D],
        "ttcf_response_modified": [V, C.c_double, C.c_int32, D, D, L64],
        "ttcf_observable_response_modified": [V, C.c_int32, C.c_double, C.c_int32, D, D, L64],
        "ttcf_record_observables": [V, C.c_int32],
        "ttcf_spawn_colour": [V, C.c_int32, C.c_int32, C.c_int64, C.c_uint32, D, C.c_int32,
                              C.c_int32, L64],
        "ttcf_export_observables": [V, C.c_int64, C.c_int32, C.c_int32, D],
        "ttcf_spawn_elongational": [V, C.c_int32, C.c_int32, C.c_int64, C.c_uint32, D,
                                    C.c_int32, C.c_int32, L64],
        "ttcf_spawn_mixed": [V, C.c_int32, C.c_int32, C.c_int64, C.c_uint32, D, D, C.c_int32,
                             C.c_int32, L64],
        "ttcf_mother_acf": [V, C.c_int32, C.c_int32, C.c_double, D, I, D],
        "ttcf_export_states_zeta": [V, C.c_int32, C.c_int32, D],
        "ttcf_export_mother": [V, C.c_int32, D, D, D, L64],
        "ttcf_record_mother": [V, C.c_int32, C.c_int64],
        "ttcf_export_mother_series": [V, C.c_int32, C.c_int64, D, L64],
        "ttcf_export_daughter": [V, C.c_int64, D, D, L64],
        "ttcf_export_series": [V, C.c_int64, C.c_int32, C.c_int32, D],
        "ttcf_daughter_health": [V, C.c_int64, I],
        "ttcf_debug_poison": [V, C.c_int64],
        "ttcf_debug_cell_list": [S, D, I, I, I, I, V],
        "ttcf_debug_pairs": [S, C.c_double, D, C.c_double, C.c_int64, I, I, L64, V],
        "ttcf_debug_forces": [S, C.c_double, D, D, D, V],
        "ttcf_cell_grid": [S, C.c_double, I, I, D],
        "ttcf_debug_pair_form": [S, C.c_double, C.c_int64, C.c_double, C.c_int32, D, I, I, I, I,
                                 C.c_int64, I, I, L64, D, D, V],
        "ttcf_pair_forces_static": [S, C.c_double, C.c_int64, C.c_double, C.c_int32, V, V, V,
                                    V],
        "ttcf_step_timing": [V, D, L64, C.c_int32],
        "ttcf_set_step_shape": [V, C.c_int32, C.c_int32, C.c_double, C.c_int32],
        "ttcf_cv_init": [V, C.c_int32, F, C.c_int64],
        "ttcf_cv_export_weights": [V, F, C.c_int64],
        "ttcf_cv_add_training": [V, C.c_int64, C.c_int32],
        "ttcf_cv_export_training": [V, C.c_int64, C.c_int32, F, F],
        "ttcf_cv_train": [V, C.c_int32, C.c_int32, C.c_double, I, D],
        "ttcf_cv_attach": [V, C.c_int64, C.c_int32, C.c_int32],
        "ttcf_cv_calibrate": [V, C.c_double, C.c_int32, D],
        "ttcf_cv_mean_term": [V, C.c_int32, C.c_int32, D, C.c_int64, C.c_int32, C.c_int32,
                              C.c_int64, C.c_double, L64],
        "ttcf_cv_response": [V, C.c_double, C.c_int32, D, D, D, D, D, D, L64],
        "ttcf_channel_create": [P, CH, D, D, D, V],
        "ttcf_channel_run_mother": [V, C.c_int64],
        "ttcf_channel_sample_states": [V, C.c_int32, C.c_int64],
        "ttcf_channel_sample_states_replicated": [V, C.c_int32, D, C.c_int64, C.c_int32,
                                                  C.c_int64],
        "ttcf_channel_import_states": [V, C.c_int32, D, D, D],
        "ttcf_channel_export_states": [V, C.c_int32, D, D, D],
        "ttcf_channel_export_mother": [V, D, D, D, L64],
        "ttcf_channel_spawn": [V, C.c_int32, C.c_uint32, D, C.c_int32, C.c_int32, L64],
        "ttcf_channel_step": [V, C.c_int32],
        "ttcf_channel_accumulate": [V, L64],
        "ttcf_channel_response": [V, C.c_int32, C.c_double, C.c_int32, D, D, D, D, L64],
        "ttcf_channel_export_series": [V, C.c_int64, C.c_int32, C.c_int32, D, D],
        "ttcf_channel_export_daughter": [V, C.c_int64, D, D, D],
        "ttcf_channel_daughter_health": [V, C.c_int64, I],
        "ttcf_channel_debug_forces": [CH, D, D, D, D, V],
        "ttcf_channel_step_timing": [V, D, L64, C.c_int32],
        "ttcf_sample_states_replicated": [V, C.c_int32, C.c_int32, D, C.c_int64, C.c_int32,
                                          C.c_int64],
        "ttcf_graph_create": [V, C.POINTER(GraphDesc), P],
        "ttcf_graph_launch": [V, C.c_int32],
        "ttcf_graph_create_multi": [V, C.POINTER(GraphDesc), C.c_int32, P],
        "ttcf_graph_replays": [V, I],
        "ttcf_autotune": [V, C.c_int32, C.c_int32, C.c_double, C.c_int32, C.POINTER(Shape)],
        "ttcf_autotune_export": [V, C.c_char_p, C.c_int64, L64],
        "ttcf_autotune_import": [V, C.c_char_p],
        "ttcf_mlp_forward": [V, F, C.c_int32, F],
        "ttcf_mlp_gradient": [V, F, F, C.c_int32, F],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int32
    L.ttcf_destroy.argtypes = [V]
    L.ttcf_destroy.restype = None
    L.ttcf_strerror.argtypes = [C.c_int32]
    L.ttcf_strerror.restype = C.c_char_p
    L.ttcf_last_error.argtypes = [V]
    L.ttcf_last_error.restype = C.c_char_p
    L.ttcf_graph_destroy.argtypes = [V]
    L.ttcf_graph_destroy.restype = None
    L.ttcf_channel_destroy.argtypes = [V]
    L.ttcf_channel_destroy.restype = None
    L.ttcf_channel_last_error.argtypes = [V]
    L.ttcf_channel_last_error.restype = C.c_char_p
    _lib = L
    return L


# names exported by include/ttcf.h (checked by the CPU test-suite)
EXPORTED = ["ttcf_set_allocator", "ttcf_init_mother", "ttcf_spawn_daughters", "ttcf_step",
            "ttcf_accumulate", "ttcf_response", "ttcf_destroy", "ttcf_strerror",
            "ttcf_last_error", "ttcf_sample_states", "ttcf_import_states", "ttcf_export_states", "ttcf_export_mother",
            "ttcf_record_mother", "ttcf_export_mother_series", "ttcf_export_daughter",
            "ttcf_export_series", "ttcf_daughter_health", "ttcf_debug_poison",
            "ttcf_debug_cell_list", "ttcf_debug_pairs", "ttcf_debug_forces", "ttcf_step_timing",
            "ttcf_cell_grid", "ttcf_debug_pair_form", "ttcf_pair_forces_static",
            "ttcf_set_step_shape", "ttcf_cv_init", "ttcf_cv_export_weights",
            "ttcf_cv_add_training", "ttcf_cv_export_training", "ttcf_cv_train", "ttcf_cv_attach", "ttcf_cv_calibrate", "ttcf_cv_mean_term",
            "ttcf_cv_response", "ttcf_mlp_forward", "ttcf_mlp_gradient",
            "ttcf_sample_states_replicated", "ttcf_channel_create", "ttcf_channel_destroy",
            "ttcf_channel_last_error", "ttcf_channel_run_mother", "ttcf_channel_sample_states",
            "ttcf_channel_sample_states_replicated",
            "ttcf_channel_import_states", "ttcf_channel_export_states",
            "ttcf_channel_export_mother", "ttcf_channel_spawn", "ttcf_channel_step",
            "ttcf_channel_accumulate", "ttcf_channel_response", "ttcf_channel_export_series",
            "ttcf_channel_export_daughter", "ttcf_channel_daughter_health",
            "ttcf_channel_debug_forces", "ttcf_channel_step_timing", "ttcf_autotune",
            "ttcf_autotune_export", "ttcf_autotune_import", "ttcf_graph_create",
            "ttcf_graph_launch", "ttcf_graph_replays", "ttcf_graph_destroy",
            "ttcf_graph_create_multi",
            "ttcf_import_states_zeta", "ttcf_export_states_zeta", "ttcf_acf", "ttcf_mother_acf",
            "ttcf_response_modified", "ttcf_observable_response_modified",
            "ttcf_record_observables", "ttcf_export_observables", "ttcf_spawn_colour",
            "ttcf_spawn_elongational", "ttcf_spawn_mixed"]

# network shape of the learned control variate (fixed by the library)
CV_IN = 64
CV_HIDDEN = 256


def cv_param_count(n_out: int) -> int:
    return CV_IN * CV_HIDDEN + CV_HIDDEN + CV_HIDDEN * CV_HIDDEN + CV_HIDDEN + CV_HIDDEN * n_out + n_out


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int32))


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(code: int, where: str, ctx=None):
    if code != TTCF_OK:
        detail = lib().ttcf_last_error(ctx).decode() if ctx else lib().ttcf_strerror(code).decode()
        raise TTCFError(code, where, detail)


def current_stream():
    """torch's current HIP stream handle (None: the default stream)."""
    import torch
    if torch.cuda.is_available():
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return None


def use_torch_allocator():
    """Route the library's device allocations through torch's caching allocator."""
    import torch

    def _alloc(nbytes, stream, user):
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                  stream if stream else None)

    def _free(ptr, user):
        torch.cuda.caching_allocator_delete(ptr)

    a, f = _ALLOC(_alloc), _FREE(_free)
    _keep.extend([a, f])
    _check(lib().ttcf_set_allocator(a, f, None), "ttcf_set_allocator")


# ----------------------------------------------------------------------------------------
# stateless kernels
# ----------------------------------------------------------------------------------------

def ttcf_cell_grid(sys: System, skin: float = 0.0):
    """(cells, list_cells, list_skin): the canonical cell grid and the pair-list form's list
    grid for `skin` (<= 0: automatic), as the library sizes them."""
    cells = np.zeros(3, np.int32)
    lcells = np.zeros(3, np.int32)
    ls = C.c_double(0.0)
    _check(lib().ttcf_cell_grid(C.byref(sys), float(skin), _ip(cells), _ip(lcells), C.byref(ls)),
           "ttcf_cell_grid")
    return cells, lcells, ls.value


def ttcf_debug_cell_list(sys: System, r, stream=None):
    r = _f64(r).ravel()
    n = sys.n_atoms
    dims = np.zeros(3, np.int32)
    ncell = int(np.prod(ttcf_cell_grid(sys)[0]))
    cell_of = np.zeros(n, np.int32)
    order = np.zeros(n, np.int32)
    start = np.zeros(ncell + 1, np.int32)
    _check(lib().ttcf_debug_cell_list(C.byref(sys), _dp(r), _ip(dims), _ip(cell_of), _ip(order),
                                      _ip(start), stream), "ttcf_debug_cell_list")
    return dims, cell_of, order, start


def ttcf_debug_pairs(sys: System, r, dxle: float = 0.0, rlist: float | None = None, stream=None):
    r = _f64(r).ravel()
    cap = 64 * sys.n_atoms
    pi = np.zeros(cap, np.int32)
    pj = np.zeros(cap, np.int32)
    cnt = C.c_int64(0)
    rl = sys.r_cut if rlist is None else float(rlist)
    _check(lib().ttcf_debug_pairs(C.byref(sys), float(dxle), _dp(r), rl, cap, _ip(pi), _ip(pj),
                                  C.byref(cnt), stream), "ttcf_debug_pairs")
    if cnt.value < 0:
        raise TTCFError(TTCF_EINVAL, "ttcf_debug_pairs", "capacity too small")
    return pi[:cnt.value].copy(), pj[:cnt.value].copy()


def ttcf_debug_pair_form(sys: System, r, gamma_dot: float = 0.0, kstep: int = 0,
                         skin: float = 0.0, kcap: int = 0, stream=None):
    """The pair-list form's own list build and force pass on positions r. Returns a dict:
    dims (list grid), cell_of, order, start, pairs (pi, pj: atom ids, pi < pj, sorted), f
    (3, n) forces as the integrator uses them, w_xy, dxle (the offset used), rlist, close
    (a pair inside the fixed-point force range's guard radius), overflow (capacity)."""
    r = _f64(r).ravel()
    n = sys.n_atoms
    _, lc, _ = ttcf_cell_grid(sys, skin)
    ncell = int(np.prod(lc))
    dims = np.zeros(3, np.int32)
    cell_of = np.zeros(n, np.int32)
    order = np.zeros(n, np.int32)
    start = np.zeros(ncell + 1, np.int32)
    cap = 64 * n
    pi = np.zeros(cap, np.int32)
    pj = np.zeros(cap, np.int32)
    cnt = C.c_int64(0)
    f = np.zeros(3 * n)
    out = np.zeros(4)
    code = lib().ttcf_debug_pair_form(C.byref(sys), float(gamma_dot), int(kstep), float(skin),
                                      int(kcap), _dp(r), _ip(dims), _ip(cell_of), _ip(order),
                                      _ip(start), cap, _ip(pi), _ip(pj), C.byref(cnt), _dp(f),
                                      _dp(out), stream)
    if code not in (TTCF_OK, TTCF_EUNSTABLE):
        _check(code, "ttcf_debug_pair_form")
    if cnt.value < 0:
        raise TTCFError(TTCF_EINVAL, "ttcf_debug_pair_form", "capacity too small")
    k = cnt.value
    return dict(dims=dims, cell_of=cell_of, order=order, start=start,
                pairs=(pi[:k].copy(), pj[:k].copy()), f=f.reshape(3, n), w_xy=out[0],
                dxle=out[1], rlist=out[2], close=bool(out[3] != 0.0),
                overflow=code == TTCF_EUNSTABLE)


def ttcf_pair_forces_static(sys: System, gamma_dot: float, kstep: int, skin: float, kcap: int,
                            r_dev: int, f_dev: int, out_dev: int, stream=None) -> int:
    """The allocation-free form of ttcf_debug_pair_form's force pass: device pointers r_dev
    (3n FP64 positions), f_dev (3n FP64 forces out), out_dev (4 FP64 out: W_xy, close flag,
    offset used, overflow flag), enqueued on `stream` (a HIP stream handle or None). Returns
    the status (TTCF_ESCRATCH when the input outgrows the static scratch); raises on any
    other error."""
    code = lib().ttcf_pair_forces_static(C.byref(sys), float(gamma_dot), int(kstep),
                                         float(skin), int(kcap), r_dev, f_dev, out_dev, stream)
    if code not in (TTCF_OK, TTCF_ESCRATCH):
        _check(code, "ttcf_pair_forces_static")
    return code


def ttcf_debug_forces(sys: System, r, dxle: float = 0.0, stream=None):
    r = _f64(r).ravel()
    f = np.zeros(3 * sys.n_atoms)
    out = np.zeros(2)
    _check(lib().ttcf_debug_forces(C.byref(sys), float(dxle), _dp(r), _dp(f), _dp(out), stream),
           "ttcf_debug_forces")
    return f.reshape(3, sys.n_atoms), out[0], out[1]


# ----------------------------------------------------------------------------------------
# context
# ----------------------------------------------------------------------------------------

class Context:
    """One ttcf_ctx: mothers, live daughters and accumulated start-state groups."""

    def __init__(self, stream=None):
        self._ctx = C.c_void_p(None)
        self._stream = stream
        self.systems = []
        self._graphs = []

    @property
    def handle(self):
        return self._ctx

    def close(self):
        for g in list(self._graphs):
            g.destroy()
        if self._ctx:
            lib().ttcf_destroy(self._ctx)
            self._ctx = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- the five calls
    def ttcf_init_mother(self, sys: System, r0, p0, n_equil: int, n_melt: int = 0,
                         t_melt: float = 0.0) -> int:
        r0 = _f64(r0).ravel()
        p0 = _f64(p0).ravel()
        assert r0.size == 3 * sys.n_atoms and p0.size == 3 * sys.n_atoms
        mid = C.c_int32(-1)
        code = lib().ttcf_init_mother(C.byref(self._ctx), C.byref(sys), _dp(r0), _dp(p0),
                                      int(n_melt), float(t_melt), int(n_equil), self._stream,
                                      C.byref(mid))
        _check(code, "ttcf_init_mother", self._ctx if self._ctx else None)
        self.systems.append(sys)
        return mid.value

    def ttcf_spawn_daughters(self, mother: int, n_states: int, steps_between: int,
                             gamma_dot, n_steps: int, mapping_mask: int = 0xF) -> int:
        g = _f64(np.atleast_1d(gamma_dot))
        first = C.c_int64(-1)
        _check(lib().ttcf_spawn_daughters(self._ctx, int(mother), int(n_states), int(steps_between),
                                          int(mapping_mask), _dp(g), int(g.size), int(n_steps),
                                          C.byref(first)), "ttcf_spawn_daughters", self._ctx)
        return first.value

    def ttcf_spawn_colour(self, mother: int, n_states: int, steps_between: int, field,
                          n_steps: int, mapping_mask: int = 0xF) -> int:
        """Colour-field daughters (field strengths F_e in place of shear rates)."""
        g = _f64(np.atleast_1d(field))
        first = C.c_int64(-1)
        _check(lib().ttcf_spawn_colour(self._ctx, int(mother), int(n_states), int(steps_between),
                                       int(mapping_mask), _dp(g), int(g.size), int(n_steps),
                                       C.byref(first)), "ttcf_spawn_colour", self._ctx)
        return first.value

    def ttcf_spawn_elongational(self, mother: int, n_states: int, steps_between: int, rate,
                                n_steps: int, mapping_mask: int = 0xF) -> int:
        """Planar-elongation daughters (elongation rates in place of shear rates)."""
        g = _f64(np.atleast_1d(rate))
        first = C.c_int64(-1)
        _check(lib().ttcf_spawn_elongational(self._ctx, int(mother), int(n_states),
                                             int(steps_between), int(mapping_mask), _dp(g),
                                             int(g.size), int(n_steps), C.byref(first)),
               "ttcf_spawn_elongational", self._ctx)
        return first.value

    def ttcf_spawn_mixed(self, mother: int, n_states: int, steps_between: int, erate, srate,
                         n_steps: int, mapping_mask: int = 0xF) -> int:
        """Mixed-flow daughters (u_x = erate x + srate y, u_y = -erate y), one rate pair for
        all states or one per state."""
        e = _f64(np.atleast_1d(erate))
        g = _f64(np.atleast_1d(srate))
        if e.size != g.size:
            raise ValueError("erate and srate need the same length")
        first = C.c_int64(-1)
        _check(lib().ttcf_spawn_mixed(self._ctx, int(mother), int(n_states), int(steps_between),
                                      int(mapping_mask), _dp(e), _dp(g), int(e.size),
                                      int(n_steps), C.byref(first)), "ttcf_spawn_mixed",
               self._ctx)
        return first.value

    def ttcf_step(self, n_steps: int):
        _check(lib().ttcf_step(self._ctx, int(n_steps)), "ttcf_step", self._ctx)

    def ttcf_accumulate(self) -> int:
        groups = C.c_int64(0)
        _check(lib().ttcf_accumulate(self._ctx, C.byref(groups)), "ttcf_accumulate", self._ctx)
        return groups.value

    def ttcf_response(self, n_t: int, gamma_dot_filter: float, observable: int = TTCF_OBS_PXY):
        """(ttcf_mean, ttcf_se, dav_mean, dav_se, n_states); TTCF_OBS_SLAB_PX gives arrays of
        shape (n_t, TTCF_BULK_SLABS)."""
        cols = TTCF_BULK_SLABS if observable == TTCF_OBS_SLAB_PX else 1
        out = [np.zeros(n_t * cols) for _ in range(4)]
        used = C.c_int64(0)
        _check(lib().ttcf_response(self._ctx, int(observable), float(gamma_dot_filter), int(n_t),
                                   *[_dp(o) for o in out], C.byref(used)), "ttcf_response",
               self._ctx)
        if cols > 1:
            out = [o.reshape(n_t, cols) for o in out]
        return out[0], out[1], out[2], out[3], used.value

    def ttcf_response_modified(self, n_t: int, gamma_dot_filter: float,
                               observable: int = TTCF_OBS_PXY):
        """Eq. (corr_modified): (mean, jackknife se, n_states)."""
        cols = TTCF_BULK_SLABS if observable == TTCF_OBS_SLAB_PX else 1
        m = np.zeros(n_t * cols)
        se = np.zeros(n_t * cols)
        used = C.c_int64(0)
        if observable == TTCF_OBS_PXY:
            rc = lib().ttcf_response_modified(self._ctx, float(gamma_dot_filter), int(n_t), _dp(m),
                                              _dp(se), C.byref(used))
        else:
            rc = lib().ttcf_observable_response_modified(self._ctx, int(observable),
                                                         float(gamma_dot_filter), int(n_t),
                                                         _dp(m), _dp(se), C.byref(used))
        _check(rc, "ttcf_response_modified", self._ctx)
        if cols > 1:
            m, se = m.reshape(n_t, cols), se.reshape(n_t, cols)
        return m, se, used.value

    def ttcf_record_observables(self, on: bool = True):
        _check(lib().ttcf_record_observables(self._ctx, int(bool(on))), "ttcf_record_observables",
               self._ctx)

    def ttcf_export_observables(self, first: int, count: int, n_t: int):
        """(count, n_t, OBS_COLS): P_xx - P_yy, P_yy - P_zz, (K + U)/N, slab momentum profile."""
        out = np.zeros((count, n_t, OBS_COLS))
        _check(lib().ttcf_export_observables(self._ctx, int(first), int(count), int(n_t),
                                             _dp(out)), "ttcf_export_observables", self._ctx)
        return out

    # ---- inspection hooks
    def ttcf_sample_states(self, mother: int, n_states: int, steps_between: int):
        _check(lib().ttcf_sample_states(self._ctx, int(mother), int(n_states), int(steps_between)),
               "ttcf_sample_states", self._ctx)

    def ttcf_import_states(self, mother: int, r, p):
        r = _f64(r)
        p = _f64(p)
        ns = r.shape[0]
        _check(lib().ttcf_import_states(self._ctx, int(mother), ns, _dp(r), _dp(p)),
               "ttcf_import_states", self._ctx)

    def ttcf_sample_states_replicated(self, mother: int, n_replicas: int, kicks,
                                      decorrelate_steps: int, states_per_replica: int,
                                      steps_between: int):
        k = None if kicks is None else _f64(kicks).ravel()
        _check(lib().ttcf_sample_states_replicated(self._ctx, int(mother), int(n_replicas), _dp(k),
                                                   int(decorrelate_steps), int(states_per_replica),
                                                   int(steps_between)),
               "ttcf_sample_states_replicated", self._ctx)

    def ttcf_acf(self, series, max_lag: int, threshold: float = 0.05):
        """(acf[0..max_lag), first lag below threshold, integrated correlation time)."""
        x = _f64(np.ravel(series))
        out = np.zeros(max_lag)
        fb = C.c_int32(0)
        tau = C.c_double(0.0)
        _check(lib().ttcf_acf(self._ctx, _dp(x), int(x.size), int(max_lag), float(threshold),
                              _dp(out), C.byref(fb), C.byref(tau)), "ttcf_acf", self._ctx)
        return out, fb.value, tau.value

    def ttcf_mother_acf(self, mother: int, max_lag: int, threshold: float = 0.05):
        out = np.zeros(max_lag)
        fb = C.c_int32(0)
        tau = C.c_double(0.0)
        _check(lib().ttcf_mother_acf(self._ctx, int(mother), int(max_lag), float(threshold),
                                     _dp(out), C.byref(fb), C.byref(tau)), "ttcf_mother_acf",
               self._ctx)
        return out, fb.value, tau.value

    def ttcf_import_states_zeta(self, mother: int, zeta):
        z = _f64(np.atleast_1d(zeta))
        _check(lib().ttcf_import_states_zeta(self._ctx, int(mother), int(z.size), _dp(z)),
               "ttcf_import_states_zeta", self._ctx)

    def ttcf_export_states_zeta(self, mother: int, n_states: int):
        z = np.zeros(n_states)
        _check(lib().ttcf_export_states_zeta(self._ctx, int(mother), int(n_states), _dp(z)),
               "ttcf_export_states_zeta", self._ctx)
        return z

    def ttcf_export_states(self, mother: int, n_states: int):
        n = self.systems[mother].n_atoms
        r = np.zeros((n_states, 3 * n))
        p = np.zeros((n_states, 3 * n))
        _check(lib().ttcf_export_states(self._ctx, int(mother), int(n_states), _dp(r), _dp(p)),
               "ttcf_export_states", self._ctx)
        return r, p

    def ttcf_export_mother(self, mother: int):
        n = self.systems[mother].n_atoms
        r = np.zeros(3 * n)
        p = np.zeros(3 * n)
        z = np.zeros(1)
        steps = C.c_int64(0)
        _check(lib().ttcf_export_mother(self._ctx, int(mother), _dp(r), _dp(p), _dp(z),
                                        C.byref(steps)), "ttcf_export_mother", self._ctx)
        return r, p, float(z[0]), steps.value

    def ttcf_record_mother(self, mother: int, capacity: int):
        _check(lib().ttcf_record_mother(self._ctx, int(mother), int(capacity)),
               "ttcf_record_mother", self._ctx)

    def ttcf_export_mother_series(self, mother: int, n: int):
        out = np.zeros(n)
        cnt = C.c_int64(0)
        _check(lib().ttcf_export_mother_series(self._ctx, int(mother), int(n), _dp(out),
                                               C.byref(cnt)), "ttcf_export_mother_series", self._ctx)
        return out[:min(n, cnt.value)]

    def ttcf_export_daughter(self, daughter: int, n_atoms: int):
        r = np.zeros(3 * n_atoms)
        p = np.zeros(3 * n_atoms)
        k = C.c_int64(0)
        _check(lib().ttcf_export_daughter(self._ctx, int(daughter), _dp(r), _dp(p), C.byref(k)),
               "ttcf_export_daughter", self._ctx)
        return r, p, k.value

    def ttcf_export_series(self, first: int, count: int, n_t: int):
        out = np.zeros((count, n_t))
        _check(lib().ttcf_export_series(self._ctx, int(first), int(count), int(n_t), _dp(out)),
               "ttcf_export_series", self._ctx)
        return out

    def ttcf_daughter_health(self, daughter: int) -> int:
        h = C.c_int32(0)
        _check(lib().ttcf_daughter_health(self._ctx, int(daughter), C.byref(h)),
               "ttcf_daughter_health", self._ctx)
        return h.value

    def ttcf_debug_poison(self, daughter: int):
        _check(lib().ttcf_debug_poison(self._ctx, int(daughter)), "ttcf_debug_poison", self._ctx)

    def ttcf_set_step_shape(self, variant: int = 0, threads: int = 0, skin: float = 0.0,
                            kmax: int = 0):
        """variant 0 auto, 1 cell list, 2 neighbour list (see include/ttcf.h)."""
        _check(lib().ttcf_set_step_shape(self._ctx, int(variant), int(threads), float(skin),
                                         int(kmax)), "ttcf_set_step_shape", self._ctx)

    def ttcf_step_timing(self, reset: bool = False):
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        _check(lib().ttcf_step_timing(self._ctx, C.byref(ms), C.byref(n), int(reset)),
               "ttcf_step_timing", self._ctx)
        return ms.value, n.value

    def ttcf_graph_create(self, mother: int, states_per_replica: int, steps_between: int,
                          gamma_dot, n_steps: int, max_replays: int, n_replicas: int = 0,
                          kicks=None, decorrelate_steps: int = 0, mapping_mask: int = 0xF):
        """Records one batch cycle of ``mother`` as a HIP graph (see include/ttcf.h)."""
        g = _f64(np.atleast_1d(gamma_dot))
        k = None if kicks is None else _f64(kicks).ravel()
        d = GraphDesc(int(mother), int(n_replicas), _dp(k), int(decorrelate_steps),
                      int(states_per_replica), int(steps_between), int(mapping_mask), _dp(g),
                      int(g.size), int(n_steps), int(max_replays))
        h = C.c_void_p(None)
        _check(lib().ttcf_graph_create(self._ctx, C.byref(d), C.byref(h)), "ttcf_graph_create",
               self._ctx)
        gr = Graph(self, h)
        self._graphs.append(gr)
        return gr

    def ttcf_graph_create_multi(self, parts, n_steps: int, max_replays: int):
        """Records one batch cycle over several mothers as one HIP graph (see include/ttcf.h).
        parts: dicts with keys mother, states_per_replica, steps_between, gamma_dot and
        optionally n_replicas, kicks, decorrelate_steps, mapping_mask."""
        keep = []
        arr = (GraphDesc * len(parts))()
        for k, p in enumerate(parts):
            g = _f64(np.atleast_1d(p["gamma_dot"]))
            kk = p.get("kicks")
            kk = None if kk is None else _f64(kk).ravel()
            keep += [g, kk]
            arr[k] = GraphDesc(int(p["mother"]), int(p.get("n_replicas", 0)), _dp(kk),
                               int(p.get("decorrelate_steps", 0)), int(p["states_per_replica"]),
                               int(p["steps_between"]), int(p.get("mapping_mask", 0xF)), _dp(g),
                               int(g.size), int(n_steps), int(max_replays))
        h = C.c_void_p(None)
        _check(lib().ttcf_graph_create_multi(self._ctx, arr, len(parts), C.byref(h)),
               "ttcf_graph_create_multi", self._ctx)
        gr = Graph(self, h)
        self._graphs.append(gr)
        return gr

    def ttcf_autotune(self, mother: int, n_states: int = 0, gamma_dot: float = 1e-3,
                      probe_steps: int = 200) -> dict:
        """Times the candidate step shapes on probe daughters of ``mother`` and caches the
        fastest for its system (see include/ttcf.h)."""
        out = Shape()
        _check(lib().ttcf_autotune(self._ctx, int(mother), int(n_states), float(gamma_dot),
                                   int(probe_steps), C.byref(out)), "ttcf_autotune", self._ctx)
        return {"variant": out.variant, "threads": out.threads, "kmax": out.kmax,
                "skin": out.skin, "ms_per_step": out.ms_per_step, "candidates": out.candidates}

    def ttcf_autotune_export(self) -> str:
        n = C.c_int64(0)
        _check(lib().ttcf_autotune_export(self._ctx, None, 0, C.byref(n)), "ttcf_autotune_export",
               self._ctx)
        buf = C.create_string_buffer(n.value + 1)
        _check(lib().ttcf_autotune_export(self._ctx, buf, n.value + 1, C.byref(n)),
               "ttcf_autotune_export", self._ctx)
        return buf.value.decode()

    def ttcf_autotune_import(self, text: str):
        _check(lib().ttcf_autotune_import(self._ctx, text.encode()), "ttcf_autotune_import",
               self._ctx)

    # ---- learned control variate
    def ttcf_cv_init(self, n_out: int, weights):
        w = _f32(weights).ravel()
        _check(lib().ttcf_cv_init(self._ctx, int(n_out), _fp(w), int(w.size)), "ttcf_cv_init",
               self._ctx)
        self.cv_out = int(n_out)

    def ttcf_cv_export_weights(self):
        w = np.zeros(cv_param_count(self.cv_out), np.float32)
        _check(lib().ttcf_cv_export_weights(self._ctx, _fp(w), int(w.size)),
               "ttcf_cv_export_weights", self._ctx)
        return w

    def ttcf_cv_add_training(self, first: int, count: int):
        _check(lib().ttcf_cv_add_training(self._ctx, int(first), int(count)),
               "ttcf_cv_add_training", self._ctx)

    def ttcf_cv_export_training(self, first_row: int, count: int):
        x = np.zeros((count, CV_IN), np.float32)
        t = np.zeros((count, self.cv_out), np.float32)
        _check(lib().ttcf_cv_export_training(self._ctx, int(first_row), int(count), _fp(x), _fp(t)),
               "ttcf_cv_export_training", self._ctx)
        return x, t

    def ttcf_cv_train(self, epochs: int, batch: int, lr: float, order=None):
        """order: (epochs, rows) int32 permutations or None. Returns the per-epoch losses."""
        o = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
        loss = np.zeros(max(int(epochs), 1))
        _check(lib().ttcf_cv_train(self._ctx, int(epochs), int(batch), float(lr), _ip(o),
                                   _dp(loss)), "ttcf_cv_train", self._ctx)
        return loss[:int(epochs)]

    def ttcf_cv_attach(self, first: int, count: int, role: int = 1):
        """role 1 (TTCF_CV_ESTIMATE) or 2 (TTCF_CV_CALIBRATE)."""
        _check(lib().ttcf_cv_attach(self._ctx, int(first), int(count), int(role)),
               "ttcf_cv_attach", self._ctx)

    def ttcf_cv_calibrate(self, n_t: int, gamma_dot_filter: float):
        beta = np.zeros(n_t)
        _check(lib().ttcf_cv_calibrate(self._ctx, float(gamma_dot_filter), int(n_t), _dp(beta)),
               "ttcf_cv_calibrate", self._ctx)
        return beta

    def ttcf_cv_mean_term(self, mother: int, n_replicas: int, kicks, decorrelate_steps: int,
                          rounds: int, states_per_replica: int, steps_between: int,
                          gamma_dot: float) -> int:
        k = None if kicks is None else _f64(kicks).ravel()
        out = C.c_int64(0)
        _check(lib().ttcf_cv_mean_term(self._ctx, int(mother), int(n_replicas), _dp(k),
                                       int(decorrelate_steps), int(rounds),
                                       int(states_per_replica), int(steps_between),
                                       float(gamma_dot), C.byref(out)),
               "ttcf_cv_mean_term", self._ctx)
        return out.value

    def ttcf_cv_response(self, n_t: int, gamma_dot_filter: float):
        """(cv_mean, cv_se, plain_mean, plain_se, mu_h, mu_h_se, n_states)."""
        out = [np.zeros(n_t) for _ in range(6)]
        used = C.c_int64(0)
        _check(lib().ttcf_cv_response(self._ctx, float(gamma_dot_filter), int(n_t),
                                      *[_dp(o) for o in out], C.byref(used)),
               "ttcf_cv_response", self._ctx)
        return (*out, used.value)

    def ttcf_mlp_forward(self, x):
        x = _f32(x)
        y = np.zeros((x.shape[0], self.cv_out), np.float32)
        _check(lib().ttcf_mlp_forward(self._ctx, _fp(x), int(x.shape[0]), _fp(y)),
               "ttcf_mlp_forward", self._ctx)
        return y

    def ttcf_mlp_gradient(self, x, target):
        x = _f32(x)
        t = _f32(target)
        g = np.zeros(cv_param_count(self.cv_out), np.float32)
        _check(lib().ttcf_mlp_gradient(self._ctx, _fp(x), _fp(t), int(x.shape[0]), _fp(g)),
               "ttcf_mlp_gradient", self._ctx)
        return g


# ----------------------------------------------------------------------------------------
# the confined channel
# ----------------------------------------------------------------------------------------

class Graph:
    """A captured batch cycle; destroyed with its context at the latest."""

    def __init__(self, ctx: Context, handle):
        self._owner = ctx
        self._h = handle

    def launch(self, n_replays: int = 1):
        _check(lib().ttcf_graph_launch(self._h, int(n_replays)), "ttcf_graph_launch",
               self._owner._ctx)

    @property
    def replays(self) -> int:
        r = C.c_int32(0)
        _check(lib().ttcf_graph_replays(self._h, C.byref(r)), "ttcf_graph_replays",
               self._owner._ctx)
        return r.value

    def destroy(self):
        if self._h:
            lib().ttcf_graph_destroy(self._h)
            self._h = C.c_void_p(None)
            if self in self._owner._graphs:
                self._owner._graphs.remove(self)


def ttcf_channel_debug_forces(ch: Channel, r, lattice, stream=None):
    """(f (3n,), out[5]) of one configuration at the given lattice sites."""
    r = _f64(r).ravel()
    lat = _f64(lattice).ravel()
    n = ch.n_fluid + ch.n_wall
    f = np.zeros(3 * n)
    out = np.zeros(5)
    code = lib().ttcf_channel_debug_forces(C.byref(ch), _dp(r), _dp(lat), _dp(f), _dp(out), stream)
    if code != 0:
        detail = lib().ttcf_channel_last_error(None)
        raise TTCFError(code, "ttcf_channel_debug_forces", detail.decode() if detail else "")
    return f, out


class ChannelContext:
    """One ttcf_channel_ctx: the channel mother, its stored states, daughters and rows.
    stream: a HIP stream handle (e.g. current_stream()), or None for the default stream."""

    def __init__(self, ch: Channel, r0, p0, lattice, stream=None):
        self.ch = ch
        self.n = ch.n_fluid + ch.n_wall
        self.n_obs = 1 + ch.n_bins
        self._ctx = C.c_void_p(None)
        r0 = _f64(r0).ravel()
        p0 = _f64(p0).ravel()
        lat = _f64(lattice).ravel()
        assert r0.size == 3 * self.n and p0.size == 3 * self.n and lat.size == 3 * ch.n_wall
        code = lib().ttcf_channel_create(C.byref(self._ctx), C.byref(ch), _dp(r0), _dp(p0),
                                         _dp(lat), stream)
        if code != 0:
            detail = lib().ttcf_channel_last_error(None)
            raise TTCFError(code, "ttcf_channel_create", detail.decode() if detail else "")

    def _chk(self, code, where):
        if code != 0:
            detail = lib().ttcf_channel_last_error(self._ctx)
            raise TTCFError(code, where, detail.decode() if detail else "")

    def close(self):
        if self._ctx:
            lib().ttcf_channel_destroy(self._ctx)
            self._ctx = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def run_mother(self, n_steps: int):
        self._chk(lib().ttcf_channel_run_mother(self._ctx, int(n_steps)), "ttcf_channel_run_mother")

    def sample_states(self, n_states: int, steps_between: int):
        self._chk(lib().ttcf_channel_sample_states(self._ctx, int(n_states), int(steps_between)),
                  "ttcf_channel_sample_states")

    def sample_states_replicated(self, n_replicas: int, kicks, decorrelate_steps: int,
                                 states_per_replica: int, steps_between: int):
        """Start states from n_replicas kicked copies of the mother (kicks: (R, 3n) or None)."""
        k = None if kicks is None else _f64(kicks).ravel()
        self._chk(lib().ttcf_channel_sample_states_replicated(
            self._ctx, int(n_replicas), _dp(k), int(decorrelate_steps), int(states_per_replica),
            int(steps_between)), "ttcf_channel_sample_states_replicated")

    def import_states(self, r, p, zeta):
        r = _f64(r)
        p = _f64(p)
        z = _f64(zeta)
        self._chk(lib().ttcf_channel_import_states(self._ctx, int(r.shape[0]), _dp(r), _dp(p), _dp(z)),
                  "ttcf_channel_import_states")

    def export_states(self, n_states: int):
        r = np.zeros((n_states, 3 * self.n))
        p = np.zeros((n_states, 3 * self.n))
        z = np.zeros(n_states)
        self._chk(lib().ttcf_channel_export_states(self._ctx, int(n_states), _dp(r), _dp(p), _dp(z)),
                  "ttcf_channel_export_states")
        return r, p, z

    def export_mother(self):
        r = np.zeros(3 * self.n)
        p = np.zeros(3 * self.n)
        z = np.zeros(1)
        steps = C.c_int64(0)
        self._chk(lib().ttcf_channel_export_mother(self._ctx, _dp(r), _dp(p), _dp(z), C.byref(steps)),
                  "ttcf_channel_export_mother")
        return r, p, float(z[0]), steps.value

    def spawn(self, n_states: int, v, n_steps: int, mapping_mask: int = 0xF) -> int:
        vv = _f64(np.atleast_1d(v))
        first = C.c_int64(-1)
        self._chk(lib().ttcf_channel_spawn(self._ctx, int(n_states), int(mapping_mask), _dp(vv),
                                           int(vv.size), int(n_steps), C.byref(first)),
                  "ttcf_channel_spawn")
        return first.value

    def step(self, n_steps: int):
        self._chk(lib().ttcf_channel_step(self._ctx, int(n_steps)), "ttcf_channel_step")

    def accumulate(self) -> int:
        g = C.c_int64(0)
        self._chk(lib().ttcf_channel_accumulate(self._ctx, C.byref(g)), "ttcf_channel_accumulate")
        return g.value

    def response(self, observable: int, v_filter: float, n_t: int):
        """(ttcf, ttcf_se, dav, dav_se, n_states); arrays (n_t,) or (n_t, n_bins)."""
        cols = 1 if observable == TTCF_OBS_WALL_STRESS else self.ch.n_bins
        out = [np.zeros(n_t * cols) for _ in range(4)]
        used = C.c_int64(0)
        self._chk(lib().ttcf_channel_response(self._ctx, int(observable), float(v_filter), int(n_t),
                                              *[_dp(o) for o in out], C.byref(used)),
                  "ttcf_channel_response")
        shape = (n_t,) if cols == 1 else (n_t, cols)
        return (*[o.reshape(shape) for o in out], used.value)

    def export_series(self, first: int, count: int, n_t: int):
        obs = np.zeros((count, n_t, self.n_obs))
        s0 = np.zeros(count)
        self._chk(lib().ttcf_channel_export_series(self._ctx, int(first), int(count), int(n_t),
                                                   _dp(obs), _dp(s0)), "ttcf_channel_export_series")
        return obs, s0

    def export_daughter(self, daughter: int):
        r = np.zeros(3 * self.n)
        p = np.zeros(3 * self.n)
        z = np.zeros(1)
        self._chk(lib().ttcf_channel_export_daughter(self._ctx, int(daughter), _dp(r), _dp(p), _dp(z)),
                  "ttcf_channel_export_daughter")
        return r, p, float(z[0])

    def daughter_health(self, daughter: int) -> int:
        h = C.c_int32(0)
        self._chk(lib().ttcf_channel_daughter_health(self._ctx, int(daughter), C.byref(h)),
                  "ttcf_channel_daughter_health")
        return h.value

    def step_timing(self, reset: bool = False):
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        self._chk(lib().ttcf_channel_step_timing(self._ctx, C.byref(ms), C.byref(n), int(reset)),
                  "ttcf_channel_step_timing")
        return ms.value, n.value
