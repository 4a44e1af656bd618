"""FP64 CPU oracle for the TTCF daughter path of arxiv 2312.02990 (TTCF4LAMMPS).

TEST INFRASTRUCTURE: only the test-suite, the smoke check and the benchmark's CPU-baseline
leg import this module. The GPU library shares no code with it.

Two layers:
  * ctypes bindings of ``libttcf_oracle.so`` (dynamics, forces, cell lists; plain C, FP64);
  * the TTCF / direct-average estimators and the Green-Kubo integral written with numpy
    in FP64, each following the equation it cites.

Sign convention: ``vpxy`` is V * P_xy with P_xy the pressure-tensor component. The paper's
Eq. (TTCF1) writes Omega = +gamma_dot V P_xy / k_B T with P_xy read as a shear stress; in the
pressure-tensor convention the same dissipation function is Omega = -gamma_dot V P_xy / T,
which is what the adiabatic energy balance dH0/dt = -gamma_dot V P_xy gives (the paper defines
Omega as beta times the adiabatic rate of change of the internal energy).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

WCA_RC = 2.0 ** (1.0 / 6.0)


class Box(C.Structure):
    _fields_ = [("n", C.c_int32), ("pad_", C.c_int32), ("lx", C.c_double), ("ly", C.c_double),
                ("lz", C.c_double), ("rc", C.c_double), ("c_attr", C.c_double),
                ("u_shift", C.c_double)]


def lj_shift(rc: float, c_attr: float) -> float:
    """Constant that makes 4[(1/r)^12 - c (1/r)^6] + shift vanish at r = rc (Example 1:
    the shift guarantees continuity at the cutoff)."""
    s6 = 1.0 / rc ** 6
    return -4.0 * (s6 * s6 - c_attr * s6)


def make_box(n: int, l, rc: float = WCA_RC, c_attr: float = 1.0, u_shift: float | None = None) -> Box:
    if np.isscalar(l):
        l = (float(l),) * 3
    if u_shift is None:
        u_shift = lj_shift(rc, c_attr)
    return Box(int(n), 0, float(l[0]), float(l[1]), float(l[2]), float(rc), float(c_attr),
               float(u_shift))


def _load():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "libttcf_oracle.so")
        if not os.path.exists(path) or any(
                os.path.getmtime(path) < os.path.getmtime(src) for src in _build.SOURCES):
            _build.build()
        lib = C.CDLL(path)
        D = C.POINTER(C.c_double)
        I = C.POINTER(C.c_int32)
        L = C.POINTER(C.c_int64)
        B = C.POINTER(Box)
        lib.orc_cell_dims.argtypes = [B, I]
        lib.orc_cell_list.argtypes = [B, D, I, I, I]
        lib.orc_grid_dims.argtypes = [B, C.c_double, I]
        lib.orc_cell_list_grid.argtypes = [B, I, D, I, I, I]
        lib.orc_forces.argtypes = [B, C.c_double, D, D, D]
        lib.orc_forces_brute.argtypes = [B, C.c_double, D, D, D]
        lib.orc_pairs.argtypes = [B, C.c_double, D, C.c_double, C.c_int64, I, I]
        lib.orc_pairs.restype = C.c_int64
        lib.orc_pairs_brute.argtypes = [B, C.c_double, D, C.c_double, C.c_int64, I, I]
        lib.orc_pairs_brute.restype = C.c_int64
        lib.orc_vpxy.argtypes = [B, C.c_double, D, D]
        lib.orc_vpxy.restype = C.c_double
        lib.orc_map.argtypes = [B, C.c_int32, D, D, D, D]
        lib.orc_map.restype = None
        lib.orc_nh_run.argtypes = [B, C.c_double, C.c_double, C.c_double, C.c_double, D, D, D,
                                   C.c_int64, D, D, D]
        lib.orc_sllod_run.argtypes = [B, C.c_double, C.c_double, C.c_int32, C.c_double, D, D, L,
                                      C.c_int64, D, D, D]
        lib.orc_iso_kick.argtypes = [C.c_int32, D, D, C.c_double]
        lib.orc_iso_kick.restype = None
        lib.orc_iso_shear.argtypes = [C.c_int32, D, C.c_double, C.c_double]
        lib.orc_iso_shear.restype = None
        lib.orc_mother_sample.argtypes = [B, C.c_double, C.c_double, C.c_double, C.c_double, D, D,
                                          D, C.c_int64, C.c_int32, C.c_int64, D, D]
        lib.orc_run_daughters.argtypes = [B, C.c_double, D, D, C.c_int32, I, I, D, C.c_int64,
                                          C.c_int32, D, D, D]
        lib.orc_nh_sllod_run.argtypes = [B, C.c_double, C.c_double, C.c_double, C.c_double,
                                         C.c_double, D, D, D, L, C.c_int64, D, D, D, D]
        lib.orc_mother_sample_zeta.argtypes = [B, C.c_double, C.c_double, C.c_double, C.c_double,
                                               D, D, D, C.c_int64, C.c_int32, C.c_int64, D, D, D]
        lib.orc_run_daughters_nh.argtypes = [B, C.c_double, C.c_double, C.c_double, C.c_double, D,
                                             D, D, C.c_int32, I, I, D, C.c_int64, C.c_int32, D, D,
                                             D]
        lib.orc_observables.argtypes = [B, C.c_double, D, D, C.c_int32, D]
        lib.orc_run_daughters_obs.argtypes = [B, C.c_double, C.c_double, C.c_double, C.c_double,
                                              D, D, D, C.c_int32, I, I, D, C.c_int64, C.c_int32,
                                              D, C.c_int32, D]
        lib.orc_colour_run.argtypes = [B, C.c_double, C.c_double, C.c_int32, C.c_double, D, D,
                                       C.c_int64, D, D, D]
        lib.orc_run_daughters_colour.argtypes = [B, C.c_double, D, D, D, C.c_double, C.c_double,
                                                 C.c_double, C.c_int32, I, I, D, C.c_int64,
                                                 C.c_int32, D, D, D]
        lib.orc_nh_colour_run.argtypes = [B, C.c_double, C.c_double, C.c_double, C.c_double,
                                          C.c_double, D, D, D, C.c_int64, D, D, D, D]
        lib.orc_pef_forces.argtypes = [B, D, D, D]
        lib.orc_map_pef.argtypes = [B, C.c_int32, D, D, D, D]
        lib.orc_map_pef.restype = None
        lib.orc_pef_run.argtypes = [B, C.c_double, C.c_double, C.c_int32, C.c_double, D, D, D,
                                    C.c_int64, D, D, D]
        lib.orc_run_daughters_pef.argtypes = [B, C.c_double, D, D, C.c_int32, I, I, D, C.c_int64,
                                              C.c_int32, D, D, D]
        lib.orc_nh_pef_run.argtypes = [B, C.c_double, C.c_double, C.c_double, C.c_double,
                                       C.c_double, D, D, D, D, C.c_int64, D, D, D, D]
        lib.orc_run_daughters_pef_nh.argtypes = [B, C.c_double, C.c_double, C.c_double,
                                                 C.c_double, D, D, D, C.c_int32, I, I, D,
                                                 C.c_int64, C.c_int32, D, D, D]
        lib.orc_mix_forces.argtypes = [B, D, D, D, D]
        lib.orc_map_mix.argtypes = [B, C.c_int32, D, D, D, D]
        lib.orc_map_mix.restype = None
        lib.orc_mix_run.argtypes = [B, C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32,
                                    C.c_double, C.c_double, C.c_double, D, D, D, D, C.c_int64,
                                    D, D, D, D]
        lib.orc_run_daughters_mix.argtypes = [B, C.c_double, D, D, D, C.c_double, C.c_double,
                                              C.c_double, C.c_int32, I, I, D, D, C.c_int64,
                                              C.c_int32, D, D, D, D]
        for fn in ("orc_cell_dims", "orc_cell_list", "orc_grid_dims", "orc_cell_list_grid",
                   "orc_forces", "orc_forces_brute",
                   "orc_nh_run", "orc_sllod_run", "orc_mother_sample", "orc_run_daughters",
                   "orc_nh_sllod_run", "orc_mother_sample_zeta", "orc_run_daughters_nh",
                   "orc_observables", "orc_run_daughters_obs", "orc_colour_run",
                   "orc_run_daughters_colour", "orc_nh_colour_run", "orc_pef_forces",
                   "orc_pef_run", "orc_run_daughters_pef", "orc_nh_pef_run",
                   "orc_run_daughters_pef_nh", "orc_mix_forces", "orc_mix_run",
                   "orc_run_daughters_mix"):
            getattr(lib, fn).restype = C.c_int32
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------------------
# forces, cell lists, pairs
# ----------------------------------------------------------------------------------------

def cell_dims(box: Box):
    d = np.zeros(3, np.int32)
    if _load().orc_cell_dims(C.byref(box), _ip(d)) != 0:
        raise ValueError("box too small for a 27-cell grid (need n_x >= 4, n_y, n_z >= 3)")
    return d


def grid_dims(box: Box, side: float):
    """Cells per edge of the grid whose cells are at least `side` wide: floor(L_a / side)."""
    d = np.zeros(3, np.int32)
    if _load().orc_grid_dims(C.byref(box), float(side), _ip(d)) != 0:
        raise ValueError("box too small for a 27-cell grid of that side")
    return d


def cell_list(box: Box, r, dims=None):
    """(cell_of, order, start) of the canonical cell list (cell id, then atom id), on the
    grid of side >= rc, or on the given grid dims (e.g. grid_dims(box, rc + skin))."""
    r = _f64(r)
    d = cell_dims(box) if dims is None else np.ascontiguousarray(dims, np.int32)
    cell_of = np.zeros(box.n, np.int32)
    order = np.zeros(box.n, np.int32)
    start = np.zeros(int(d.prod()) + 1, np.int32)
    rc = _load().orc_cell_list_grid(C.byref(box), _ip(d), _dp(r), _ip(cell_of), _ip(order),
                                    _ip(start))
    if rc != 0:
        raise RuntimeError(f"orc_cell_list failed: {rc}")
    return cell_of, order, start


def forces(box: Box, r, dxle: float = 0.0, brute: bool = False):
    """(F as (3, n), U, W_xy, n_pairs) at Lees-Edwards offset dxle."""
    r = _f64(r)
    f = np.zeros(3 * box.n)
    out = np.zeros(3)
    fn = _load().orc_forces_brute if brute else _load().orc_forces
    rc = fn(C.byref(box), float(dxle), _dp(r), _dp(f), _dp(out))
    if rc != 0:
        raise RuntimeError(f"oracle forces failed: {rc}")
    return f.reshape(3, box.n), out[0], out[1], int(round(out[2]))


def pairs(box: Box, r, dxle: float = 0.0, rlist: float | None = None, brute: bool = False):
    """Sorted (i, j) pairs, i<j, closer than rlist (default rc; a larger rlist gives the
    Verlet list of radius rc + skin)."""
    r = _f64(r)
    rl = box.rc if rlist is None else float(rlist)
    cap = max(64, int(8.0 * rl ** 3 * box.n / (box.lx * box.ly * box.lz) + 16)) * box.n
    pi = np.zeros(cap, np.int32)
    pj = np.zeros(cap, np.int32)
    fn = _load().orc_pairs_brute if brute else _load().orc_pairs
    cnt = fn(C.byref(box), float(dxle), _dp(r), rl, cap, _ip(pi), _ip(pj))
    if cnt < 0:
        raise RuntimeError(f"oracle pairs failed: {cnt}")
    return pi[:cnt].copy(), pj[:cnt].copy()


def verlet_lists(box: Box, r, rlist: float, dxle: float = 0.0):
    """Per-atom Verlet lists of radius rlist: lists[i] = ascending ids j != i closer than rlist
    (both directions of every pair of `pairs`)."""
    pi, pj = pairs(box, r, dxle, rlist)
    lists = [[] for _ in range(box.n)]
    for i, j in zip(pi.tolist(), pj.tolist()):
        lists[i].append(j)
        lists[j].append(i)
    return [np.array(sorted(x), np.int32) for x in lists]


def vpxy(box: Box, r, p, dxle: float = 0.0) -> float:
    return _load().orc_vpxy(C.byref(box), float(dxle), _dp(_f64(r)), _dp(_f64(p)))


def apply_mapping(box: Box, m: int, r, p):
    """Eq. (mappings): m=0 identity, 1 p->-p, 2 (x,px)->(-x,-px), 3 (x,py,pz)->(-x,-py,-pz)."""
    r = _f64(r)
    p = _f64(p)
    ro = np.empty_like(r)
    po = np.empty_like(p)
    _load().orc_map(C.byref(box), int(m), _dp(r), _dp(p), _dp(ro), _dp(po))
    return ro, po


# ----------------------------------------------------------------------------------------
# dynamics
# ----------------------------------------------------------------------------------------

def le_offset(box: Box, gamma_dot: float, dt: float, k: int) -> float:
    """Sliding-brick offset of the image above the box after k steps."""
    return float(np.fmod(gamma_dot * box.ly * (float(k) * dt), box.lx))


def nh_q(nf: float, temperature: float, tau: float) -> float:
    """Nose-Hoover mass Q = nf T tau^2 (the paper calls Q a damping factor and leaves it free)."""
    return nf * temperature * tau * tau


@dataclass
class NHState:
    r: np.ndarray
    p: np.ndarray
    zeta: float = 0.0


def nh_run(box: Box, state: NHState, nsteps: int, temperature: float, dt: float, q: float,
           nf: float, record: bool = False):
    """Advance a Nose-Hoover mother in place. With record: (vpxy, ke, pe) per step."""
    z = np.array([state.zeta])
    outs = [np.zeros(nsteps + 1) for _ in range(3)] if record else [None, None, None]
    rc = _load().orc_nh_run(C.byref(box), temperature, q, nf, dt, _dp(state.r), _dp(state.p),
                            _dp(z), int(nsteps), *[_dp(o) for o in outs])
    if rc != 0:
        raise RuntimeError(f"orc_nh_run failed: {rc}")
    state.zeta = float(z[0])
    return tuple(outs) if record else None


def mother_sample(box: Box, state: NHState, n_equil: int, n_states: int, steps_between: int,
                  temperature: float, dt: float, q: float, nf: float, with_zeta: bool = False):
    """Alg. LAMMPS SCRIPT, mother side: equilibrate n_equil steps, then n_states times run
    steps_between steps and save the state. Returns (states_r, states_p), (n_states, 3n),
    and with_zeta also the thermostat variable of every state."""
    sr = np.zeros((n_states, 3 * box.n))
    sp = np.zeros((n_states, 3 * box.n))
    sz = np.zeros(n_states)
    z = np.array([state.zeta])
    rc = _load().orc_mother_sample_zeta(C.byref(box), temperature, q, nf, dt, _dp(state.r),
                                        _dp(state.p), _dp(z), int(n_equil), int(n_states),
                                        int(steps_between), _dp(sr), _dp(sp), _dp(sz))
    if rc != 0:
        raise RuntimeError(f"orc_mother_sample failed: {rc}")
    state.zeta = float(z[0])
    return (sr, sp, sz) if with_zeta else (sr, sp)


def nh_sllod_run(box: Box, r, p, zeta: float, gamma_dot: float, dt: float, temperature: float,
                 q: float, nf: float, nsteps: int, kstep: int = 0):
    """Advance one Nose-Hoover SLLOD trajectory (Eq. system1 as printed) in place.
    Returns (vpxy, ke, pe, zeta series, k_final, zeta_final), series of length nsteps+1."""
    assert r.dtype == np.float64 and p.dtype == np.float64 and r.flags.c_contiguous
    outs = [np.zeros(nsteps + 1) for _ in range(4)]
    k = np.array([kstep], dtype=np.int64)
    z = np.array([float(zeta)])
    rc = _load().orc_nh_sllod_run(C.byref(box), float(gamma_dot), float(dt), float(temperature),
                                  float(q), float(nf), _dp(r), _dp(p), _dp(z),
                                  k.ctypes.data_as(C.POINTER(C.c_int64)), int(nsteps),
                                  *[_dp(o) for o in outs])
    if rc != 0:
        raise RuntimeError(f"orc_nh_sllod_run failed: {rc}")
    return outs[0], outs[1], outs[2], outs[3], int(k[0]), float(z[0])


def run_daughters_nh(box: Box, states_r, states_p, states_zeta, state_of, map_of, gamma_of,
                     dt: float, temperature: float, q: float, nf: float, nsteps: int,
                     nthreads: int = 0, final_state: bool = False):
    """Nose-Hoover daughters (orc_run_daughters_nh): as run_daughters, each start state with
    its thermostat variable, reversed by the time-reversing mappings."""
    states_r = _f64(states_r)
    states_p = _f64(states_p)
    states_zeta = _f64(states_zeta)
    state_of = np.ascontiguousarray(state_of, np.int32)
    map_of = np.ascontiguousarray(map_of, np.int32)
    gamma_of = _f64(gamma_of)
    nd = len(state_of)
    out = np.zeros((nd, nsteps + 1))
    ro = np.zeros((nd, 3 * box.n)) if final_state else None
    po = np.zeros((nd, 3 * box.n)) if final_state else None
    if nthreads <= 0:
        nthreads = os.cpu_count() or 1
    used = _load().orc_run_daughters_nh(C.byref(box), float(dt), float(temperature), float(q),
                                        float(nf), _dp(states_r), _dp(states_p), _dp(states_zeta),
                                        nd, _ip(state_of), _ip(map_of), _dp(gamma_of), int(nsteps),
                                        int(nthreads), _dp(out), _dp(ro), _dp(po))
    if used < 0:
        raise RuntimeError(f"orc_run_daughters_nh failed: {used}")
    if final_state:
        return out, ro, po, used
    return out, used


def colour_charges(n: int) -> np.ndarray:
    """Colour charge of each atom: +1 for even index, -1 for odd."""
    return np.where(np.arange(n) % 2 == 0, 1.0, -1.0)


def colour_run(box: Box, r, p, fe: float, dt: float, nsteps: int, gik: bool = True,
               k0: float = 0.0):
    """Advance one colour-field trajectory in place (orc_colour_run). Returns the series
    (V J_x, K, U), each of length nsteps+1."""
    assert r.dtype == np.float64 and p.dtype == np.float64 and r.flags.c_contiguous
    outs = [np.zeros(nsteps + 1) for _ in range(3)]
    rc = _load().orc_colour_run(C.byref(box), float(fe), float(dt), int(gik), float(k0), _dp(r),
                                _dp(p), int(nsteps), *[_dp(o) for o in outs])
    if rc != 0:
        raise RuntimeError(f"orc_colour_run failed: {rc}")
    return outs[0], outs[1], outs[2]


def nh_colour_run(box: Box, r, p, zeta: float, fe: float, dt: float, temperature: float,
                  q: float, nf: float, nsteps: int):
    """Advance one Nose-Hoover colour-field trajectory in place (orc_nh_colour_run). Returns
    (V J_x, K, U, zeta series, zeta_final), series of length nsteps+1."""
    assert r.dtype == np.float64 and p.dtype == np.float64 and r.flags.c_contiguous
    outs = [np.zeros(nsteps + 1) for _ in range(4)]
    z = np.array([float(zeta)])
    rc = _load().orc_nh_colour_run(C.byref(box), float(fe), float(dt), float(temperature),
                                   float(q), float(nf), _dp(r), _dp(p), _dp(z), int(nsteps),
                                   *[_dp(o) for o in outs])
    if rc != 0:
        raise RuntimeError(f"orc_nh_colour_run failed: {rc}")
    return outs[0], outs[1], outs[2], outs[3], float(z[0])


def run_daughters_colour(box: Box, states_r, states_p, state_of, map_of, fe_of, dt: float,
                         nsteps: int, nthreads: int = 0, final_state: bool = False,
                         states_zeta=None, temperature: float = 0.0, q: float = 0.0,
                         nf: float = 0.0):
    """Colour-field daughters on a CPU thread pool (isokinetic, or Nose-Hoover from each
    state's zeta when states_zeta is given): V J_x (n_d, nsteps+1) [and final r, p] and the
    number of threads used."""
    states_r = _f64(states_r)
    states_p = _f64(states_p)
    state_of = np.ascontiguousarray(state_of, np.int32)
    map_of = np.ascontiguousarray(map_of, np.int32)
    fe_of = _f64(fe_of)
    nd = len(state_of)
    out = np.zeros((nd, nsteps + 1))
    ro = np.zeros((nd, 3 * box.n)) if final_state else None
    po = np.zeros((nd, 3 * box.n)) if final_state else None
    if nthreads <= 0:
        nthreads = os.cpu_count() or 1
    zeta = _f64(states_zeta) if states_zeta is not None else None
    used = _load().orc_run_daughters_colour(C.byref(box), float(dt), _dp(states_r),
                                            _dp(states_p), _dp(zeta), float(temperature),
                                            float(q), float(nf), nd, _ip(state_of), _ip(map_of),
                                            _dp(fe_of), int(nsteps), int(nthreads), _dp(out),
                                            _dp(ro), _dp(po))
    if used < 0:
        raise RuntimeError(f"orc_run_daughters_colour failed: {used}")
    if final_state:
        return out, ro, po, used
    return out, used


def omega0_colour(vjx0, fe, temperature):
    """Dissipation function of the colour field at t=0: Omega = (V/T) F_e J_x(0)."""
    return (np.asarray(fe, np.float64) / temperature) * np.asarray(vjx0, np.float64)


def pef_box(box: Box, strain: float) -> Box:
    """The planar-elongation box at strain e: L_x e^e, L_y e^-e, L_z."""
    return Box(box.n, 0, box.lx * np.exp(strain), box.ly * np.exp(-strain), box.lz, box.rc,
               box.c_attr, box.u_shift)


def pef_forces(box: Box, r):
    """All-pairs forces in the (deformed) orthorhombic box (orc_pef_forces): (f, U,
    W_xx - W_yy, pairs)."""
    r = _f64(r)
    f = np.zeros(3 * box.n)
    out = np.zeros(3)
    rc = _load().orc_pef_forces(C.byref(box), _dp(r), _dp(f), _dp(out))
    if rc != 0:
        raise RuntimeError(f"orc_pef_forces failed: {rc}")
    return f, out[0], out[1], out[2]


def map_pef(box: Box, m: int, r, p):
    """Mapping m of planar elongation (bit 0: p -> -p, bit 1: exchange of the x and y axes)."""
    r = _f64(r)
    p = _f64(p)
    ro = np.zeros(3 * box.n)
    po = np.zeros(3 * box.n)
    _load().orc_map_pef(C.byref(box), int(m), _dp(r), _dp(p), _dp(ro), _dp(po))
    return ro, po


def pef_run(box: Box, r, p, rate: float, dt: float, nsteps: int, gik: bool = True,
            strain0: float = 0.0, k0: float = 0.0):
    """Advance one planar-elongation trajectory in place (orc_pef_run) from strain strain0.
    Returns (V (P_xx - P_yy), K, U) series of length nsteps+1 and the final strain."""
    assert r.dtype == np.float64 and p.dtype == np.float64 and r.flags.c_contiguous
    outs = [np.zeros(nsteps + 1) for _ in range(3)]
    e = np.array([float(strain0)])
    rc = _load().orc_pef_run(C.byref(box), float(rate), float(dt), int(gik), float(k0), _dp(e),
                             _dp(r), _dp(p), int(nsteps), *[_dp(o) for o in outs])
    if rc != 0:
        raise RuntimeError(f"orc_pef_run failed: {rc}")
    return outs[0], outs[1], outs[2], float(e[0])


def nh_pef_run(box: Box, r, p, zeta: float, rate: float, dt: float, temperature: float,
               q: float, nf: float, nsteps: int, strain0: float = 0.0):
    """Advance one Nose-Hoover planar-elongation trajectory in place (orc_nh_pef_run).
    Returns (V (P_xx - P_yy), K, U, zeta series, zeta_final, final strain)."""
    assert r.dtype == np.float64 and p.dtype == np.float64 and r.flags.c_contiguous
    outs = [np.zeros(nsteps + 1) for _ in range(4)]
    z = np.array([float(zeta)])
    e = np.array([float(strain0)])
    rc = _load().orc_nh_pef_run(C.byref(box), float(rate), float(dt), float(temperature),
                                float(q), float(nf), _dp(e), _dp(r), _dp(p), _dp(z), int(nsteps),
                                *[_dp(o) for o in outs])
    if rc != 0:
        raise RuntimeError(f"orc_nh_pef_run failed: {rc}")
    return outs[0], outs[1], outs[2], outs[3], float(z[0]), float(e[0])


def run_daughters_pef(box: Box, states_r, states_p, state_of, map_of, rate_of, dt: float,
                      nsteps: int, nthreads: int = 0, final_state: bool = False,
                      states_zeta=None, temperature: float = 0.0, q: float = 0.0,
                      nf: float = 0.0):
    """Planar-elongation daughters on a CPU thread pool (isokinetic, or Nose-Hoover from each
    state's zeta when states_zeta is given): V (P_xx - P_yy) (n_d, nsteps+1) [and final r, p
    in the deformed box] and the number of threads used."""
    states_r = _f64(states_r)
    states_p = _f64(states_p)
    state_of = np.ascontiguousarray(state_of, np.int32)
    map_of = np.ascontiguousarray(map_of, np.int32)
    rate_of = _f64(rate_of)
    nd = len(state_of)
    out = np.zeros((nd, nsteps + 1))
    ro = np.zeros((nd, 3 * box.n)) if final_state else None
    po = np.zeros((nd, 3 * box.n)) if final_state else None
    if nthreads <= 0:
        nthreads = os.cpu_count() or 1
    if states_zeta is not None:
        used = _load().orc_run_daughters_pef_nh(C.byref(box), float(dt), float(temperature),
                                                float(q), float(nf), _dp(states_r),
                                                _dp(states_p), _dp(_f64(states_zeta)), nd,
                                                _ip(state_of), _ip(map_of), _dp(rate_of),
                                                int(nsteps), int(nthreads), _dp(out), _dp(ro),
                                                _dp(po))
    else:
        used = _load().orc_run_daughters_pef(C.byref(box), float(dt), _dp(states_r),
                                             _dp(states_p), nd, _ip(state_of), _ip(map_of),
                                             _dp(rate_of), int(nsteps), int(nthreads), _dp(out),
                                             _dp(ro), _dp(po))
    if used < 0:
        raise RuntimeError(f"orc_run_daughters_pef failed: {used}")
    if final_state:
        return out, ro, po, used
    return out, used


def mix_cell(box: Box, erate: float, srate: float, t: float):
    """(H_xx, H_xy, H_yy) of the mixed-flow cell at time t: exp(A t) diag(L)."""
    x = erate * t
    sh = 1.0 if x == 0.0 else np.sinh(x) / x
    return np.array([box.lx * np.exp(x), box.ly * srate * t * sh, box.ly * np.exp(-x)])


def mix_forces(box: Box, h, r):
    """Forces in the mixed-flow cell (orc_mix_forces): (f, U, W_xx - W_yy, W_xy, pairs)."""
    r = _f64(r)
    h = _f64(h)
    f = np.zeros(3 * box.n)
    out = np.zeros(4)
    rc = _load().orc_mix_forces(C.byref(box), _dp(h), _dp(r), _dp(f), _dp(out))
    if rc != 0:
        raise RuntimeError(f"orc_mix_forces failed: {rc}")
    return f, out[0], out[1], out[2], out[3]


def map_mix(box: Box, m: int, r, p):
    """Mapping m of mixed flow (bit 1: exchange of the x and y axes, then bit 0: x-reflection)."""
    r = _f64(r)
    p = _f64(p)
    ro = np.zeros(3 * box.n)
    po = np.zeros(3 * box.n)
    _load().orc_map_mix(C.byref(box), int(m), _dp(r), _dp(p), _dp(ro), _dp(po))
    return ro, po


def mix_run(box: Box, r, p, erate: float, srate: float, dt: float, nsteps: int,
            gik: bool = True, t0: float = 0.0, zeta=None, temperature: float = 0.0,
            q: float = 0.0, nf: float = 0.0):
    """Advance one mixed-flow trajectory in place (orc_mix_run); Nose-Hoover when zeta is
    given. Returns (V J, K, U) series of length nsteps+1, the final time and the final zeta."""
    assert r.dtype == np.float64 and p.dtype == np.float64 and r.flags.c_contiguous
    outs = [np.zeros(nsteps + 1) for _ in range(3)]
    t = np.array([float(t0)])
    z = np.array([float(zeta) if zeta is not None else 0.0])
    rc = _load().orc_mix_run(C.byref(box), float(erate), float(srate), float(dt), int(gik),
                             int(zeta is not None), float(temperature), float(q), float(nf),
                             _dp(t), _dp(r), _dp(p), _dp(z), int(nsteps), *[_dp(o) for o in outs],
                             None)
    if rc != 0:
        raise RuntimeError(f"orc_mix_run failed: {rc}")
    return outs[0], outs[1], outs[2], float(t[0]), float(z[0])


def run_daughters_mix(box: Box, states_r, states_p, state_of, map_of, er_of, sr_of, dt: float,
                      nsteps: int, nthreads: int = 0, final_state: bool = False,
                      states_zeta=None, temperature: float = 0.0, q: float = 0.0,
                      nf: float = 0.0, components: bool = False):
    """Mixed-flow daughters on a CPU thread pool: V J (n_d, nsteps+1) [and final r, p] and the
    number of threads used; with components, also V (P_xx - P_yy) and V P_xy as
    (n_d, nsteps+1, 2) after the thread count."""
    states_r = _f64(states_r)
    states_p = _f64(states_p)
    state_of = np.ascontiguousarray(state_of, np.int32)
    map_of = np.ascontiguousarray(map_of, np.int32)
    er_of = _f64(er_of)
    sr_of = _f64(sr_of)
    nd = len(state_of)
    out = np.zeros((nd, nsteps + 1))
    ro = np.zeros((nd, 3 * box.n)) if final_state else None
    po = np.zeros((nd, 3 * box.n)) if final_state else None
    if nthreads <= 0:
        nthreads = os.cpu_count() or 1
    zeta = _f64(states_zeta) if states_zeta is not None else None
    comp = np.zeros((nd, nsteps + 1, 2)) if components else None
    used = _load().orc_run_daughters_mix(C.byref(box), float(dt), _dp(states_r), _dp(states_p),
                                         _dp(zeta), float(temperature), float(q), float(nf), nd,
                                         _ip(state_of), _ip(map_of), _dp(er_of), _dp(sr_of),
                                         int(nsteps), int(nthreads), _dp(out), _dp(ro), _dp(po),
                                         _dp(comp))
    if used < 0:
        raise RuntimeError(f"orc_run_daughters_mix failed: {used}")
    res = (out, ro, po, used) if final_state else (out, used)
    return res + (comp,) if components else res


N_SLABS = 8  # slabs of the bulk momentum profile


def observables(box: Box, r, p, dxle: float = 0.0, n_slabs: int = N_SLABS) -> np.ndarray:
    """Observables beyond P_xy (orc_observables): [P_xx - P_yy, P_yy - P_zz, (K + U)/N,
    then per y slab the summed p_x over the slab volume], length 3 + n_slabs."""
    r = _f64(r)
    p = _f64(p)
    out = np.zeros(3 + n_slabs)
    rc = _load().orc_observables(C.byref(box), float(dxle), _dp(r), _dp(p), int(n_slabs),
                                 _dp(out))
    if rc != 0:
        raise RuntimeError(f"orc_observables failed: {rc}")
    return out


def run_daughters_obs(box: Box, states_r, states_p, state_of, map_of, gamma_of, dt: float,
                      nsteps: int, states_zeta=None, temperature: float = 0.0, q: float = 0.0,
                      nf: float = 0.0, n_slabs: int = N_SLABS, nthreads: int = 0):
    """Daughters (GIK, or Nose-Hoover when states_zeta is given) that also record the
    observables of `observables` after every step. Returns vpxy (n_d, nsteps+1) and
    obs (n_d, nsteps+1, 3+n_slabs)."""
    states_r = _f64(states_r)
    states_p = _f64(states_p)
    zeta = _f64(states_zeta) if states_zeta is not None else None
    state_of = np.ascontiguousarray(state_of, np.int32)
    map_of = np.ascontiguousarray(map_of, np.int32)
    gamma_of = _f64(gamma_of)
    nd = len(state_of)
    vp = np.zeros((nd, nsteps + 1))
    ob = np.zeros((nd, nsteps + 1, 3 + n_slabs))
    if nthreads <= 0:
        nthreads = os.cpu_count() or 1
    used = _load().orc_run_daughters_obs(C.byref(box), float(dt), float(temperature), float(q),
                                         float(nf), _dp(states_r), _dp(states_p), _dp(zeta), nd,
                                         _ip(state_of), _ip(map_of), _dp(gamma_of), int(nsteps),
                                         int(nthreads), _dp(vp), int(n_slabs), _dp(ob))
    if used < 0:
        raise RuntimeError(f"orc_run_daughters_obs failed: {used}")
    return vp, ob


def sllod_run(box: Box, r, p, gamma_dot: float, dt: float, nsteps: int, gik: bool = True,
              k0: float = 0.0, kstep: int = 0):
    """Advance one SLLOD trajectory in place (r, p float64 SoA arrays).
    Returns (vpxy, ke, pe, k_final), series of length nsteps+1."""
    assert r.dtype == np.float64 and p.dtype == np.float64 and r.flags.c_contiguous
    outs = [np.zeros(nsteps + 1) for _ in range(3)]
    k = np.array([kstep], dtype=np.int64)
    rc = _load().orc_sllod_run(C.byref(box), float(gamma_dot), float(dt), int(bool(gik)),
                               float(k0), _dp(r), _dp(p),
                               k.ctypes.data_as(C.POINTER(C.c_int64)), int(nsteps),
                               *[_dp(o) for o in outs])
    if rc != 0:
        raise RuntimeError(f"orc_sllod_run failed: {rc}")
    return outs[0], outs[1], outs[2], int(k[0])


def iso_kick(p, f, tau: float):
    """Exact isokinetic force kick (returns a new array; p, f are flat SoA)."""
    p = _f64(p).copy()
    f = _f64(f)
    _load().orc_iso_kick(len(p) // 3, _dp(p), _dp(f), float(tau))
    return p


def iso_shear(p, gamma_dot: float, tau: float):
    """Exact isokinetic shear flow of the momenta (returns a new array)."""
    p = _f64(p).copy()
    _load().orc_iso_shear(len(p) // 3, _dp(p), float(gamma_dot), float(tau))
    return p


def run_daughters(box: Box, states_r, states_p, state_of, map_of, gamma_of, dt: float,
                  nsteps: int, nthreads: int = 0, final_state: bool = False):
    """Alg. LAMMPS SCRIPT, daughter side, on a CPU thread pool. Returns vpxy (n_d, nsteps+1)
    [and final r, p] and the number of threads used."""
    states_r = _f64(states_r)
    states_p = _f64(states_p)
    state_of = np.ascontiguousarray(state_of, np.int32)
    map_of = np.ascontiguousarray(map_of, np.int32)
    gamma_of = _f64(gamma_of)
    nd = len(state_of)
    out = np.zeros((nd, nsteps + 1))
    ro = np.zeros((nd, 3 * box.n)) if final_state else None
    po = np.zeros((nd, 3 * box.n)) if final_state else None
    if nthreads <= 0:
        nthreads = os.cpu_count() or 1
    used = _load().orc_run_daughters(C.byref(box), float(dt), _dp(states_r), _dp(states_p), nd,
                                     _ip(state_of), _ip(map_of), _dp(gamma_of), int(nsteps),
                                     int(nthreads), _dp(out), _dp(ro), _dp(po))
    if used < 0:
        raise RuntimeError(f"orc_run_daughters failed: {used}")
    if final_state:
        return out, ro, po, used
    return out, used


# ----------------------------------------------------------------------------------------
# estimators (numpy, FP64)
# ----------------------------------------------------------------------------------------

def omega0(vpxy0, gamma_dot, temperature):
    """Dissipation function at t=0, Eq. (TTCF1) in the pressure-tensor convention:
    Omega = -(V/T) gamma_dot P_xy(0) = -(gamma_dot/T) * (V P_xy(0))."""
    return -(np.asarray(gamma_dot, np.float64) / temperature) * np.asarray(vpxy0, np.float64)


@dataclass
class Response:
    ttcf: np.ndarray       # <B(t)> by Eq. (TTCF)
    ttcf_se: np.ndarray    # block standard error over start states
    dav: np.ndarray        # direct average of B(t)
    dav_se: np.ndarray
    g: np.ndarray          # per-start-state TTCF series G_n(t), (n_states, n_t)
    d: np.ndarray          # per-start-state direct-average series D_n(t)
    integrand: np.ndarray  # <Omega(0) B(t)> over all daughters, Eq. (integrand)
    integrand_se_paper: np.ndarray  # sigma/sqrt(N_daughters) of Omega(0)B(t) (paper's SE)
    dav_se_paper: np.ndarray        # sigma/sqrt(N_daughters) of B(t)


def ttcf_response(b, vpxy0, gamma_of, temperature: float, dt: float, n_maps: int = 4,
                  omega=None) -> Response:
    """TTCF and direct-average responses from per-daughter series.

    b[d, k]   : observable B of daughter d at t_k = k dt, k = 0..n_t-1
    vpxy0[d]  : V * P_xy of daughter d at t = 0 (gives Omega(0))
    gamma_of[d]: shear rate of daughter d
    Daughters are ordered state-major: d = n * n_maps + m.

    Eq. (TTCF): <B(t)> = <B(0)> + int_0^t <Omega(0) B(s)> ds, with the ensemble average of
    Eq. (integrand) and the integral taken by the trapezoid rule on the step grid. The
    standard error is the block error over start states (each block = the n_maps mapped
    daughters of one state), std with ddof=1 over sqrt(number of states).
    """
    b = np.asarray(b, np.float64)
    nd, nt = b.shape
    assert nd % n_maps == 0
    ns = nd // n_maps
    # Omega(0) of each daughter: the shear field's unless given (e.g. omega0_colour)
    om = omega0(vpxy0, gamma_of, temperature) if omega is None else np.asarray(omega, np.float64)
    ob = om[:, None] * b                       # Omega(0) B(t)
    integ = np.zeros_like(ob)
    integ[:, 1:] = np.cumsum(0.5 * dt * (ob[:, :-1] + ob[:, 1:]), axis=1)
    per_d = b[:, :1] + integ                   # B(0) + int_0^t Omega(0) B(s) ds
    g = per_d.reshape(ns, n_maps, nt).mean(axis=1)
    dd = b.reshape(ns, n_maps, nt).mean(axis=1)
    sq = np.sqrt(ns)
    return Response(
        ttcf=g.mean(axis=0), ttcf_se=(g.std(axis=0, ddof=1) / sq) if ns > 1 else np.full(nt, np.nan),
        dav=dd.mean(axis=0), dav_se=(dd.std(axis=0, ddof=1) / sq) if ns > 1 else np.full(nt, np.nan),
        g=g, d=dd, integrand=ob.mean(axis=0),
        integrand_se_paper=ob.std(axis=0, ddof=1) / np.sqrt(nd),
        dav_se_paper=b.std(axis=0, ddof=1) / np.sqrt(nd))


def ttcf_response_modified(b, vpxy0, gamma_of, temperature: float, dt: float, n_maps: int = 4):
    """Eq. (corr_modified): <B(0)> + int_0^t [<Omega(0)B(s)> - <Omega(0)><B(s)>] ds, the
    averages over all daughters, the integral by the trapezoid rule on the step grid. The
    standard error is the jackknife over start states (each left out with its n_maps mapped
    daughters). Returns (mean, se), each of length n_t."""
    b = np.asarray(b, np.float64)
    nd, nt = b.shape
    assert nd % n_maps == 0
    ns = nd // n_maps
    om = omega0(vpxy0, gamma_of, temperature)

    def estimate(keep):
        bb = b[keep]
        oo = om[keep]
        integrand = (oo[:, None] * bb).mean(axis=0) - oo.mean() * bb.mean(axis=0)
        integ = np.concatenate([[0.0], np.cumsum(0.5 * dt * (integrand[:-1] + integrand[1:]))])
        return bb[:, 0].mean() + integ

    everyone = np.arange(nd)
    full = estimate(everyone)
    if ns < 2:
        return full, np.full(nt, np.nan)
    jack = np.array([estimate(everyone[(everyone // n_maps) != n]) for n in range(ns)])
    se = np.sqrt((ns - 1) / ns * ((jack - jack.mean(axis=0)) ** 2).sum(axis=0))
    return full, se


def viscosity(response_mean, gamma_dot):
    """Eq. (visc): eta(t) = <P_xy(t)>/gamma_dot in the paper's shear-stress sign, i.e.
    -<P_xy(t)>/gamma_dot with the pressure-tensor P_xy used here."""
    return -np.asarray(response_mean) / gamma_dot


def green_kubo(pxy_series, volume: float, temperature: float, dt: float, max_lag: int):
    """Equilibrium limit of Eq. (visc) (TTCF as a generalisation of Green-Kubo):
    C(s) = <P_xy(0) P_xy(s)> averaged over every time origin of an equilibrium series,
    eta_GK(t) = (V/T) int_0^t C(s) ds by the trapezoid rule. Returns (C, eta_GK)."""
    x = np.asarray(pxy_series, np.float64)
    n = len(x)
    c = np.array([np.dot(x[: n - s], x[s:]) / (n - s) for s in range(max_lag + 1)])
    eta = np.zeros(max_lag + 1)
    eta[1:] = np.cumsum(0.5 * dt * (c[:-1] + c[1:]))
    return c, (volume / temperature) * eta


# ----------------------------------------------------------------------------------------
# autocorrelation of the mother's P_xy (Sec. Mathematical Framework: choice of T_s)
# ----------------------------------------------------------------------------------------

def acf(series, max_lag: int) -> np.ndarray:
    """acf[k] = C(k)/C(0), C(k) = sum_{i < n-k} (x_i - m)(x_{i+k} - m) / (n - k): the
    definition, one dot product per lag."""
    x = _f64(np.ravel(series))
    d = x - x.mean()
    n = len(d)
    c = np.array([np.dot(d[:n - k], d[k:]) / (n - k) for k in range(max_lag)])
    return c / c[0]


def acf_summary(a: np.ndarray, threshold: float):
    """(first lag k >= 1 with a[k] < threshold or -1, integrated correlation time
    1/2 + sum_{1 <= k < k0} a[k] with k0 the first lag where a[k] <= 0)."""
    below = [k for k in range(1, len(a)) if a[k] < threshold]
    tau = 0.5
    for k in range(1, len(a)):
        if not a[k] > 0.0:
            break
        tau += a[k]
    return (below[0] if below else -1), tau
