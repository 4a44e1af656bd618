"""FP64 oracle of the confined-channel example (Eq. system2 and Eq. TTCF2).

TEST INFRASTRUCTURE: only the test-suite and the benchmark import this module; the GPU
library shares no code with it.

ctypes bindings of the channel part of ``libttcf_oracle.so`` (forces by direct summation,
velocity Verlet with a Nose-Hoover thermostat on the wall atoms, moving lattices, mappings,
daughters) and the channel's TTCF estimator written with numpy. Dissipation function:
Omega(0) = -(k v / (2 T_w)) S(0), with S the difference of the summed x tether extensions of
the top and the bottom wall (Eq. TTCF2 with beta = 1/T_w and the sign of the adiabatic energy
balance: the moving lattices do work -sum_i k (r^w_i - r^l_i) . u_i per unit time).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from .oracle import _load as _load_lib


class Channel(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_fluid", C.c_int32), ("n_wall", C.c_int32),
                ("n_bins", C.c_int32), ("lx", C.c_double), ("lz", C.c_double),
                ("rc", C.c_double), ("c_ff", C.c_double), ("c_wf", C.c_double),
                ("k_spring", C.c_double), ("bin_lo", C.c_double), ("bin_hi", C.c_double)]


_sig = False


def _lib():
    global _sig
    lib = _load_lib()
    if not _sig:
        D = C.POINTER(C.c_double)
        I = C.POINTER(C.c_int32)
        P = C.POINTER(Channel)
        lib.orc_ch_forces.argtypes = [P, D, D, D, D]
        lib.orc_ch_forces.restype = C.c_int32
        lib.orc_ch_observables.argtypes = [P, D, D, D, D]
        lib.orc_ch_observables.restype = None
        lib.orc_ch_run.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_double, D, D, D, D,
                                   C.c_int64, C.c_int64, D, D, D]
        lib.orc_ch_run.restype = C.c_int32
        lib.orc_ch_map.argtypes = [P, C.c_int32, D, D, C.c_double, D, D, D, D, D]
        lib.orc_ch_map.restype = None
        lib.orc_ch_run_daughters.argtypes = [P, C.c_double, C.c_double, C.c_double, D, D, D, D, I,
                                             I, D, C.c_int32, C.c_int32, D, D, C.c_int32]
        lib.orc_ch_run_daughters.restype = C.c_int32
        _sig = True
    return lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_channel(geom) -> Channel:
    """From a ttcf_inputs.ChannelSystem."""
    return Channel(int(geom.n), int(geom.n_fluid), int(geom.n_wall), int(geom.n_bins),
                   float(geom.lx), float(geom.lz), float(geom.rc), float(geom.c_ff),
                   float(geom.c_wf), float(geom.k_spring), float(geom.bin_lo),
                   float(geom.bin_hi))


def forces(ch: Channel, r, rl):
    """(f, out) with out = [U_lj, U_spring, Fx_top, Fx_bottom, S]."""
    r = _f64(r).ravel()
    rl = _f64(rl).ravel()
    f = np.zeros(3 * ch.n)
    out = np.zeros(5)
    _lib().orc_ch_forces(C.byref(ch), _dp(r), _dp(rl), _dp(f), _dp(out))
    return f, out


def observables(ch: Channel, r, p, fout):
    obs = np.zeros(1 + ch.n_bins)
    _lib().orc_ch_observables(C.byref(ch), _dp(_f64(r).ravel()), _dp(_f64(p).ravel()),
                              _dp(_f64(fout)), _dp(obs))
    return obs


def nh_q(n_wall: int, temperature: float, tau: float) -> float:
    """Thermostat mass of the wall Nose-Hoover chain-free thermostat: Q = 3 N_w T tau^2."""
    return 3.0 * n_wall * temperature * tau * tau


@dataclass
class ChState:
    r: np.ndarray
    p: np.ndarray
    zeta: float = 0.0


def run(ch: Channel, state: ChState, rl0, nsteps: int, t_wall: float, q: float, dt: float,
        v: float = 0.0, k0: int = 0):
    """Advance in place; returns (obs[nsteps+1, 1+n_bins], S[nsteps+1], energy[nsteps+1])."""
    assert state.r.dtype == np.float64 and state.r.flags.c_contiguous
    obs = np.zeros((nsteps + 1, 1 + ch.n_bins))
    s = np.zeros(nsteps + 1)
    e = np.zeros(nsteps + 1)
    z = np.array([state.zeta])
    rc = _lib().orc_ch_run(C.byref(ch), t_wall, q, dt, v, _dp(state.r), _dp(state.p), _dp(z),
                           _dp(_f64(rl0).ravel()), int(k0), int(nsteps), _dp(obs), _dp(s), _dp(e))
    if rc != 0:
        raise RuntimeError(f"orc_ch_run failed: {rc}")
    state.zeta = float(z[0])
    return obs, s, e


def apply_mapping(ch: Channel, m: int, r, p, zeta: float, rl):
    ro = np.zeros(3 * ch.n)
    po = np.zeros(3 * ch.n)
    rlo = np.zeros(3 * ch.n_wall)
    zo = np.zeros(1)
    _lib().orc_ch_map(C.byref(ch), int(m), _dp(_f64(r).ravel()), _dp(_f64(p).ravel()),
                      float(zeta), _dp(_f64(rl).ravel()), _dp(ro), _dp(po), _dp(zo), _dp(rlo))
    return ro, po, float(zo[0]), rlo


def mother_sample(ch: Channel, state: ChState, rl, n_equil: int, n_states: int,
                  steps_between: int, t_wall: float, q: float, dt: float):
    """Equilibrium mother (v = 0): n_equil steps, then n_states states steps_between apart."""
    run(ch, state, rl, n_equil, t_wall, q, dt)
    sr = np.zeros((n_states, 3 * ch.n))
    sp = np.zeros((n_states, 3 * ch.n))
    sz = np.zeros(n_states)
    for k in range(n_states):
        run(ch, state, rl, steps_between, t_wall, q, dt)
        sr[k] = state.r
        sp[k] = state.p
        sz[k] = state.zeta
    return sr, sp, sz


def run_daughters(ch: Channel, states_r, states_p, states_zeta, rl, state_of, map_of, v_of,
                  t_wall: float, q: float, dt: float, nsteps: int, nthreads: int = 8):
    """Returns (obs[nd, nsteps+1, 1+n_bins], S(0)[nd])."""
    sr = _f64(states_r)
    sp = _f64(states_p)
    sz = _f64(states_zeta)
    so = np.ascontiguousarray(state_of, dtype=np.int32)
    mo = np.ascontiguousarray(map_of, dtype=np.int32)
    vo = _f64(v_of)
    nd = len(so)
    obs = np.zeros((nd, nsteps + 1, 1 + ch.n_bins))
    s0 = np.zeros(nd)
    _lib().orc_ch_run_daughters(C.byref(ch), t_wall, q, dt, _dp(sr), _dp(sp), _dp(sz),
                                _dp(_f64(rl).ravel()),
                                so.ctypes.data_as(C.POINTER(C.c_int32)),
                                mo.ctypes.data_as(C.POINTER(C.c_int32)), _dp(vo), nd, int(nsteps),
                                _dp(obs), _dp(s0), int(nthreads))
    return obs, s0


@dataclass
class ChannelResponse:
    ttcf: np.ndarray      # (n_t, n_obs)
    ttcf_se: np.ndarray
    dav: np.ndarray
    dav_se: np.ndarray
    g: np.ndarray         # per start state (n_states, n_t, n_obs)
    d: np.ndarray


def ttcf_response(obs, s0, v_of, k_spring: float, t_wall: float, dt: float,
                  n_maps: int = 4) -> ChannelResponse:
    """Eq. TTCF with Omega(0) = -(k v / (2 T_w)) S(0): per start state (its n_maps mapped
    daughters, state-major), G_n(t) = mean_m B_m(0) + int_0^t mean_m Omega_m(0) B_m(s) ds by
    the trapezoid rule; D_n(t) = mean_m B_m(t); means and block standard errors over states."""
    obs = np.asarray(obs, np.float64)
    nd, nt, nobs = obs.shape
    om = -(k_spring * np.asarray(v_of) / (2.0 * t_wall)) * np.asarray(s0)
    integrand = om[:, None, None] * obs
    integ = np.zeros_like(obs)
    integ[:, 1:] = np.cumsum(0.5 * dt * (integrand[:, :-1] + integrand[:, 1:]), axis=1)
    per_d = obs[:, :1, :] + integ
    ns = nd // n_maps
    g = per_d.reshape(ns, n_maps, nt, nobs).mean(axis=1)
    d = obs.reshape(ns, n_maps, nt, nobs).mean(axis=1)
    se = lambda a: a.std(axis=0, ddof=1) / np.sqrt(ns)
    return ChannelResponse(g.mean(axis=0), se(g), d.mean(axis=0), se(d), g, d)
