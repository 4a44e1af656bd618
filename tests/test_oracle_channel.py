"""Pins of the confined-channel oracle (Eq. system2, Eq. TTCF2) by checks independent of its
own formulas: gradients by central differences, Newton's third law, momentum balance,
energy conservation and its dt^2 scaling, the energy balance of the moving lattices (which
fixes the sign of Omega), time reversibility, and the signs of Omega and B under the
mappings."""
import numpy as np
import pytest

import ttcf_inputs as I
from oracle import channel as CH

SMALL = I.ChannelSystem(n_x=6, n_z=6, n_fluid=220)


@pytest.fixture(scope="module")
def sys_small():
    ch = SMALL
    r, p, rl = I.channel_initial_state(ch, 1)
    c = CH.make_channel(ch)
    # a disordered state: a short thermostatted run from the initial grid
    st = CH.ChState(r.ravel().copy(), p.ravel().copy())
    CH.run(c, st, rl, 300, ch.temperature, CH.nh_q(ch.n_wall, ch.temperature, ch.nh_tau), ch.dt)
    return ch, c, st.r.copy(), st.p.copy(), st.zeta, rl.ravel().copy()


def energy(c, r, rl):
    _, out = CH.forces(c, r, rl)
    return out[0] + out[1]


def test_force_is_minus_energy_gradient(sys_small):
    ch, c, r, p, z, rl = sys_small
    f, _ = CH.forces(c, r, rl)
    rng = np.random.Generator(np.random.PCG64(3))
    h = 1e-6
    for idx in rng.choice(3 * ch.n, size=24, replace=False):
        rp = r.copy()
        rm = r.copy()
        rp[idx] += h
        rm[idx] -= h
        num = -(energy(c, rp, rl) - energy(c, rm, rl)) / (2 * h)
        assert f[idx] == pytest.approx(num, rel=1e-5, abs=1e-5)


def test_newton_third_law_and_wall_momentum_balance(sys_small):
    ch, c, r, p, z, rl = sys_small
    f, out = CH.forces(c, r, rl)
    f3 = f.reshape(3, ch.n)
    # LJ forces sum to zero: the total equals the sum of the tether forces
    f_spring = np.zeros_like(f3)
    rr = r.reshape(3, ch.n)
    rlr = rl.reshape(3, ch.n_wall)
    dx = rr[0, ch.n_fluid:] - rlr[0]
    dx -= ch.lx * np.rint(dx / ch.lx)
    dy = rr[1, ch.n_fluid:] - rlr[1]
    dz = rr[2, ch.n_fluid:] - rlr[2]
    dz -= ch.lz * np.rint(dz / ch.lz)
    scale = np.abs(f3).max()
    np.testing.assert_allclose(f3.sum(axis=1), -ch.k_spring * np.array([dx.sum(), dy.sum(), dz.sum()]),
                               atol=1e-10 * scale * ch.n)
    # fluid-fluid forces cancel: the walls' x force on the fluid is the fluid's total x force
    assert out[2] + out[3] == pytest.approx(f3[0, :ch.n_fluid].sum(), abs=1e-10 * scale * ch.n)
    # S is the difference of the summed x tether extensions
    half = ch.n_wall // 2
    assert out[4] == pytest.approx(dx[half:].sum() - dx[:half].sum(), abs=1e-12)


def _nve_rms(c, ch, r, p, rl, dt, t_total):
    st = CH.ChState(r.copy(), p.copy())
    _, _, e = CH.run(c, st, rl, int(round(t_total / dt)), ch.temperature, 0.0, dt)
    return np.sqrt(np.mean((e - e[0]) ** 2)), e


def test_energy_error_scales_as_dt_squared(sys_small):
    ch, c, r, p, z, rl = sys_small
    e1, _ = _nve_rms(c, ch, r, p, rl, 0.004, 0.4)
    e2, _ = _nve_rms(c, ch, r, p, rl, 0.002, 0.4)
    assert 3.0 < e1 / e2 < 5.0


def test_moving_lattice_energy_balance_fixes_omega_sign(sys_small):
    """Without thermostat, dE/dt = -sum_i k (r^w_i - r^l_i) . u_i = -(k v / 2) S: the
    dissipation function of Eq. TTCF2 is beta times this rate."""
    ch, c, r, p, z, rl = sys_small
    v = 0.5
    for dt in (0.002, 0.001):
        st = CH.ChState(r.copy(), p.copy())
        n = int(round(0.2 / dt))
        _, s, e = CH.run(c, st, rl, n, ch.temperature, 0.0, dt, v=v)
        work = -(ch.k_spring * v / 2.0) * np.concatenate([[0.0], np.cumsum(0.5 * dt * (s[:-1] + s[1:]))])
        err = np.abs((e - e[0]) - work).max()
        if dt == 0.002:
            err_big = err
            scale = np.abs(work).max()
    assert scale > 1.0  # the lattices did real work
    assert err < 0.4 * err_big  # second order in dt
    assert err < 1e-2 * scale   # the opposite sign would miss by twice the work


def test_time_reversibility(sys_small):
    ch, c, r, p, z, rl = sys_small
    q = CH.nh_q(ch.n_wall, ch.temperature, ch.nh_tau)
    st = CH.ChState(r.copy(), p.copy(), z)
    CH.run(c, st, rl, 100, ch.temperature, q, ch.dt)
    r1, p1, z1, _ = CH.apply_mapping(c, 1, st.r, st.p, st.zeta, rl)
    back = CH.ChState(r1, p1, z1)
    CH.run(c, back, rl, 100, ch.temperature, q, ch.dt)
    dr = back.r - r
    dr3 = dr.reshape(3, ch.n)
    dr3[0] -= ch.lx * np.rint(dr3[0] / ch.lx)
    dr3[2] -= ch.lz * np.rint(dr3[2] / ch.lz)
    assert np.abs(dr3).max() < 1e-8
    assert np.abs(back.p + p).max() < 1e-8 * np.abs(p).max()
    assert back.zeta == pytest.approx(-z, abs=1e-9)


def test_mapping_signs_of_omega_and_observables(sys_small):
    ch, c, r, p, z, rl = sys_small
    s, bw, prof = [], [], []
    for m in range(4):
        rm, pm, zm, rlm = CH.apply_mapping(c, m, r, p, z, rl)
        _, out = CH.forces(c, rm, rlm)
        obs = CH.observables(c, rm, pm, out)
        s.append(out[4])
        bw.append(obs[0])
        prof.append(obs[1:])
    assert abs(s[0]) > 1e-3 and abs(bw[0]) > 1e-3 and np.abs(prof[0]).max() > 1e-3
    # p reversal: positions unchanged, so S and the wall stress are unchanged; p_x flips
    assert s[1] == pytest.approx(s[0], rel=1e-12)
    assert bw[1] == pytest.approx(bw[0], rel=1e-12)
    np.testing.assert_allclose(prof[1], -prof[0], atol=1e-12)
    # x reflection: S, the wall x force and p_x all flip
    for m in (2, 3):
        assert s[m] == pytest.approx(-s[0], rel=1e-9)
        assert bw[m] == pytest.approx(-bw[0], rel=1e-9)
    np.testing.assert_allclose(prof[2], -prof[0], atol=1e-12)
    np.testing.assert_allclose(prof[3], prof[0], atol=1e-12)
    # Omega sums to zero over the four mappings
    assert abs(sum(s)) < 1e-9 * abs(s[0])


def test_estimator_closed_form():
    """Synthetic series with B linear in time: the trapezoid integral is exact."""
    rng = np.random.Generator(np.random.PCG64(7))
    nd, nt, nobs, dt = 8, 6, 3, 0.1
    a = rng.standard_normal((nd, 1, nobs))
    b = rng.standard_normal((nd, 1, nobs))
    t = dt * np.arange(nt)[None, :, None]
    obs = a + b * t
    s0 = rng.standard_normal(nd)
    v = np.full(nd, 0.3)
    res = CH.ttcf_response(obs, s0, v, 150.0, 1.0, dt)
    om = -(150.0 * 0.3 / 2.0) * s0
    exact = a + om[:, None, None] * (a * t + 0.5 * b * t * t)
    g = exact.reshape(2, 4, nt, nobs).mean(axis=1)
    np.testing.assert_allclose(res.ttcf, g.mean(axis=0), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(res.dav, obs.reshape(2, 4, nt, nobs).mean(axis=1).mean(axis=0),
                               rtol=1e-12)


@pytest.mark.slow
def test_ttcf_equals_direct_average_at_strong_driving(sys_small):
    """At strong driving the direct average resolves the response: TTCF and DAV agree
    within two standard errors of their paired difference (same daughters) at nearly every
    (t, observable). A consistency check only: the TTCF error of this small system is far
    larger than the direct average's, so the sign of Omega is pinned by the energy balance."""
    ch, c, r, p, z, rl = sys_small
    q = CH.nh_q(ch.n_wall, ch.temperature, ch.nh_tau)
    st = CH.ChState(r.copy(), p.copy(), z)
    ns = 48
    sr, sp, sz = CH.mother_sample(c, st, rl, 0, ns, 40, ch.temperature, q, ch.dt)
    nst, v = 60, 2.0
    state_of = np.repeat(np.arange(ns), 4)
    map_of = np.tile(np.arange(4), ns)
    obs, s0 = CH.run_daughters(c, sr, sp, sz, rl, state_of, map_of, np.full(4 * ns, v),
                               ch.temperature, q, ch.dt, nst)
    res = CH.ttcf_response(obs, s0, np.full(4 * ns, v), ch.k_spring, ch.temperature, ch.dt)
    diff = res.g - res.d
    se = diff.std(axis=0, ddof=1) / np.sqrt(ns)
    k = slice(1, None)
    assert np.mean(np.abs(diff.mean(axis=0)[k]) <= 2.0 * se[k] + 1e-15) > 0.85
    # and the wall stress has responded: DAV at the end is many standard errors from zero
    assert abs(res.dav[-1, 0]) > 3.0 * res.dav_se[-1, 0]
