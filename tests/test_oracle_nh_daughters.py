"""Pins of the oracle's Nose-Hoover SLLOD daughters (Eq. system1 as printed, alpha the
Nose-Hoover variable) by checks independent of its own formulas: the extended-energy balance
against the shear work (fixes the signs of the shear and thermostat parts), time reversal
under (p, zeta, gamma_dot) -> (-p, -zeta, -gamma_dot) (which is why the time-reversing
mappings reverse zeta), the canonical kinetic temperature, and agreement with the pinned
Nose-Hoover mother step at zero shear."""
import numpy as np
import pytest

import ttcf_inputs as I

TAU = 0.25


@pytest.fixture(scope="module")
def liquid(orc):
    s = I.System(4)  # N = 256
    r, p = I.initial_state(s, 31)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    q = orc.nh_q(s.nf, s.temperature, TAU)
    orc.nh_run(box, st, 1500, s.temperature, s.dt, q, s.nf)
    return s, box, st, q


def test_zero_shear_is_the_mother_step(orc, liquid):
    s, box, st, q = liquid
    r1, p1 = st.r.copy(), st.p.copy()
    vp1, ke1, pe1, zs, k, z1 = orc.nh_sllod_run(box, r1, p1, st.zeta, 0.0, s.dt, s.temperature,
                                                q, s.nf, 200)
    m = orc.NHState(st.r.copy(), st.p.copy(), st.zeta)
    vp2, ke2, pe2 = orc.nh_run(box, m, 200, s.temperature, s.dt, q, s.nf, record=True)
    assert k == 200
    np.testing.assert_allclose(r1, m.r, rtol=0, atol=1e-12)
    np.testing.assert_allclose(p1, m.p, rtol=0, atol=1e-12)
    assert z1 == pytest.approx(m.zeta, abs=1e-12)
    np.testing.assert_allclose(vp1, vp2, rtol=1e-12, atol=1e-9)


def test_extended_energy_balance_fixes_the_signs(orc, liquid):
    """E = K + U + Q zeta^2/2 + nf T int zeta dt obeys dE/dt = -gamma_dot V P_xy (the shear
    work); the thermostat terms cancel. The residual of the integrated balance falls as dt^2,
    and the work is far larger than it (a sign error would miss by twice the work)."""
    s, box, st, q = liquid
    gd = 0.5
    res = []
    for dt in (0.004, 0.002):
        r, p = st.r.copy(), st.p.copy()
        nst = int(round(1.0 / dt))
        vp, ke, pe, zs, _, _ = orc.nh_sllod_run(box, r, p, 0.2, gd, dt, s.temperature, q, s.nf,
                                                nst)
        tr = lambda f: np.concatenate([[0.0], np.cumsum(0.5 * dt * (f[:-1] + f[1:]))])
        e = ke + pe + 0.5 * q * zs ** 2 + s.nf * s.temperature * tr(zs)
        work = -gd * tr(vp)
        resid = (e - e[0]) - work
        res.append(np.abs(resid).max())
        assert np.abs(work).max() > 50 * res[-1]
    assert res[0] / res[1] == pytest.approx(4.0, abs=1.2)


def test_time_reversal_reverses_zeta(orc, liquid):
    """n steps forward; then (p, zeta, gamma_dot) -> (-p, -zeta, -gamma_dot) with the strain
    counter continuing from -n; n steps recover the start with p and zeta reversed."""
    s, box, st, q = liquid
    n = 100
    for gd in (0.0, 0.3, 1.0):
        r, p = st.r.copy(), st.p.copy()
        _, _, _, _, k, z = orc.nh_sllod_run(box, r, p, 0.4, gd, s.dt, s.temperature, q, s.nf, n)
        assert k == n
        p = -p
        _, _, _, _, k2, z2 = orc.nh_sllod_run(box, r, p, -z, -gd, s.dt, s.temperature, q, s.nf, n,
                                              kstep=-n)
        assert k2 == 0
        dr = r - st.r
        dr -= s.box * np.rint(dr / s.box)
        assert np.abs(dr).max() < 1e-9
        assert np.abs(-p - st.p).max() < 1e-9
        assert -z2 == pytest.approx(0.4, abs=1e-9)


def test_sheared_nose_hoover_temperature(orc, liquid):
    """The thermostat holds the mean kinetic temperature (2K/nf) at T under shear."""
    s, box, st, q = liquid
    r, p = st.r.copy(), st.p.copy()
    _, ke, _, _, _, _ = orc.nh_sllod_run(box, r, p, st.zeta, 0.5, s.dt, s.temperature, q, s.nf,
                                         6000)
    t = 2.0 * ke[1:] / s.nf
    assert t.mean() == pytest.approx(s.temperature, rel=0.02)


def test_batch_carries_and_reverses_zeta(orc, liquid):
    """The batch driver starts every daughter from its mapped state with zeta reversed by the
    time-reversing mappings: its series equal single runs from those states."""
    s, box, st, q = liquid
    sr, sp, sz = orc.mother_sample(box, orc.NHState(st.r.copy(), st.p.copy(), st.zeta), 0, 2, 50,
                                   s.temperature, s.dt, q, s.nf, with_zeta=True)
    assert np.all(sz != 0.0)
    state_of = np.repeat(np.arange(2), 4)
    map_of = np.tile(np.arange(4), 2)
    out, used = orc.run_daughters_nh(box, sr, sp, sz, state_of, map_of, np.full(8, 0.1), s.dt,
                                     s.temperature, q, s.nf, 30, nthreads=4)
    for d in range(8):
        r, p = orc.apply_mapping(box, map_of[d], sr[state_of[d]], sp[state_of[d]])
        z = -sz[state_of[d]] if map_of[d] in (1, 3) else sz[state_of[d]]
        vp, _, _, _, _, _ = orc.nh_sllod_run(box, r, p, z, 0.1, s.dt, s.temperature, q, s.nf, 30)
        np.testing.assert_array_equal(out[d], vp)
