"""Pins of the oracle's colour-field daughters (the colour-conductivity field: charge +1 on
even atoms, -1 on odd ones, force c_i F_e along x, Gaussian isokinetic thermostat) by checks
that do not reuse its formulas: the adiabatic energy balance dH/dt = F_e sum_i c_i p_x,i with
second-order residuals (fixes the sign and size of the field term, hence of Omega), reduction
to the pinned zero-shear SLLOD step at F_e = 0, the isokinetic constraint, time reversal, the
signs of J_x(0) under Eq. (mappings), and the weak-field TTCF against the Green-Kubo integral
of the same daughters' equilibrium current autocorrelation."""
import numpy as np
import pytest

import ttcf_inputs as I

TAU = 0.25


@pytest.fixture(scope="module")
def liquid(orc):
    s = I.System(3)  # N = 108
    r, p = I.initial_state(s, 23)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, 1500, s.temperature, s.dt, orc.nh_q(s.nf, s.temperature, TAU), s.nf)
    return s, box, st


def test_zero_field_is_the_zero_shear_step(orc, liquid):
    s, box, st = liquid
    r1, p1 = st.r.copy(), st.p.copy()
    j, k1, u1 = orc.colour_run(box, r1, p1, 0.0, s.dt, 100)
    r2, p2 = st.r.copy(), st.p.copy()
    vp, k2, u2, _ = orc.sllod_run(box, r2, p2, 0.0, s.dt, 100)
    np.testing.assert_array_equal(r1, r2)
    np.testing.assert_array_equal(p1, p2)
    np.testing.assert_array_equal(u1, u2)
    c = orc.colour_charges(s.n)
    assert j[-1] == pytest.approx(c @ p1[: s.n], rel=1e-14)


@pytest.mark.parametrize("fe", [0.5, -0.3])
def test_adiabatic_energy_balance_fixes_the_field_term(orc, liquid, fe):
    s, box, st = liquid

    def residual(dt, nsteps):
        r, p = st.r.copy(), st.p.copy()
        j, k, u = orc.colour_run(box, r, p, fe, dt, nsteps, gik=False)
        h = k + u
        work = fe * np.concatenate([[0.0], np.cumsum(0.5 * dt * (j[1:] + j[:-1]))])
        return np.abs((h - h[0]) - work).max(), np.abs(work).max()

    res1, work = residual(s.dt, 200)
    res2, _ = residual(s.dt / 2, 400)
    assert work > 20 * res1             # the field does visible work, and the balance holds
    assert 3.0 < res1 / res2 < 5.0      # with a second-order residual
    # with the field term of the wrong sign the balance fails by the whole work
    r, p = st.r.copy(), st.p.copy()
    j, k, u = orc.colour_run(box, r, p, fe, s.dt, 200, gik=False)
    work_wrong = -fe * np.concatenate([[0.0], np.cumsum(0.5 * s.dt * (j[1:] + j[:-1]))])
    assert np.abs((k + u - k[0] - u[0]) - work_wrong).max() > 10 * res1


def test_isokinetic_constraint_and_time_reversal(orc, liquid):
    s, box, st = liquid
    r, p = st.r.copy(), st.p.copy()
    k0 = 0.5 * (p @ p)
    j, k, u = orc.colour_run(box, r, p, 0.8, s.dt, 300)
    np.testing.assert_allclose(k, k0, rtol=1e-13)
    assert abs(j[-1] - j[0]) > 1.0      # the field drives a current
    # the colour force is time-even: reversing p retraces the path under the same field
    p = -p
    orc.colour_run(box, r, p, 0.8, s.dt, 300)
    dr = r - st.r
    dr -= s.box * np.rint(dr / s.box)
    assert np.abs(dr).max() < 1e-8
    assert np.abs(-p - st.p).max() < 1e-8


def test_current_signs_under_the_mappings(orc, liquid):
    s, box, st = liquid
    c = orc.colour_charges(s.n)
    j0 = c @ st.p[: s.n]
    signs = []
    for m in range(4):
        rm, pm = orc.apply_mapping(box, m, st.r, st.p)
        signs.append((c @ pm[: s.n]) / j0)
    np.testing.assert_allclose(signs, [1.0, -1.0, -1.0, 1.0], rtol=1e-14)


def test_weak_field_ttcf_is_the_green_kubo_integral(orc):
    # The TTCF per unit field at F_e -> 0 is (V/T) int_0^t <J(0) J(s)> ds over the same
    # mapped start states, with J from the field-free daughters (the linear limit)
    s = I.System(3)
    r, p = I.initial_state(s, 5)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    q = orc.nh_q(s.nf, s.temperature, TAU)
    sr, sp = orc.mother_sample(box, st, 1000, 16, 100, s.temperature, s.dt, q, s.nf)
    nst = 200
    state_of = np.repeat(np.arange(16), 4)
    map_of = np.tile(np.arange(4), 16)
    fe = 1e-6
    j_f, _ = orc.run_daughters_colour(box, sr, sp, state_of, map_of, np.full(64, fe), s.dt, nst,
                                      nthreads=8)
    j_0, _ = orc.run_daughters_colour(box, sr, sp, state_of, map_of, np.zeros(64), s.dt, nst,
                                      nthreads=8)
    vol = s.volume
    om = orc.omega0_colour(j_f[:, 0], fe, s.temperature)
    resp = orc.ttcf_response(j_f / vol, j_f[:, 0], np.full(64, fe), s.temperature, s.dt,
                             omega=om)
    acf = (j_0[:, :1] * j_0).mean(axis=0) / vol          # <J(0) J(s)> V over the daughters
    gk = np.concatenate([[0.0], np.cumsum(0.5 * s.dt * (acf[1:] + acf[:-1]))]) / s.temperature
    # <J(0)> vanishes over the mapped daughters, so TTCF(t)/F_e = <J(0)>/F_e + GK(t) = GK(t)
    assert abs(resp.ttcf[0]) < 1e-12
    np.testing.assert_allclose(resp.ttcf[1:] / fe, gk[1:], rtol=1e-4,
                               atol=1e-6 * np.abs(gk).max())
    # the initial rise is (V/T) <J(0)^2> dt / 2 per step, positive; a field term of the wrong
    # sign in Omega would turn the whole curve over
    assert gk[1] > 0 and resp.ttcf[1] > 0


def test_nose_hoover_colour_step(orc, liquid):
    """Nose-Hoover colour daughters: at F_e = 0 the zero-shear Nose-Hoover SLLOD step; the
    extended energy K + U + Q zeta^2/2 + nf T int zeta changes by the field work
    F_e int V J_x with a second-order residual; (p, zeta) -> (-p, -zeta) retraces the path under
    the same field."""
    s, box, st = liquid
    q = orc.nh_q(s.nf, s.temperature, TAU)
    z0 = 0.3
    r1, p1 = st.r.copy(), st.p.copy()
    orc.nh_colour_run(box, r1, p1, z0, 0.0, s.dt, s.temperature, q, s.nf, 80)
    r2, p2 = st.r.copy(), st.p.copy()
    orc.nh_sllod_run(box, r2, p2, z0, 0.0, s.dt, s.temperature, q, s.nf, 80)
    np.testing.assert_array_equal(r1, r2)
    np.testing.assert_array_equal(p1, p2)

    fe = 0.6

    def residual(dt, nsteps):
        r, p = st.r.copy(), st.p.copy()
        j, k, u, zs, _ = orc.nh_colour_run(box, r, p, z0, fe, dt, s.temperature, q, s.nf, nsteps)
        izeta = np.concatenate([[0.0], np.cumsum(0.5 * dt * (zs[1:] + zs[:-1]))])
        h = k + u + 0.5 * q * zs ** 2 + s.nf * s.temperature * izeta
        work = fe * np.concatenate([[0.0], np.cumsum(0.5 * dt * (j[1:] + j[:-1]))])
        return np.abs((h - h[0]) - work).max(), np.abs(work).max()

    res1, work = residual(s.dt, 200)
    res2, _ = residual(s.dt / 2, 400)
    assert work > 20 * res1
    assert 3.0 < res1 / res2 < 5.0
    r, p = st.r.copy(), st.p.copy()
    *_, z1 = orc.nh_colour_run(box, r, p, z0, fe, s.dt, s.temperature, q, s.nf, 300)
    p = -p
    *_, z2 = orc.nh_colour_run(box, r, p, -z1, fe, s.dt, s.temperature, q, s.nf, 300)
    dr = r - st.r
    dr -= s.box * np.rint(dr / s.box)
    assert np.abs(dr).max() < 1e-8
    assert np.abs(-p - st.p).max() < 1e-8
    assert abs(-z2 - z0) < 1e-9
