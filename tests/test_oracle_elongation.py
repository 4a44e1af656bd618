"""Pins of the oracle's planar-elongation daughters (grad u = diag(rate, -rate, 0), a box
deforming as L_x e^e, L_y e^-e, Gaussian isokinetic thermostat, B = P_xx - P_yy) by checks
that do not reuse its formulas: the all-pairs forces against the cell-list and explicit-image
routines, the virial W_xx - W_yy as the strain derivative of the energy, the adiabatic energy
balance dH/dt = -rate V (P_xx - P_yy) with second-order residuals (fixes the sign and size
of the flow terms, hence of Omega), reduction to the zero-shear step at rate 0, the
isokinetic constraint, time reversal, the signs of P_xx - P_yy under the mappings, the
weak-field TTCF against the Green-Kubo integral of the same daughters, and TTCF against the
direct average at a strong rate."""
import numpy as np
import pytest

import ttcf_inputs as I

TAU = 0.25


@pytest.fixture(scope="module")
def liquid(orc):
    s = I.System(3)  # N = 108, L = 5.04
    r, p = I.initial_state(s, 31)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, 1500, s.temperature, s.dt, orc.nh_q(s.nf, s.temperature, TAU), s.nf)
    return s, box, st


def affine(r, n, strain):
    """Positions carried affinely by the strain: x e^strain, y e^-strain."""
    q = r.copy()
    q[:n] *= np.exp(strain)
    q[n:2 * n] *= np.exp(-strain)
    return q


def test_forces_match_cell_list_and_explicit_images(orc, liquid):
    s, box, st = liquid
    f, u, w, npair = orc.pef_forces(box, st.r)
    f2, u2, _, np2 = orc.forces(box, st.r)
    f2 = f2.ravel()
    np.testing.assert_allclose(f, f2, rtol=0, atol=1e-12 * np.abs(f2).max())
    assert u == pytest.approx(u2, rel=1e-13)
    assert npair == np2
    # W_xx - W_yy: the pair part of V (P_xx - P_yy), from the observables routine at p = 0
    n1 = orc.observables(box, st.r, np.zeros(3 * s.n))[0]
    assert w == pytest.approx(n1 * s.volume, rel=1e-12)
    # a strained box against the sum over explicit periodic images
    e = 0.3
    bs = orc.pef_box(box, e)
    rs = affine(st.r, s.n, e)
    f, u, w, npair = orc.pef_forces(bs, rs)
    f3, u3, _, np3 = orc.forces(bs, rs, brute=True)
    f3 = f3.ravel()
    np.testing.assert_allclose(f, f3, rtol=0, atol=1e-11 * np.abs(f3).max())
    assert u == pytest.approx(u3, rel=1e-12)
    assert npair == np3
    with pytest.raises(RuntimeError):      # an edge below 2 r_c
        orc.pef_forces(orc.pef_box(box, 0.9), affine(st.r, s.n, 0.9))


@pytest.mark.parametrize("e", [0.0, 0.2])
def test_virial_is_the_strain_derivative_of_the_energy(orc, liquid, e):
    # U(e + d) of the affinely deformed configuration: dU/dd = -(W_xx - W_yy)
    s, box, st = liquid
    d = 1e-6
    r0 = affine(st.r, s.n, e)
    _, _, w, _ = orc.pef_forces(orc.pef_box(box, e), r0)
    up = orc.pef_forces(orc.pef_box(box, e + d), affine(r0, s.n, d))[1]
    um = orc.pef_forces(orc.pef_box(box, e - d), affine(r0, s.n, -d))[1]
    assert (up - um) / (2 * d) == pytest.approx(-w, rel=1e-6)


def test_zero_rate_is_the_zero_shear_step(orc, liquid):
    s, box, st = liquid
    r1, p1 = st.r.copy(), st.p.copy()
    vn1, k1, u1, e = orc.pef_run(box, r1, p1, 0.0, s.dt, 100)
    r2, p2 = st.r.copy(), st.p.copy()
    orc.sllod_run(box, r2, p2, 0.0, s.dt, 100)
    assert e == 0.0
    np.testing.assert_allclose(r1, r2, rtol=0, atol=1e-10 * s.box)
    np.testing.assert_allclose(p1, p2, rtol=0, atol=1e-10)
    # the recorded series is V (P_xx - P_yy) of the observables routine
    assert vn1[-1] == pytest.approx(orc.observables(box, r1, p1)[0] * s.volume, rel=1e-10)


@pytest.mark.parametrize("rate", [0.5, -0.3])
def test_adiabatic_energy_balance_fixes_the_flow_terms(orc, liquid, rate):
    s, box, st = liquid

    def residual(dt, nsteps, sign=1.0):
        r, p = st.r.copy(), st.p.copy()
        vn1, k, u, _ = orc.pef_run(box, r, p, rate, dt, nsteps, gik=False)
        h = k + u
        work = -sign * rate * np.concatenate([[0.0], np.cumsum(0.5 * dt * (vn1[1:] + vn1[:-1]))])
        return np.abs((h - h[0]) - work).max(), np.abs(work).max()

    res1, work = residual(s.dt, 160)
    res2, _ = residual(s.dt / 2, 320)
    assert work > 20 * res1             # the flow does visible work, and the balance holds
    assert 3.0 < res1 / res2 < 5.0      # with a second-order residual
    wrong, _ = residual(s.dt, 160, sign=-1.0)
    assert wrong > 10 * res1            # a flow term of the wrong sign fails by the whole work


def test_isokinetic_constraint_and_time_reversal(orc, liquid):
    s, box, st = liquid
    r, p = st.r.copy(), st.p.copy()
    k0 = 0.5 * (p @ p)
    vn1, k, u, e = orc.pef_run(box, r, p, 0.8, s.dt, 200)
    np.testing.assert_allclose(k, k0, rtol=1e-13)
    assert e == pytest.approx(0.8 * 200 * s.dt, rel=1e-14)
    assert abs(vn1[-1] - vn1[0]) > 10.0  # the flow builds up a normal-stress difference
    # reversing p and the rate from the final strain retraces the path back to strain 0
    p = -p
    _, _, _, e2 = orc.pef_run(box, r, p, -0.8, s.dt, 200, strain0=e)
    assert abs(e2) < 1e-14
    dr = r - st.r
    dr -= s.box * np.rint(dr / s.box)
    assert np.abs(dr).max() < 1e-8
    assert np.abs(-p - st.p).max() < 1e-8


def test_normal_stress_signs_under_the_mappings(orc, liquid):
    s, box, st = liquid
    n = s.n
    n1 = []
    for m in range(4):
        rm, pm = orc.map_pef(box, m, st.r, st.p)
        n1.append(orc.observables(box, rm, pm)[0])
        if m == 3:   # exchanged axes and reversed momenta
            np.testing.assert_array_equal(rm[:n], st.r[n:2 * n])
            np.testing.assert_array_equal(pm[n:2 * n], -st.p[:n])
            np.testing.assert_array_equal(pm[2 * n:], -st.p[2 * n:])
    np.testing.assert_allclose(np.array(n1) / n1[0], [1.0, 1.0, -1.0, -1.0], rtol=1e-12)


@pytest.fixture(scope="module")
def start_states(orc):
    s = I.System(3)
    r, p = I.initial_state(s, 7)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    q = orc.nh_q(s.nf, s.temperature, TAU)
    sr, sp = orc.mother_sample(box, st, 1000, 24, 100, s.temperature, s.dt, q, s.nf)
    return s, box, sr, sp


def test_weak_field_ttcf_is_the_green_kubo_integral(orc, start_states):
    # TTCF(t)/rate at rate -> 0 is -(1/(T V)) int_0^t <X(0) X(s)> ds, X = V (P_xx - P_yy),
    # with X from the field-free daughters of the same mapped start states
    s, box, sr, sp = start_states
    nst, ns = 200, 16
    state_of = np.repeat(np.arange(ns), 4)
    map_of = np.tile(np.arange(4), ns)
    rate = 1e-6
    x_f, _ = orc.run_daughters_pef(box, sr, sp, state_of, map_of, np.full(4 * ns, rate), s.dt,
                                   nst, nthreads=8)
    x_0, _ = orc.run_daughters_pef(box, sr, sp, state_of, map_of, np.zeros(4 * ns), s.dt, nst,
                                   nthreads=8)
    vol = s.volume
    resp = orc.ttcf_response(x_f / vol, x_f[:, 0], np.full(4 * ns, rate), s.temperature, s.dt)
    acf = (x_0[:, :1] * x_0).mean(axis=0) / vol
    gk = np.concatenate([[0.0], np.cumsum(0.5 * s.dt * (acf[1:] + acf[:-1]))]) / s.temperature
    assert abs(resp.ttcf[0]) < 1e-12     # <P_xx - P_yy> vanishes over the mapped start states
    np.testing.assert_allclose(resp.ttcf[1:] / rate, -gk[1:], rtol=1e-4,
                               atol=1e-6 * np.abs(gk).max())
    assert gk[1] > 0 and resp.ttcf[1] < 0


def test_ttcf_agrees_with_the_direct_average_at_a_strong_rate(orc, start_states):
    # At rate 0.5 the direct average resolves the response: TTCF, built from Omega(0) and the
    # same trajectories, must agree with it; an Omega of the wrong sign or size would not
    s, box, sr, sp = start_states
    nst, ns, rate = 200, 24, 0.5
    state_of = np.repeat(np.arange(ns), 4)
    map_of = np.tile(np.arange(4), ns)
    x, _ = orc.run_daughters_pef(box, sr, sp, state_of, map_of, np.full(4 * ns, rate), s.dt,
                                 nst, nthreads=8)
    resp = orc.ttcf_response(x / s.volume, x[:, 0], np.full(4 * ns, rate), s.temperature, s.dt)
    for k in (50, 100, 200):
        se = np.hypot(resp.ttcf_se[k], resp.dav_se[k])
        assert resp.dav[k] < -4 * resp.dav_se[k]     # compression along y raises P_yy
        assert abs(resp.ttcf[k] - resp.dav[k]) < 3 * se
    wrong = orc.ttcf_response(x / s.volume, -x[:, 0], np.full(4 * ns, rate), s.temperature, s.dt)
    for k in (50, 100):
        assert abs(wrong.ttcf[k] - resp.dav[k]) > 4 * np.hypot(wrong.ttcf_se[k], resp.dav_se[k])


def test_nose_hoover_elongation_step(orc, liquid):
    """Nose-Hoover planar elongation: at rate 0 the zero-shear Nose-Hoover SLLOD step; the
    extended energy K + U + Q zeta^2/2 + nf T int zeta changes by -rate int V (P_xx - P_yy)
    with a second-order residual (and fails by the whole work with the wrong sign);
    (p, zeta, rate) -> (-p, -zeta, -rate) from the final strain retraces the path."""
    s, box, st = liquid
    q = orc.nh_q(s.nf, s.temperature, TAU)
    z0 = 0.3
    r1, p1 = st.r.copy(), st.p.copy()
    orc.nh_pef_run(box, r1, p1, z0, 0.0, s.dt, s.temperature, q, s.nf, 80)
    r2, p2 = st.r.copy(), st.p.copy()
    orc.nh_sllod_run(box, r2, p2, z0, 0.0, s.dt, s.temperature, q, s.nf, 80)
    np.testing.assert_allclose(r1, r2, rtol=0, atol=1e-10 * s.box)
    np.testing.assert_allclose(p1, p2, rtol=0, atol=1e-10)

    rate = 0.6

    def residual(dt, nsteps, sign=1.0):
        r, p = st.r.copy(), st.p.copy()
        vn1, k, u, zs, _, _ = orc.nh_pef_run(box, r, p, z0, rate, dt, s.temperature, q, s.nf,
                                             nsteps)
        izeta = np.concatenate([[0.0], np.cumsum(0.5 * dt * (zs[1:] + zs[:-1]))])
        h = k + u + 0.5 * q * zs ** 2 + s.nf * s.temperature * izeta
        work = -sign * rate * np.concatenate([[0.0], np.cumsum(0.5 * dt * (vn1[1:] + vn1[:-1]))])
        return np.abs((h - h[0]) - work).max(), np.abs(work).max()

    res1, work = residual(s.dt, 160)
    res2, _ = residual(s.dt / 2, 320)
    assert work > 20 * res1
    assert 3.0 < res1 / res2 < 5.0
    wrong, _ = residual(s.dt, 160, sign=-1.0)
    assert wrong > 10 * res1
    r, p = st.r.copy(), st.p.copy()
    *_, z1, e1 = orc.nh_pef_run(box, r, p, z0, rate, s.dt, s.temperature, q, s.nf, 250)
    p = -p
    *_, z2, e2 = orc.nh_pef_run(box, r, p, -z1, -rate, s.dt, s.temperature, q, s.nf, 250,
                                strain0=e1)
    assert abs(e2) < 1e-14
    dr = r - st.r
    dr -= s.box * np.rint(dr / s.box)
    assert np.abs(dr).max() < 1e-8
    assert np.abs(-p - st.p).max() < 1e-8
    assert abs(-z2 - z0) < 1e-9
