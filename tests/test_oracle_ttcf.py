"""Pins of the oracle's TTCF estimator against what the paper and statistical mechanics fix:
a closed-form integral on synthetic series, TTCF = DAV where both are valid (strong field),
the equilibrium (Green-Kubo) limit at weak field, linear response in gamma_dot, the
initial slope of the direct average (-gamma_dot G_inf, G_inf = (V/T)<P_xy^2>), and the
exact zero of the mapped direct average at t = 0."""
import numpy as np
import pytest

import ttcf_inputs as I

NS = 256          # start states
NSTEPS = 400      # daughter steps
TAU = 0.25


def test_estimator_closed_form():
    """For B_d(t) = a_d + b_d t the trapezoid rule is exact:
    TTCF(t) = <B(0)> + <Omega_d (a_d t + b_d t^2/2)>."""
    import oracle as orc
    rng = np.random.Generator(np.random.PCG64(3))
    nd, nt, dt, temp = 16, 21, 0.01, 0.7
    a = rng.standard_normal(nd)
    b = rng.standard_normal(nd)
    t = dt * np.arange(nt)
    series = a[:, None] + b[:, None] * t[None, :]
    vp0 = rng.standard_normal(nd) * 10.0
    gam = np.full(nd, 0.3)
    res = orc.ttcf_response(series, vp0, gam, temp, dt)
    om = -(0.3 / temp) * vp0
    per_d = a[:, None] + om[:, None] * (a[:, None] * t + 0.5 * b[:, None] * t ** 2)
    np.testing.assert_allclose(res.ttcf, per_d.mean(axis=0), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(res.dav, series.mean(axis=0), rtol=1e-12, atol=1e-12)
    blocks = per_d.reshape(4, 4, nt).mean(axis=1)
    np.testing.assert_allclose(res.ttcf_se, blocks.std(axis=0, ddof=1) / 2.0, rtol=1e-10)


@pytest.fixture(scope="module")
def ensemble(orc):
    """A WCA mother (N=108, rho=0.8442, T=0.722) melted at T=2, equilibrated, then sampled
    every 100 steps; the 4 mapped daughters of every start state at several shear rates."""
    s = I.System(3)
    r, p = I.initial_state(s, 7)
    box = orc.make_box(s.n, s.box)
    q = orc.nh_q(s.nf, s.temperature, TAU)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, 1000, 2.0, s.dt, q, s.nf)
    sr, sp = orc.mother_sample(box, st, 2000, NS, 100, s.temperature, s.dt, q, s.nf)
    state_of = np.repeat(np.arange(NS), 4)
    map_of = np.tile(np.arange(4), NS)
    out = {}
    for gd in (1.0, 1e-4, 1e-6):
        vp, _ = orc.run_daughters(box, sr, sp, state_of, map_of, np.full(4 * NS, gd), s.dt,
                                  NSTEPS, nthreads=8)
        out[gd] = orc.ttcf_response(vp / s.volume, vp[:, 0], np.full(4 * NS, gd),
                                    s.temperature, s.dt)
        out[gd].b0 = vp[:, 0] / s.volume
    return s, box, st, q, out


@pytest.mark.slow
def test_ttcf_equals_direct_average_at_strong_field(ensemble):
    """Example 1: DAV and TTCF agree at high shear rates. Paired per-state difference of the
    two estimators within 3 block standard errors at several times."""
    s, _, _, _, out = ensemble
    res = out[1.0]
    for k in (10, 50, 100, 200, 400):
        diff = res.g[:, k] - res.d[:, k]
        se = diff.std(ddof=1) / np.sqrt(NS)
        assert abs(diff.mean()) < 3.0 * se, k
    # the response is a real signal here: shear stress many DAV standard errors from 0
    assert abs(res.dav[200]) > 50 * res.dav_se[200]


@pytest.mark.slow
def test_direct_average_vanishes_at_t0_and_initial_slope(ensemble):
    """<P_xy(0)> over the four mappings is exactly zero, so DAV(0) = 0 with zero spread.
    The initial slope of DAV is -gamma_dot G_inf with G_inf = (V/T)<P_xy(0)^2> (the zero-lag
    Green-Kubo value); the DAV itself never uses Omega, so this pins Omega's normalisation."""
    s, _, _, _, out = ensemble
    res = out[1e-4]
    assert abs(res.dav[0]) < 1e-13 and res.dav_se[0] < 1e-13
    # G_inf from the start states (the four mapped copies share |P_xy(0)|)
    sq = (res.b0 ** 2).reshape(NS, 4).mean(axis=1)
    g_inf = s.volume / s.temperature * sq.mean()
    se = s.volume / s.temperature * sq.std(ddof=1) / np.sqrt(NS)
    slope = res.dav[1] / (1e-4 * s.dt)
    assert slope == pytest.approx(-g_inf, abs=3.0 * se + 0.01 * g_inf)


@pytest.mark.slow
def test_linear_response_in_shear_rate(ensemble):
    """In the linear regime the TTCF response per unit shear rate does not depend on
    gamma_dot: 1e-4 and 1e-6 give the same eta(t) to far below its standard error."""
    s, _, _, _, out = ensemble
    eta4 = -out[1e-4].ttcf / 1e-4
    eta6 = -out[1e-6].ttcf / 1e-6
    se = out[1e-6].ttcf_se / 1e-6
    assert np.all(np.abs(eta4 - eta6)[1:] < 0.02 * se[1:])
    # the TTCF standard error is proportional to gamma_dot (SNR model, Eq. SNR)
    ratio = out[1e-4].ttcf_se[1:] / out[1e-6].ttcf_se[1:]
    np.testing.assert_allclose(ratio, 100.0, rtol=0.02)


@pytest.mark.slow
def test_weak_field_limit_is_green_kubo(orc, ensemble):
    """TTCF generalises Green-Kubo: at gamma_dot = 1e-6 the viscosity -TTCF(t)/gamma_dot
    equals (V/T) int_0^t <P_xy(0)P_xy(s)> ds from a long equilibrium mother, within 3
    combined standard errors at t = 100 and 200 steps."""
    s, box, st, q, out = ensemble
    state = orc.NHState(st.r.copy(), st.p.copy(), st.zeta)
    vp, _, _ = orc.nh_run(box, state, 60000, s.temperature, s.dt, q, s.nf, record=True)
    pxy = vp[1:] / s.volume
    nb = 12
    blk = len(pxy) // nb
    etas = np.array([orc.green_kubo(pxy[i * blk:(i + 1) * blk], s.volume, s.temperature,
                                    s.dt, 200)[1] for i in range(nb)])
    eta_gk = etas.mean(axis=0)
    se_gk = etas.std(axis=0, ddof=1) / np.sqrt(nb)
    eta_tt = -out[1e-6].ttcf / 1e-6
    se_tt = out[1e-6].ttcf_se / 1e-6
    for k in (100, 200):
        comb = np.hypot(se_gk[k], se_tt[k])
        assert abs(eta_tt[k] - eta_gk[k]) < 3.0 * comb, (k, eta_tt[k], eta_gk[k], comb)
    assert eta_gk[200] > 5 * se_gk[200]


def test_modified_integrand_closed_forms(orc):
    """Eq. (corr_modified) on synthetic series: with B the same constant for every daughter
    the modified integrand is zero, so the estimate is B at all t, while Eq. (integrand)
    drifts by B <Omega(0)> t when the sample's <Omega(0)> is not zero; with B linear in time
    the estimate is the closed form of the sample covariance."""
    rng = np.random.Generator(np.random.PCG64(11))
    nd, nt, dt, T = 12, 7, 0.1, 0.9
    vp0 = rng.standard_normal(nd)
    gam = np.full(nd, 0.3)
    om = -(gam / T) * vp0
    t = dt * np.arange(nt)
    b = np.full((nd, nt), 1.7)
    m, se = orc.ttcf_response_modified(b, vp0, gam, T, dt, n_maps=1)
    np.testing.assert_allclose(m, 1.7, rtol=0, atol=1e-14)
    np.testing.assert_allclose(se, 0.0, atol=1e-14)
    plain = orc.ttcf_response(b, vp0, gam, T, dt, n_maps=1)
    np.testing.assert_allclose(plain.ttcf, 1.7 + 1.7 * om.mean() * t, rtol=1e-12)
    a = rng.standard_normal(nd)
    c = rng.standard_normal(nd)
    b = a[:, None] + c[:, None] * t[None, :]
    m, _ = orc.ttcf_response_modified(b, vp0, gam, T, dt, n_maps=1)
    cov = lambda u, v: (u * v).mean() - u.mean() * v.mean()
    exact = a.mean() + cov(om, a) * t + 0.5 * cov(om, c) * t * t
    np.testing.assert_allclose(m, exact, rtol=1e-12, atol=1e-14)


def test_modified_equals_plain_with_the_four_mappings(orc):
    """With all four mappings <Omega(0)> vanishes state by state, so Eq. (corr_modified)
    equals Eq. (integrand); the estimator is then linear in the state means, and the
    jackknife error equals the block standard error (an identity for linear estimators).
    Without the mappings the correction is active."""
    s = I.System(3)
    r, p = I.initial_state(s, 13)
    box = orc.make_box(s.n, s.box)
    q = orc.nh_q(s.nf, s.temperature, TAU)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, 600, 2.0, s.dt, q, s.nf)
    ns, nst, gd = 16, 60, 0.5
    sr, sp = orc.mother_sample(box, st, 600, ns, 50, s.temperature, s.dt, q, s.nf)
    vp, _ = orc.run_daughters(box, sr, sp, np.repeat(np.arange(ns), 4), np.tile(np.arange(4), ns),
                              np.full(4 * ns, gd), s.dt, nst, nthreads=8)
    b = vp / s.volume
    g = np.full(4 * ns, gd)
    plain = orc.ttcf_response(b, vp[:, 0], g, s.temperature, s.dt)
    m, se = orc.ttcf_response_modified(b, vp[:, 0], g, s.temperature, s.dt)
    scale = np.abs(plain.g).max()
    assert np.abs(m - plain.ttcf).max() <= 1e-12 * scale
    np.testing.assert_allclose(se[1:], plain.ttcf_se[1:], rtol=1e-9)
    # the unmapped daughters alone: the sample <Omega(0)> is not zero and the estimates differ
    one = np.arange(0, 4 * ns, 4)
    p1 = orc.ttcf_response(b[one], vp[one, 0], g[one], s.temperature, s.dt, n_maps=1)
    m1, _ = orc.ttcf_response_modified(b[one], vp[one, 0], g[one], s.temperature, s.dt, n_maps=1)
    assert np.abs(m1 - p1.ttcf).max() > 1e-6 * scale
