"""Pins of the oracle's dynamics: Verlet error scaling, time reversibility, the adiabatic
SLLOD energy balance (fixes the sign of P_xy and Omega), the kinetic-energy constraint,
the Nose-Hoover conserved quantity, momentum conservation, the mapping relations of
Omega and the zero mean of the equilibrium dissipation function."""
import numpy as np
import pytest

import ttcf_inputs as I

TAU = 0.25


@pytest.fixture(scope="module")
def liquid(orc):
    s = I.System(4)  # N = 256, the size of the paper's Example 1
    r, p = I.initial_state(s, 21)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, 1500, s.temperature, s.dt, orc.nh_q(s.nf, s.temperature, TAU), s.nf)
    return s, box, st


def test_nve_error_scales_as_dt_squared(orc, liquid):
    s, box, st = liquid
    fl = []
    for dt in (0.004, 0.002):
        r = st.r.copy()
        p = st.p.copy()
        _, ke, pe, _ = orc.sllod_run(box, r, p, 0.0, dt, int(round(1.0 / dt)), gik=False)
        e = ke + pe
        fl.append(e.std())
        assert abs(e[-1] - e[0]) < 2e-3 * abs(e[0])
    assert fl[0] / fl[1] == pytest.approx(4.0, abs=0.5)


def test_time_reversibility(orc, liquid):
    """n steps forward, then (p, gamma_dot) -> (-p, -gamma_dot) with the strain counter
    continuing from -n retraces the LE offsets; n steps back recover the start."""
    s, box, st = liquid
    n = 100
    for gd in (0.0, 0.2, 1.0):
        r = st.r.copy()
        p = st.p.copy()
        _, _, _, k = orc.sllod_run(box, r, p, gd, s.dt, n, gik=True)
        assert k == n
        p = -p
        _, _, _, k2 = orc.sllod_run(box, r, p, -gd, s.dt, n, gik=True, kstep=-n)
        assert k2 == 0
        dr = r - st.r
        dr -= s.box * np.rint(dr / s.box)
        assert np.abs(dr).max() < 1e-9
        assert np.abs(-p - st.p).max() < 1e-9


def test_adiabatic_sllod_energy_balance(orc, liquid):
    """Without a thermostat, dH0/dt = -gamma_dot V P_xy (pressure-tensor sign). The residual
    of the integrated balance is a discretisation error: it falls as dt^2."""
    s, box, st = liquid
    gd = 0.5
    res = []
    for dt in (0.004, 0.002):
        r = st.r.copy()
        p = st.p.copy()
        nst = int(round(1.0 / dt))
        vp, ke, pe, _ = orc.sllod_run(box, r, p, gd, dt, nst, gik=False)
        h = ke + pe
        integ = np.concatenate([[0.0], np.cumsum(0.5 * dt * (vp[:-1] + vp[1:]))])
        resid = h - h[0] + gd * integ
        res.append(np.abs(resid).max())
        # the work term is not small: the balance is a real test of the sign
        assert abs(gd * integ[-1]) > 50 * res[-1]
    assert res[0] / res[1] == pytest.approx(4.0, abs=1.0)


def test_isokinetic_constraint_and_momentum(orc, liquid):
    s, box, st = liquid
    r = st.r.copy()
    p = st.p.copy()
    _, ke, _, _ = orc.sllod_run(box, r, p, 0.7, s.dt, 300, gik=True)
    assert np.abs(ke / ke[0] - 1.0).max() < 1e-14
    # total momentum stays zero under SLLOD + constraint (sum p_y = 0 keeps sum p_x = 0)
    assert np.abs(p.reshape(3, s.n).sum(axis=1)).max() < 1e-10


def test_nose_hoover_conserved_quantity(orc, liquid):
    """H_NH = K + U + Q zeta^2/2 + nf T int zeta dt is conserved by the Nose-Hoover flow;
    its discrete drift falls with dt. zeta is recovered from the per-step K series:
    zeta_k - zeta_{k-1} = (h/2)[(2K_{k-1} - nf T) + (2K_k - nf T)]/Q."""
    s, box, st = liquid
    q = orc.nh_q(s.nf, s.temperature, TAU)
    drifts = []
    for dt in (0.004, 0.002):
        state = orc.NHState(st.r.copy(), st.p.copy(), 0.3)
        nst = int(round(1.0 / dt))
        _, ke, pe = orc.nh_run(box, state, nst, s.temperature, dt, q, s.nf, record=True)
        g = 2.0 * ke - s.nf * s.temperature
        zeta = 0.3 + np.concatenate([[0.0], np.cumsum(0.5 * dt * (g[:-1] + g[1:]) / q)])
        assert zeta[-1] == pytest.approx(state.zeta, abs=1e-12)
        int_z = np.concatenate([[0.0], np.cumsum(0.5 * dt * (zeta[:-1] + zeta[1:]))])
        hnh = ke + pe + 0.5 * q * zeta ** 2 + s.nf * s.temperature * int_z
        drifts.append(np.abs(hnh - hnh[0]).max())
        assert drifts[-1] < 1e-2 * abs(hnh[0])
    assert drifts[0] > 2.0 * drifts[1]


def test_nose_hoover_temperature(orc, liquid):
    s, box, st = liquid
    q = orc.nh_q(s.nf, s.temperature, TAU)
    state = orc.NHState(st.r.copy(), st.p.copy(), st.zeta)
    _, ke, _ = orc.nh_run(box, state, 8000, s.temperature, s.dt, q, s.nf, record=True)
    t = 2.0 * ke / s.nf
    blocks = t[1:].reshape(4, 2000).mean(axis=1)
    assert t.mean() == pytest.approx(s.temperature, rel=0.02)
    assert blocks.std() < 0.03


def test_mappings_and_dissipation_signs(orc, liquid):
    """Eq. (mappings): P_xy is even under p -> -p and odd under the two x-reflections, so
    Omega(0) keeps its sign under the first mapping and flips under the other two, and the
    four-state sum of Omega(0) vanishes."""
    s, box, st = liquid
    v = []
    for m in range(4):
        rm, pm = orc.apply_mapping(box, m, st.r, st.p)
        assert np.all(rm >= 0.0) and np.all(rm.reshape(3, s.n)[0] < s.box)
        v.append(orc.vpxy(box, rm, pm))
        # every mapping is an involution (up to the rounding of L - (L - x))
        r2, p2 = orc.apply_mapping(box, m, rm, pm)
        assert np.abs(r2 - st.r).max() < 1e-13 and np.array_equal(p2, st.p)
    assert abs(v[0]) > 1e-3
    assert v[1] == pytest.approx(v[0], rel=1e-12)
    assert v[2] == pytest.approx(-v[0], rel=1e-12)
    assert v[3] == pytest.approx(-v[0], rel=1e-12)
    om = orc.omega0(np.array(v), 1e-3, s.temperature)
    assert abs(om.sum()) < 1e-12 * np.abs(om).sum()
    # each daughter's Omega(0) B(0) = -(gamma_dot/T) V P_xy(0)^2 <= 0
    assert np.all(om * np.array(v) <= 0.0)


def test_equilibrium_dissipation_has_zero_mean(orc, liquid):
    """<Omega(0)> = 0 at equilibrium (Mathematical Framework): the mean of P_xy over an
    equilibrium mother is zero within three block standard errors."""
    s, box, st = liquid
    q = orc.nh_q(s.nf, s.temperature, TAU)
    state = orc.NHState(st.r.copy(), st.p.copy(), st.zeta)
    vp, _, _ = orc.nh_run(box, state, 20000, s.temperature, s.dt, q, s.nf, record=True)
    blocks = vp[1:].reshape(40, -1).mean(axis=1)
    se = blocks.std(ddof=1) / np.sqrt(len(blocks))
    assert abs(blocks.mean()) < 3.0 * se
    assert se > 0


def _rk4(fun, y, t, nsub=4000):
    h = t / nsub
    for _ in range(nsub):
        k1 = fun(y)
        k2 = fun(y + 0.5 * h * k1)
        k3 = fun(y + 0.5 * h * k2)
        k4 = fun(y + h * k3)
        y = y + (h / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


def test_isokinetic_kick_solves_its_ode(orc):
    """The closed-form kick equals a fine RK4 solution of dp/dt = F - (F.p/p.p) p."""
    rng = np.random.Generator(np.random.PCG64(9))
    n = 40
    p = rng.standard_normal(3 * n)
    f = 30.0 * rng.standard_normal(3 * n)
    tau = 0.02
    ref = _rk4(lambda q: f - (f @ q) / (q @ q) * q, p.copy(), tau)
    got = orc.iso_kick(p, f, tau)
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()
    assert got @ got == pytest.approx(p @ p, rel=1e-14)
    # F = 0 leaves p unchanged
    assert np.array_equal(orc.iso_kick(p, np.zeros_like(f), tau), p)


def test_isokinetic_shear_solves_its_ode(orc):
    """The rescaled shear flow equals RK4 of dpx/dt = -g py - a px, dpy,z/dt = -a p(y,z)
    with a = -g (sum px py)/(p.p)."""
    rng = np.random.Generator(np.random.PCG64(10))
    n = 40
    p = rng.standard_normal(3 * n)
    g, tau = 3.0, 0.05

    def rhs(q):
        px, py, pz = q[:n], q[n:2 * n], q[2 * n:]
        a = -g * (px @ py) / (q @ q)
        return np.concatenate([-g * py - a * px, -a * py, -a * pz])

    ref = _rk4(rhs, p.copy(), tau)
    got = orc.iso_shear(p, g, tau)
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()


def test_isokinetic_sllod_is_second_order(orc, liquid):
    """Global error at fixed time falls 4x per halving of dt (against a dt/8 reference)."""
    s, box, st = liquid
    t_end, gd = 0.08, 1.0
    finals = {}
    for dt in (0.004, 0.002, 0.0005):
        r = st.r.copy()
        p = st.p.copy()
        orc.sllod_run(box, r, p, gd, dt, int(round(t_end / dt)), gik=True)
        finals[dt] = p
    e1 = np.abs(finals[0.004] - finals[0.0005]).max()
    e2 = np.abs(finals[0.002] - finals[0.0005]).max()
    assert e1 / e2 == pytest.approx(4.0 * (1 - 1 / 64) / (1 - 1 / 16), rel=0.25)
