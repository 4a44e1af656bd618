"""Pins of the oracle's mixed-flow daughters (u_x = erate x + srate y, u_y = -erate y, the
triclinic cell H(t) = exp(A t) diag(L) carried by the flow, B = J = (erate (P_xx - P_yy) +
srate P_xy) / |rate|) by checks that do not reuse its formulas: forces in the tilted cell
against the Lees-Edwards sliding brick with the same image lattice and against the
orthorhombic routine at srate = 0; pure shear (erate = 0) against the Lees-Edwards SLLOD
oracle, and pure elongation (srate = 0) against the planar-elongation oracle; the adiabatic
energy balance dH/dt = -V grad u : P with second-order residuals and the wrong-sign check;
the Nose-Hoover extended-energy balance; time reversal; the signs of the flux under the
mappings; and TTCF against the direct average at a strong field."""
import numpy as np
import pytest

import ttcf_inputs as I

TAU = 0.25


@pytest.fixture(scope="module")
def liquid(orc):
    s = I.System(3)  # N = 108, L = 5.04
    r, p = I.initial_state(s, 41)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, 1500, s.temperature, s.dt, orc.nh_q(s.nf, s.temperature, TAU), s.nf)
    return s, box, st


def carried(r, n, h, L):
    """Positions of the undeformed box carried into the cell h (r -> H H0^-1 r)."""
    q = r.copy()
    q[:n] = r[:n] * (h[0] / L) + r[n:2 * n] * (h[1] / L)
    q[n:2 * n] = r[n:2 * n] * (h[2] / L)
    return q


def test_tilted_cell_forces_match_the_sliding_brick(orc, liquid):
    s, box, st = liquid
    n = s.n
    for er, sr, t in ((0.0, 1.0, 0.3), (0.0, -0.7, 0.5), (0.4, 0.0, 0.5)):
        h = orc.mix_cell(box, er, sr, t)
        r = carried(st.r, n, h, s.box)
        f, u, wn, wxy, npair = orc.mix_forces(box, h, r)
        if er == 0.0:
            # the same image lattice as the sliding brick with offset H_xy
            rl = r.copy()
            rl[:n] = np.mod(rl[:n], s.box)
            fl, ul, wl, nl = orc.forces(box, rl, dxle=float(np.fmod(h[1], s.box)), brute=True)
            np.testing.assert_allclose(f, fl.ravel(), rtol=0, atol=1e-11 * np.abs(fl).max())
            assert u == pytest.approx(ul, rel=1e-12)
            assert wxy == pytest.approx(wl, rel=1e-11)
            assert npair == nl
        else:
            fp, up, wp, _ = orc.pef_forces(orc.pef_box(box, er * t), r)
            np.testing.assert_allclose(f, fp, rtol=0, atol=1e-11 * np.abs(fp).max())
            assert wn == pytest.approx(wp, rel=1e-11)


def test_pure_shear_is_the_sliding_brick_sllod(orc, liquid):
    s, box, st = liquid
    r1, p1 = st.r.copy(), st.p.copy()
    vj, _, _, t, _ = orc.mix_run(box, r1, p1, 0.0, 0.8, s.dt, 100)
    r2, p2 = st.r.copy(), st.p.copy()
    vp, _, _, _ = orc.sllod_run(box, r2, p2, 0.8, s.dt, 100)
    # J = P_xy (sign of the shear rate) and the momenta agree; positions agree modulo the
    # image lattice
    np.testing.assert_allclose(vj, vp, rtol=0, atol=1e-9 * np.abs(vp).max())
    np.testing.assert_allclose(p1, p2, rtol=0, atol=1e-9)
    assert t == pytest.approx(100 * s.dt, rel=1e-14)


def test_pure_elongation_is_the_planar_elongation_oracle(orc, liquid):
    s, box, st = liquid
    r1, p1 = st.r.copy(), st.p.copy()
    vj, _, _, _, _ = orc.mix_run(box, r1, p1, -0.6, 0.0, s.dt, 100)
    r2, p2 = st.r.copy(), st.p.copy()
    vn, _, _, _ = orc.pef_run(box, r2, p2, -0.6, s.dt, 100)
    # J = (erate N1) / |erate| = -N1 for a negative rate
    np.testing.assert_allclose(vj, -vn, rtol=0, atol=1e-9 * np.abs(vn).max())
    np.testing.assert_allclose(r1, r2, rtol=0, atol=1e-9 * s.box)
    np.testing.assert_allclose(p1, p2, rtol=0, atol=1e-9)


@pytest.mark.parametrize("er,sr", [(0.3, 0.5), (-0.4, 0.2)])
def test_adiabatic_energy_balance_fixes_the_flow_terms(orc, liquid, er, sr):
    s, box, st = liquid
    rn = np.hypot(er, sr)

    def residual(dt, nsteps, sign=1.0):
        r, p = st.r.copy(), st.p.copy()
        vj, k, u, _, _ = orc.mix_run(box, r, p, er, sr, dt, nsteps, gik=False)
        h = k + u
        work = -sign * rn * np.concatenate([[0.0], np.cumsum(0.5 * dt * (vj[1:] + vj[:-1]))])
        return np.abs((h - h[0]) - work).max(), np.abs(work).max()

    res1, work = residual(s.dt, 160)
    res2, _ = residual(s.dt / 2, 320)
    assert work > 20 * res1
    assert 3.0 < res1 / res2 < 5.0
    wrong, _ = residual(s.dt, 160, sign=-1.0)
    assert wrong > 10 * res1


def test_nose_hoover_energy_balance_and_isokinetic_constraint(orc, liquid):
    s, box, st = liquid
    er, sr = 0.3, -0.5
    rn = np.hypot(er, sr)
    q = orc.nh_q(s.nf, s.temperature, TAU)

    def residual(dt, nsteps):
        r, p = st.r.copy(), st.p.copy()
        zs = []
        # zeta after each step from single-step runs (the run returns only the final value)
        z = 0.3
        vj_all, k_all, u_all = [], [], []
        t = 0.0
        for i in range(nsteps):
            vj, k, u, t, z = orc.mix_run(box, r, p, er, sr, dt, 1, t0=t, zeta=z,
                                         temperature=s.temperature, q=q, nf=s.nf)
            if i == 0:
                vj_all.append(vj[0])
                k_all.append(k[0])
                u_all.append(u[0])
                zs.append(0.3)
            vj_all.append(vj[1])
            k_all.append(k[1])
            u_all.append(u[1])
            zs.append(z)
        vj, k, u, zs = map(np.array, (vj_all, k_all, u_all, zs))
        izeta = np.concatenate([[0.0], np.cumsum(0.5 * dt * (zs[1:] + zs[:-1]))])
        h = k + u + 0.5 * q * zs ** 2 + s.nf * s.temperature * izeta
        work = -rn * np.concatenate([[0.0], np.cumsum(0.5 * dt * (vj[1:] + vj[:-1]))])
        return np.abs((h - h[0]) - work).max(), np.abs(work).max()

    res1, work = residual(s.dt, 120)
    res2, _ = residual(s.dt / 2, 240)
    assert work > 20 * res1
    assert 3.0 < res1 / res2 < 5.0
    r, p = st.r.copy(), st.p.copy()
    k0 = 0.5 * (p @ p)
    _, k, _, _, _ = orc.mix_run(box, r, p, er, sr, s.dt, 150)
    np.testing.assert_allclose(k, k0, rtol=1e-13)


def test_time_reversal(orc, liquid):
    # (p, A) -> (-p, -A) from the final cell retraces the path back to the initial cell
    s, box, st = liquid
    er, sr = 0.5, 0.8
    r, p = st.r.copy(), st.p.copy()
    _, _, _, t1, _ = orc.mix_run(box, r, p, er, sr, s.dt, 200)
    p = -p
    _, _, _, t2, _ = orc.mix_run(box, r, p, -er, -sr, s.dt, 200, t0=-t1)
    assert abs(t2) < 1e-14
    dr = r - st.r
    dr -= s.box * np.rint(dr / s.box)
    assert np.abs(dr).max() < 1e-8
    assert np.abs(-p - st.p).max() < 1e-8


def test_flux_signs_under_the_mappings(orc, liquid):
    s, box, st = liquid
    n = s.n
    n1, pxy = [], []
    for m in range(4):
        rm, pm = orc.map_mix(box, m, st.r, st.p)
        n1.append(orc.observables(box, rm, pm)[0])
        pxy.append(orc.vpxy(box, rm, pm))
        if m == 1:   # x-reflection only
            np.testing.assert_array_equal(pm[:n], -st.p[:n])
            np.testing.assert_array_equal(rm[n:], st.r[n:])
    np.testing.assert_allclose(np.array(n1) / n1[0], [1.0, 1.0, -1.0, -1.0], rtol=1e-12)
    np.testing.assert_allclose(np.array(pxy) / pxy[0], [1.0, -1.0, 1.0, -1.0], rtol=1e-12)


def test_ttcf_agrees_with_the_direct_average_at_a_strong_field(orc):
    s = I.System(3)
    r, p = I.initial_state(s, 9)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    q = orc.nh_q(s.nf, s.temperature, TAU)
    ns, nst, er, sr = 24, 200, 0.3, 0.5
    sr_, sp_ = orc.mother_sample(box, st, 1000, ns, 100, s.temperature, s.dt, q, s.nf)
    state_of = np.repeat(np.arange(ns), 4)
    map_of = np.tile(np.arange(4), ns)
    x, _ = orc.run_daughters_mix(box, sr_, sp_, state_of, map_of, np.full(4 * ns, er),
                                 np.full(4 * ns, sr), s.dt, nst, nthreads=8)
    rn = np.full(4 * ns, np.hypot(er, sr))
    resp = orc.ttcf_response(x / s.volume, x[:, 0], rn, s.temperature, s.dt)
    assert abs(resp.ttcf[0]) < 1e-12
    for k in (50, 100, 200):
        se = np.hypot(resp.ttcf_se[k], resp.dav_se[k])
        assert resp.dav[k] < -4 * resp.dav_se[k]     # the flux opposes the flow: dissipation
        assert abs(resp.ttcf[k] - resp.dav[k]) < 3 * se
    wrong = orc.ttcf_response(x / s.volume, -x[:, 0], rn, s.temperature, s.dt)
    for k in (50, 100):
        assert abs(wrong.ttcf[k] - resp.dav[k]) > 4 * np.hypot(wrong.ttcf_se[k], resp.dav_se[k])


def test_recorded_components_make_up_the_flux(orc, liquid):
    # V (P_xx - P_yy) and V P_xy of the batch driver: the first equals the observables
    # routine at the start, and (erate N1 + srate P_xy) / |rate| is the recorded flux
    s, box, st = liquid
    sr_, sp_ = st.r.reshape(1, -1), st.p.reshape(1, -1)
    er, srate = 0.3, -0.5
    x, _, comp = orc.run_daughters_mix(box, sr_, sp_, np.zeros(4, np.int32), np.arange(4),
                                       np.full(4, er), np.full(4, srate), s.dt, 30, nthreads=4,
                                       components=True)
    rn = np.hypot(er, srate)
    np.testing.assert_allclose((er * comp[..., 0] + srate * comp[..., 1]) / rn, x, rtol=1e-12,
                               atol=1e-12 * np.abs(x).max())
    rm, pm = orc.map_mix(box, 2, st.r, st.p)
    assert comp[2, 0, 0] == pytest.approx(orc.observables(box, rm, pm)[0] * s.volume, rel=1e-10)
    assert comp[2, 0, 1] == pytest.approx(orc.vpxy(box, rm, pm), rel=1e-10)
