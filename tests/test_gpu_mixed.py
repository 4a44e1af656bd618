"""Mixed-flow daughters on the GPU (ttcf_spawn_mixed: shear and planar elongation together in
the triclinic cell the flow carries) against the oracle: the flux series V J and final states
of mapped daughters over split step calls at several rate pairs, both thermostats; the
responses against the estimator on the GPU's own series and against the oracle's; the
refusals; and the full-size system (N = 2048) on sampled daughters."""
import sys

import numpy as np
import pytest

import ttcf_inputs as I

pytestmark = pytest.mark.gpu

TAU = 0.25
PAIRS = np.array([[0.0, 1.0], [0.5, 0.0], [0.3, -0.5], [-1e-3, 2e-3]])


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    from paper_2312_02990_amd import ttcf
    ttcf.lib()
    return ttcf


def oracle_states(orc, s, seed, n_states, n_equil=800, with_zeta=False):
    r, p = I.initial_state(s, seed)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, 300, 2.0, s.dt, orc.nh_q(s.nf, 2.0, TAU), s.nf)
    out = orc.mother_sample(box, st, n_equil, n_states, 100, s.temperature, s.dt,
                            orc.nh_q(s.nf, s.temperature, TAU), s.nf, with_zeta=with_zeta)
    return (box,) + tuple(out)


def run(T, s, sr, sp, er, srate, nst, n_states, sz=None):
    with T.Context() as ctx:
        kw = {"nh_tau": TAU, "thermostat": T.TTCF_DAUGHTER_NH} if sz is not None else {}
        sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1, **kw)
        mid = ctx.ttcf_init_mother(sysd, sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        if sz is not None:
            ctx.ttcf_import_states_zeta(mid, sz)
        first = ctx.ttcf_spawn_mixed(mid, n_states, 0, er, srate, nst)
        ctx.ttcf_step(nst // 3)
        ctx.ttcf_step(nst)
        nd = 4 * n_states
        ser = ctx.ttcf_export_series(first, nd, nst + 1)
        fin = [ctx.ttcf_export_daughter(first + d, s.n) for d in range(nd)]
    return ser, fin


def check_final(orc, box, s, fin, ro, po, er_of, sr_of, nst, tol):
    """Final states against the oracle's, positions compared modulo the lattice of the
    carried cell at the end of the run."""
    n = s.n
    for d in range(len(fin)):
        rg, pg, k = fin[d]
        assert k == nst
        h = orc.mix_cell(box, er_of[d], sr_of[d], nst * s.dt)
        dr = (rg - ro[d]).reshape(3, n)
        fy = dr[1] / h[2]
        fx = (dr[0] - h[1] * fy) / h[0]
        fz = dr[2] / s.box
        fx -= np.rint(fx)
        fy -= np.rint(fy)
        fz -= np.rint(fz)
        back = np.stack([h[0] * fx + h[1] * fy, h[2] * fy, s.box * fz])
        assert np.abs(back).max() / s.box <= tol
        assert np.abs(pg - po[d]).max() / np.sqrt(np.mean(po[d] ** 2)) <= tol


@pytest.mark.parametrize("cells", [3, 5])
def test_trajectories_match_oracle(T, orc, cells):
    s = I.System(cells)  # N = 108, 500
    n_states, nst = 4, 60
    box, sr, sp = oracle_states(orc, s, 90 + cells, n_states)
    say(f"mixed flow vs oracle, N={s.n}")
    ser, fin = run(T, s, sr, sp, PAIRS[:, 0], PAIRS[:, 1], nst, n_states)
    state_of = np.repeat(np.arange(n_states), 4)
    map_of = np.tile(np.arange(4), n_states)
    vo, ro, po, _ = orc.run_daughters_mix(box, sr, sp, state_of, map_of, PAIRS[state_of, 0],
                                          PAIRS[state_of, 1], s.dt, nst, nthreads=8,
                                          final_state=True)
    np.testing.assert_allclose(ser[:, 0], vo[:, 0], rtol=1e-12, atol=1e-12 * np.abs(vo).max())
    assert np.abs(ser - vo).max() / np.std(vo) <= 1e-9
    check_final(orc, box, s, fin, ro, po, PAIRS[state_of, 0], PAIRS[state_of, 1], nst, 1e-9)


def test_nose_hoover_daughters_match_oracle(T, orc):
    s = I.System(3)
    n_states, nst = 4, 60
    box, sr, sp, sz = oracle_states(orc, s, 95, n_states, with_zeta=True)
    say("mixed flow Nose-Hoover vs oracle")
    ser, fin = run(T, s, sr, sp, PAIRS[:, 0], PAIRS[:, 1], nst, n_states, sz=sz)
    state_of = np.repeat(np.arange(n_states), 4)
    map_of = np.tile(np.arange(4), n_states)
    q = orc.nh_q(s.nf, s.temperature, TAU)
    vo, ro, po, _ = orc.run_daughters_mix(box, sr, sp, state_of, map_of, PAIRS[state_of, 0],
                                          PAIRS[state_of, 1], s.dt, nst, nthreads=8,
                                          final_state=True, states_zeta=sz,
                                          temperature=s.temperature, q=q, nf=s.nf)
    assert np.abs(ser - vo).max() / np.std(vo) <= 1e-9
    check_final(orc, box, s, fin, ro, po, PAIRS[state_of, 0], PAIRS[state_of, 1], nst, 1e-9)


def test_responses_match_the_estimator_and_the_oracle(T, orc):
    s = I.System(3)
    n_states, nst, er, srate = 12, 80, 0.3, 0.5
    box, sr, sp = oracle_states(orc, s, 96, n_states)
    say("mixed flow responses")
    rn = float(np.sqrt(er * er + srate * srate))
    with T.Context() as ctx:
        sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1)
        mid = ctx.ttcf_init_mother(sysd, sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        first = ctx.ttcf_spawn_mixed(mid, n_states, 0, er, srate, nst)
        ctx.ttcf_step(nst)
        ser = ctx.ttcf_export_series(first, 4 * n_states, nst + 1)
        assert ctx.ttcf_accumulate() == n_states
        tm, tse, dm, dse, used = ctx.ttcf_response(nst + 1, rn, observable=T.TTCF_OBS_MIX_J)
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_response(nst + 1, rn, observable=T.TTCF_OBS_PEF_N1)
        assert e.value.code == T.TTCF_ESTATE
    assert used == n_states
    rates = np.full(4 * n_states, rn)
    # the oracle's own daughters through the oracle's estimator (series equal to 1e-9)
    state_of = np.repeat(np.arange(n_states), 4)
    map_of = np.tile(np.arange(4), n_states)
    vo, _ = orc.run_daughters_mix(box, sr, sp, state_of, map_of, np.full(4 * n_states, er),
                                  np.full(4 * n_states, srate), s.dt, nst, nthreads=8)
    assert np.abs(ser - vo).max() <= 1e-9 * np.std(vo)
    ref = orc.ttcf_response(vo / s.volume, vo[:, 0], rates, s.temperature, s.dt)
    for got, want, per in ((tm, ref.ttcf, ref.g), (tse, ref.ttcf_se, ref.g), (dm, ref.dav, ref.d),
                           (dse, ref.dav_se, ref.d)):
        assert np.abs(got - want).max() <= 1e-7 * np.abs(per).max()


def test_refusals(T, orc):
    s = I.System(3)
    box, sr, sp = oracle_states(orc, s, 97, 2, n_equil=200)
    say("mixed flow refusals")
    with T.Context() as ctx:
        sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1)
        mid = ctx.ttcf_init_mother(sysd, sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        for er, srate, nst in ((0.0, 0.0, 20), (1.0, 0.0, 200), (0.0, 3.0, 200),
                               (float("nan"), 1.0, 20)):
            with pytest.raises(T.TTCFError) as e:
                ctx.ttcf_spawn_mixed(mid, 2, 0, er, srate, nst)
            assert e.value.code == T.TTCF_EINVAL
        with pytest.raises(ValueError):
            ctx.ttcf_spawn_mixed(mid, 2, 0, [0.1, 0.2], [0.1], 20)


def test_full_size_sampled(T, orc):
    """N = 2048: two start states x four mappings over 100 steps against the oracle."""
    s = I.System(8)
    n_states, nst = 2, 100
    er = np.array([0.5, 1e-4])
    srate = np.array([1.0, 1e-4])
    box, sr, sp = oracle_states(orc, s, 98, n_states, n_equil=300)
    say("mixed flow full size N=2048")
    ser, fin = run(T, s, sr, sp, er, srate, nst, n_states)
    state_of = np.repeat(np.arange(n_states), 4)
    map_of = np.tile(np.arange(4), n_states)
    vo, ro, po, _ = orc.run_daughters_mix(box, sr, sp, state_of, map_of, er[state_of],
                                          srate[state_of], s.dt, nst, nthreads=8,
                                          final_state=True)
    assert np.abs(ser - vo).max() / np.std(vo) <= 1e-8
    check_final(orc, box, s, fin, ro, po, er[state_of], srate[state_of], nst, 1e-8)


@pytest.mark.parametrize("thermostat", ["isokinetic", "nose-hoover"])
def test_flux_components_and_their_responses(T, orc, thermostat):
    """The recorded P_xx - P_yy and P_xy of mixed-flow daughters (either daughter thermostat)
    against the oracle's; their TTCF and direct averages against the oracle's estimator on the
    oracle's own component series (Omega from the flux), and the flux response as the same
    combination of the component responses."""
    s = I.System(3)
    n_states, nst, er, srate = 8, 60, 0.3, -0.5
    nh = thermostat == "nose-hoover"
    if nh:
        box, sr, sp, sz = oracle_states(orc, s, 99, n_states, with_zeta=True)
    else:
        (box, sr, sp), sz = oracle_states(orc, s, 99, n_states), None
    rn = float(np.sqrt(er * er + srate * srate))
    say(f"mixed flow components, {thermostat}")
    with T.Context() as ctx:
        kw = {"nh_tau": TAU, "thermostat": T.TTCF_DAUGHTER_NH} if nh else {}
        sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1, **kw)
        mid = ctx.ttcf_init_mother(sysd, sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        if nh:
            ctx.ttcf_import_states_zeta(mid, sz)
        first = ctx.ttcf_spawn_mixed(mid, n_states, 0, er, srate, nst)
        ctx.ttcf_step(nst // 2)
        ctx.ttcf_step(nst)
        nd = 4 * n_states
        ser = ctx.ttcf_export_series(first, nd, nst + 1)
        obs = ctx.ttcf_export_observables(first, nd, nst + 1)
        assert ctx.ttcf_accumulate() == n_states
        rj = ctx.ttcf_response(nst + 1, rn, observable=T.TTCF_OBS_MIX_J)
        rn1 = ctx.ttcf_response(nst + 1, rn, observable=T.TTCF_OBS_MIX_N1)
        rxy = ctx.ttcf_response(nst + 1, rn, observable=T.TTCF_OBS_MIX_PXY)
    assert np.all(obs[:, :, 2:] == 0.0)
    state_of = np.repeat(np.arange(n_states), 4)
    map_of = np.tile(np.arange(4), n_states)
    extra = dict(states_zeta=sz, temperature=s.temperature, q=orc.nh_q(s.nf, s.temperature, TAU),
                 nf=s.nf) if nh else {}
    vo, _, comp = orc.run_daughters_mix(box, sr, sp, state_of, map_of, np.full(nd, er),
                                        np.full(nd, srate), s.dt, nst, nthreads=8,
                                        components=True, **extra)
    assert np.abs(ser - vo).max() / np.std(vo) <= 1e-9
    for c in (0, 1):
        got = obs[:, :, c] * s.volume
        assert np.abs(got - comp[..., c]).max() / np.std(comp[..., c]) <= 1e-9
    rates = np.full(nd, rn)
    for c, resp in ((0, rn1), (1, rxy)):
        ref = orc.ttcf_response(comp[..., c] / s.volume, vo[:, 0], rates, s.temperature, s.dt)
        for got, want, per in ((resp[0], ref.ttcf, ref.g), (resp[1], ref.ttcf_se, ref.g),
                               (resp[2], ref.dav, ref.d), (resp[3], ref.dav_se, ref.d)):
            assert np.abs(got - want).max() <= 1e-7 * np.abs(per).max()
    # TTCF is linear in B under one Omega: J = (erate N1 + srate P_xy) / |rate|
    comb = (er * rn1[0] + srate * rxy[0]) / rn
    np.testing.assert_allclose(comb, rj[0], rtol=1e-9, atol=1e-12 * np.abs(rj[0]).max())
