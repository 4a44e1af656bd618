"""Planar-elongation daughters on the GPU (ttcf_spawn_elongational) against the oracle: the
V (P_xx - P_yy) series and final states of mapped daughters over split step calls at several
rates (FP64 forces on both sides), the responses against the estimator on the GPU's own
series and against the oracle's, shear daughters beside them unchanged bit for bit,
determinism, the refusals, and the full-size system (N = 2048) on sampled daughters."""
import sys

import numpy as np
import pytest

import ttcf_inputs as I

pytestmark = pytest.mark.gpu

TAU = 0.25


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    from paper_2312_02990_amd import ttcf
    ttcf.lib()
    return ttcf


def oracle_states(orc, s, seed, n_states, between=100, n_equil=800, n_melt=300):
    r, p = I.initial_state(s, seed)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, n_melt, 2.0, s.dt, orc.nh_q(s.nf, 2.0, TAU), s.nf)
    sr, sp = orc.mother_sample(box, st, n_equil, n_states, between, s.temperature, s.dt,
                               orc.nh_q(s.nf, s.temperature, TAU), s.nf)
    return box, sr, sp


def run(T, s, sr, sp, rates, nst, n_states, splits=(3,), shear=None):
    """PEF daughters of every state under all four mappings (and, when shear is a rate, shear
    daughters of the same states in the same step calls). Returns the PEF series, final
    states and, with shear, the shear series."""
    with T.Context() as ctx:
        sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1)
        mid = ctx.ttcf_init_mother(sysd, sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        first = ctx.ttcf_spawn_elongational(mid, n_states, 0, rates, nst)
        sfirst = ctx.ttcf_spawn_daughters(mid, n_states, 0, shear, nst) if shear else None
        for q in splits:
            ctx.ttcf_step(nst // q)
        ctx.ttcf_step(nst)
        nd = 4 * n_states
        ser = ctx.ttcf_export_series(first, nd, nst + 1)
        fin = [ctx.ttcf_export_daughter(first + d, s.n) for d in range(nd)]
        sser = ctx.ttcf_export_series(sfirst, nd, nst + 1) if shear else None
    return ser, fin, sser


def check_final(s, fin, ro, po, rate_of, nst, tol):
    for d in range(len(fin)):
        rg, pg, k = fin[d]
        assert k == nst
        e = rate_of[d] * nst * s.dt
        lb = np.repeat([s.box * np.exp(e), s.box * np.exp(-e), s.box], s.n)
        dr = rg - ro[d]
        dr -= lb * np.rint(dr / lb)
        assert np.abs(dr).max() / s.box <= tol
        assert np.abs(pg - po[d]).max() / np.sqrt(np.mean(po[d] ** 2)) <= tol


@pytest.mark.parametrize("cells", [3, 5])
def test_trajectories_match_oracle(T, orc, cells):
    s = I.System(cells)  # N = 108, 500
    n_states, nst = 4, 60
    rates = np.array([1e-3, 1.0, -0.5, 0.2])
    box, sr, sp = oracle_states(orc, s, 70 + cells, n_states)
    say(f"PEF vs oracle, N={s.n}")
    ser, fin, _ = run(T, s, sr, sp, rates, nst, n_states)
    state_of = np.repeat(np.arange(n_states), 4)
    map_of = np.tile(np.arange(4), n_states)
    rate_of = rates[state_of]
    vo, ro, po, _ = orc.run_daughters_pef(box, sr, sp, state_of, map_of, rate_of, s.dt, nst,
                                          nthreads=8, final_state=True)
    # the start values are the mapped states' own: P_xx - P_yy signs (+, +, -, -)
    np.testing.assert_allclose(ser[:, 0], vo[:, 0], rtol=1e-12, atol=1e-12 * np.abs(vo).max())
    assert np.abs(ser - vo).max() / np.std(vo) <= 1e-9
    check_final(s, fin, ro, po, rate_of, nst, 1e-9)


def test_responses_match_the_estimator_and_the_oracle(T, orc):
    s = I.System(3)
    n_states, nst, rate = 12, 80, 0.5
    box, sr, sp = oracle_states(orc, s, 81, n_states)
    say("PEF responses")
    with T.Context() as ctx:
        sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1)
        mid = ctx.ttcf_init_mother(sysd, sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        first = ctx.ttcf_spawn_elongational(mid, n_states, 0, rate, nst)
        ctx.ttcf_step(nst)
        ser = ctx.ttcf_export_series(first, 4 * n_states, nst + 1)
        assert ctx.ttcf_accumulate() == n_states   # one group per start state
        tm, tse, dm, dse, used = ctx.ttcf_response(nst + 1, rate, observable=T.TTCF_OBS_PEF_N1)
        mm, mse, mused = ctx.ttcf_response_modified(nst + 1, rate, observable=T.TTCF_OBS_PEF_N1)
        with pytest.raises(T.TTCFError) as e:   # no shear group was accumulated
            ctx.ttcf_response(nst + 1, rate)
        assert e.value.code == T.TTCF_ESTATE
    assert used == n_states and mused == n_states
    rates = np.full(4 * n_states, rate)
    # the oracle's own daughters through the oracle's estimators (the series agree to 1e-9 of
    # their spread, FP64 forces on both sides)
    state_of = np.repeat(np.arange(n_states), 4)
    map_of = np.tile(np.arange(4), n_states)
    vo, _ = orc.run_daughters_pef(box, sr, sp, state_of, map_of, rates, s.dt, nst, nthreads=8)
    assert np.abs(ser - vo).max() <= 1e-9 * np.std(vo)
    ref = orc.ttcf_response(vo / s.volume, vo[:, 0], rates, s.temperature, s.dt)
    for got, want, per in ((tm, ref.ttcf, ref.g), (tse, ref.ttcf_se, ref.g), (dm, ref.dav, ref.d),
                           (dse, ref.dav_se, ref.d)):
        assert np.abs(got - want).max() <= 1e-7 * np.abs(per).max()
    om, ose = orc.ttcf_response_modified(vo / s.volume, vo[:, 0], rates, s.temperature, s.dt)
    assert np.abs(mm - om).max() <= 1e-7 * np.abs(ref.g).max()
    assert np.abs(mse - ose).max() <= 1e-7 * np.abs(ref.g).max()
    assert tm[0] == pytest.approx(0.0, abs=1e-12 * np.abs(ser[:, 0]).max() / s.volume)


def test_shear_daughters_beside_elongation_are_unchanged(T, orc):
    s = I.System(3)
    n_states, nst = 4, 40
    box, sr, sp = oracle_states(orc, s, 82, n_states)
    say("PEF beside shear")
    a, fa, sa = run(T, s, sr, sp, 0.3, nst, n_states, shear=1e-2)
    b, fb, _ = run(T, s, sr, sp, 0.3, nst, n_states)
    np.testing.assert_array_equal(a, b)        # deterministic, and independent of the shear
    with T.Context() as ctx:                    # the shear daughters alone
        sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1)
        mid = ctx.ttcf_init_mother(sysd, sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        first = ctx.ttcf_spawn_daughters(mid, n_states, 0, 1e-2, nst)
        ctx.ttcf_step(nst // 3)
        ctx.ttcf_step(nst)
        alone = ctx.ttcf_export_series(first, 4 * n_states, nst + 1)
    np.testing.assert_array_equal(sa, alone)


def test_nose_hoover_daughters_match_oracle(T, orc):
    """Nose-Hoover planar-elongation daughters: zeta from each start state, reversed by the
    mappings that reverse the momenta; series and final states against the oracle."""
    s = I.System(3)
    n_states, nst = 4, 60
    rates = np.array([1e-3, 1.0, -0.5, 0.2])
    r, p = I.initial_state(s, 87)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, 300, 2.0, s.dt, orc.nh_q(s.nf, 2.0, TAU), s.nf)
    q = orc.nh_q(s.nf, s.temperature, TAU)
    sr, sp, sz = orc.mother_sample(box, st, 800, n_states, 100, s.temperature, s.dt, q, s.nf,
                                   with_zeta=True)
    say("PEF Nose-Hoover vs oracle")
    with T.Context() as ctx:
        sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1, nh_tau=TAU,
                             thermostat=T.TTCF_DAUGHTER_NH)
        mid = ctx.ttcf_init_mother(sysd, sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        ctx.ttcf_import_states_zeta(mid, sz)
        first = ctx.ttcf_spawn_elongational(mid, n_states, 0, rates, nst)
        ctx.ttcf_step(nst // 3)
        ctx.ttcf_step(nst)
        nd = 4 * n_states
        ser = ctx.ttcf_export_series(first, nd, nst + 1)
        fin = [ctx.ttcf_export_daughter(first + d, s.n) for d in range(nd)]
    state_of = np.repeat(np.arange(n_states), 4)
    map_of = np.tile(np.arange(4), n_states)
    rate_of = rates[state_of]
    vo, ro, po, _ = orc.run_daughters_pef(box, sr, sp, state_of, map_of, rate_of, s.dt, nst,
                                          nthreads=8, final_state=True, states_zeta=sz,
                                          temperature=s.temperature, q=q, nf=s.nf)
    assert np.abs(ser - vo).max() / np.std(vo) <= 1e-9
    check_final(s, fin, ro, po, rate_of, nst, 1e-9)
    # the thermostat acts: the isokinetic daughters of the same states differ
    vi, _ = orc.run_daughters_pef(box, sr, sp, state_of, map_of, rate_of, s.dt, nst, nthreads=8)
    assert np.abs(vi - vo).max() / np.std(vo) > 1e-6


def test_refusals(T, orc):
    s = I.System(3)
    box, sr, sp = oracle_states(orc, s, 83, 2, n_equil=200)
    say("PEF refusals")
    with T.Context() as ctx:
        sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1)
        mid = ctx.ttcf_init_mother(sysd, sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        # 5.04 e^{-1 x 200 x 0.0025} = 3.06 < 3 r_c
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_spawn_elongational(mid, 2, 0, 1.0, 200)
        assert e.value.code == T.TTCF_EINVAL
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_spawn_elongational(mid, 2, 0, -1.0, 200)
        assert e.value.code == T.TTCF_EINVAL
        ctx.ttcf_record_observables(True)
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_spawn_elongational(mid, 2, 0, 0.1, 20)
        assert e.value.code == T.TTCF_EINVAL
        ctx.ttcf_record_observables(False)
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_response(5, 0.1, observable=T.TTCF_OBS_PEF_N1)
        assert e.value.code == T.TTCF_ESTATE
    s9 = I.System(9)  # N = 2916
    r9, p9 = I.initial_state(s9, 1)
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(T.make_system(s9.n, s9.box, s9.temperature, s9.dt,
                                                 precision=1), r9, p9, n_equil=0)
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_spawn_elongational(mid, 1, 10, 0.1, 20)
        assert e.value.code == T.TTCF_EINVAL


def test_full_size_sampled(T, orc):
    """N = 2048 (the benchmark's system): two start states x four mappings over 100 steps
    at rates 1 and 1e-4 against the oracle."""
    s = I.System(8)
    n_states, nst = 2, 100
    rates = np.array([1.0, 1e-4])
    box, sr, sp = oracle_states(orc, s, 84, n_states, n_equil=300, n_melt=200)
    say("PEF full size N=2048")
    ser, fin, _ = run(T, s, sr, sp, rates, nst, n_states)
    state_of = np.repeat(np.arange(n_states), 4)
    map_of = np.tile(np.arange(4), n_states)
    rate_of = rates[state_of]
    vo, ro, po, _ = orc.run_daughters_pef(box, sr, sp, state_of, map_of, rate_of, s.dt, nst,
                                          nthreads=8, final_state=True)
    assert np.abs(ser - vo).max() / np.std(vo) <= 1e-8
    check_final(s, fin, ro, po, rate_of, nst, 1e-8)


def test_uneven_systems_in_one_step_call(T, orc):
    """N = 108 and N = 500 daughters in one launch (sized for the larger system): each
    matches the oracle as when run alone."""
    nst, n_states = 40, 2
    cases = []
    for cells, seed, rate in ((3, 85, 0.7), (5, 86, -0.4)):
        s = I.System(cells)
        box, sr, sp = oracle_states(orc, s, seed, n_states, n_equil=300)
        cases.append((s, box, sr, sp, rate))
    say("PEF uneven systems in one step call")
    firsts = []
    with T.Context() as ctx:
        for s, box, sr, sp, rate in cases:
            mid = ctx.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt,
                                                     precision=1), sr[0], sp[0], n_equil=0)
            ctx.ttcf_import_states(mid, sr, sp)
            firsts.append(ctx.ttcf_spawn_elongational(mid, n_states, 0, rate, nst))
        ctx.ttcf_step(nst)
        sers = [ctx.ttcf_export_series(f, 4 * n_states, nst + 1) for f in firsts]
    state_of = np.repeat(np.arange(n_states), 4)
    map_of = np.tile(np.arange(4), n_states)
    for (s, box, sr, sp, rate), ser in zip(cases, sers):
        vo, _ = orc.run_daughters_pef(box, sr, sp, state_of, map_of, np.full(4 * n_states, rate),
                                      s.dt, nst, nthreads=8)
        assert np.abs(ser - vo).max() / np.std(vo) <= 1e-9
