"""GPU-vs-oracle parity of the extra bulk observables (P_xx - P_yy, P_yy - P_zz, the energy
per atom and the y-slab momentum profile), recorded by the neighbour-list form beside V*P_xy.

Bars (FP32 forces, as for P_xy):
  * series over 50 steps: |GPU - oracle| <= 1e-4 of the column's spread; for the slab columns
    elementwise over the first 10 steps, and their sum (which does not depend on which slab an
    atom falls in) over all steps, since later on an atom within the trajectories' tiny
    difference of a slab boundary may be counted in the neighbouring slab;
  * the accumulated responses: equal to the estimator applied to the GPU's own exported series
    to 1e-9 of its scale (accumulator arithmetic), and within 2 combined standard errors of the
    oracle's estimate on its own daughters;
  * recording the observables leaves the P_xy series bit for bit unchanged.
"""
import sys

import numpy as np
import pytest

import ttcf_inputs as I

pytestmark = pytest.mark.gpu

TAU = 0.25
N_STATES = 8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    from paper_2312_02990_amd import ttcf
    ttcf.lib()
    return ttcf


@pytest.fixture(scope="module")
def states(orc):
    """WCA N=256 at rho=0.8442, T=0.722: 8 start states every 100 steps, with zeta."""
    s = I.System(4)
    r, p = I.initial_state(s, 17)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, 1000, 2.0, s.dt, orc.nh_q(s.nf, 2.0, TAU), s.nf)
    sr, sp, sz = orc.mother_sample(box, st, 2000, N_STATES, 100, s.temperature, s.dt,
                                   orc.nh_q(s.nf, s.temperature, TAU), s.nf, with_zeta=True)
    return s, box, sr, sp, sz


def run_gpu(T, s, sr, sp, sz, thermostat, gd, nst, record=True, accumulate=False):
    sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1, nh_tau=TAU,
                         thermostat=thermostat)
    nd = 4 * N_STATES
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(sysd, sr[0], sp[0], n_equil=0)
        ctx.ttcf_set_step_shape(variant=2)
        ctx.ttcf_import_states(mid, sr, sp)
        ctx.ttcf_import_states_zeta(mid, sz)
        ctx.ttcf_record_observables(record)
        first = ctx.ttcf_spawn_daughters(mid, N_STATES, 0, gd, nst)
        ctx.ttcf_step(nst)
        ser = ctx.ttcf_export_series(first, nd, nst + 1)
        obs = ctx.ttcf_export_observables(first, nd, nst + 1) if record else None
        resp = None
        if accumulate:
            assert ctx.ttcf_accumulate() == N_STATES
            resp = {o: ctx.ttcf_response(nst + 1, gd, observable=o)
                    for o in (T.TTCF_OBS_N1, T.TTCF_OBS_N2, T.TTCF_OBS_ENERGY,
                              T.TTCF_OBS_SLAB_PX)}
            resp["modified_n1"] = ctx.ttcf_response_modified(nst + 1, gd, T.TTCF_OBS_N1)
            resp["modified_slab"] = ctx.ttcf_response_modified(nst + 1, gd, T.TTCF_OBS_SLAB_PX)
    return ser, obs, resp


def run_oracle(orc, s, box, sr, sp, sz, thermostat, gd, nst):
    nd = 4 * N_STATES
    state_of = np.repeat(np.arange(N_STATES), 4)
    map_of = np.tile(np.arange(4), N_STATES)
    q = orc.nh_q(s.nf, s.temperature, TAU)
    return orc.run_daughters_obs(box, sr, sp, state_of, map_of, np.full(nd, gd), s.dt, nst,
                                 states_zeta=sz if thermostat else None,
                                 temperature=s.temperature, q=q, nf=s.nf, nthreads=8)


@pytest.mark.parametrize("thermostat", [0, 1])
@pytest.mark.parametrize("gd", [1e-3, 1.0])
def test_extra_observable_series_match_oracle(T, orc, states, thermostat, gd):
    s, box, sr, sp, sz = states
    nst = 50
    say(f"extra observables, thermostat={thermostat} gamma={gd}")
    ser, obs, _ = run_gpu(T, s, sr, sp, sz, thermostat, gd, nst)
    vo, oo = run_oracle(orc, s, box, sr, sp, sz, thermostat, gd, nst)
    assert np.abs(ser - vo).max() / np.std(vo) <= 1e-4
    assert obs.shape == oo.shape == (4 * N_STATES, nst + 1, T.OBS_COLS)
    for c in range(3):
        scale = np.std(oo[:, :, c])
        assert scale > 0
        assert np.abs(obs[:, :, c] - oo[:, :, c]).max() <= 1e-4 * scale, c
    slabs_g, slabs_o = obs[:, :, 3:], oo[:, :, 3:]
    scale = np.std(slabs_o)
    assert np.abs(slabs_g[:, :11] - slabs_o[:, :11]).max() <= 1e-4 * scale
    assert np.abs(slabs_g.sum(axis=2) - slabs_o.sum(axis=2)).max() <= 1e-4 * scale
    # at t = 0 the positions are the oracle's own: every slab agrees to FP64 rounding
    np.testing.assert_allclose(slabs_g[:, 0], slabs_o[:, 0], rtol=0, atol=1e-12 * scale)


def test_recording_leaves_pxy_unchanged(T, states):
    s, box, sr, sp, sz = states
    say("P_xy with and without the extra observables")
    a, _, _ = run_gpu(T, s, sr, sp, sz, 0, 1e-2, 40, record=True)
    b, _, _ = run_gpu(T, s, sr, sp, sz, 0, 1e-2, 40, record=False)
    np.testing.assert_array_equal(a, b)


def numpy_ttcf(b, vpxy0, gd, temperature, dt, volume):
    """Eq. (TTCF) per start state (four mapped daughters each), mean over states."""
    om = -(gd / temperature) * vpxy0
    ob = om[:, None] * b
    integ = np.zeros_like(ob)
    integ[:, 1:] = np.cumsum(0.5 * dt * (ob[:, :-1] + ob[:, 1:]), axis=1)
    g = (b[:, :1] + integ).reshape(-1, 4, b.shape[1]).mean(axis=1)
    d = b.reshape(-1, 4, b.shape[1]).mean(axis=1)
    return g.mean(axis=0), d.mean(axis=0)


def test_extra_observable_responses(T, orc, states):
    s, box, sr, sp, sz = states
    nst, gd = 100, 1e-3
    say("extra observable responses")
    ser, obs, resp = run_gpu(T, s, sr, sp, sz, 0, gd, nst, accumulate=True)
    vo, oo = run_oracle(orc, s, box, sr, sp, sz, 0, gd, nst)
    cols = {T.TTCF_OBS_N1: [0], T.TTCF_OBS_N2: [1], T.TTCF_OBS_ENERGY: [2],
            T.TTCF_OBS_SLAB_PX: list(range(3, T.OBS_COLS))}
    for o, cc in cols.items():
        tm, tse, dm, dse, used = resp[o]
        assert used == N_STATES
        tm, tse, dm, dse = [np.asarray(x).reshape(nst + 1, len(cc)) for x in (tm, tse, dm, dse)]
        for q, c in enumerate(cc):
            # accumulator arithmetic: the estimator on the GPU's own series
            gm, gdv = numpy_ttcf(obs[:, :, c], ser[:, 0], gd, s.temperature, s.dt, s.volume)
            sc = np.abs(obs[:, :, c]).max()
            assert np.abs(tm[:, q] - gm).max() <= 1e-9 * sc
            assert np.abs(dm[:, q] - gdv).max() <= 1e-9 * sc
            # against the oracle's own daughters: within 2 combined standard errors
            ref = orc.ttcf_response(oo[:, :, c], vo[:, 0], np.full(4 * N_STATES, gd),
                                    s.temperature, s.dt)
            comb = np.hypot(tse[:, q], ref.ttcf_se)
            assert np.all(np.abs(tm[1:, q] - ref.ttcf[1:]) <= 2.0 * comb[1:] + 1e-12 * sc), (o, q)
            assert np.all(np.abs(dm[:, q] - ref.dav) <=
                          2.0 * np.hypot(dse[:, q], ref.dav_se) + 1e-12 * sc), (o, q)
    # Eq. (corr_modified) for B = N1 and the slab profile: <Omega(0)> from P_xy(0), against
    # the definition on the GPU's own series and the oracle's on its own daughters
    for key, cc in (("modified_n1", [0]), ("modified_slab", list(range(3, T.OBS_COLS)))):
        mm, mse, used = resp[key]
        assert used == N_STATES
        mm = np.asarray(mm).reshape(nst + 1, len(cc))
        mse = np.asarray(mse).reshape(nst + 1, len(cc))
        for q, c in enumerate(cc):
            sc = np.abs(obs[:, :, c]).max()
            mg, sg = numpy_modified(obs[:, :, c], ser[:, 0], gd, s.temperature, s.dt)
            assert np.abs(mm[:, q] - mg).max() <= 1e-9 * sc
            np.testing.assert_allclose(mse[1:, q], sg[1:], rtol=1e-6, atol=1e-12 * sc)
            om, ose = orc.ttcf_response_modified(oo[:, :, c], vo[:, 0],
                                                 np.full(4 * N_STATES, gd), s.temperature, s.dt)
            assert np.all(np.abs(mm[1:, q] - om[1:]) <= 2.0 * np.hypot(mse[1:, q], ose[1:]) +
                          1e-12 * sc), (key, q)


def numpy_modified(b, vpxy0, gd, temperature, dt):
    """Eq. (corr_modified) over all daughters, jackknife over start states (4 daughters each)."""
    om = -(gd / temperature) * vpxy0
    ns = b.shape[0] // 4

    def est(keep):
        bb, oo = b[keep], om[keep]
        f = (oo[:, None] * bb).mean(axis=0) - oo.mean() * bb.mean(axis=0)
        return bb[:, 0].mean() + np.concatenate([[0.0], np.cumsum(0.5 * dt * (f[:-1] + f[1:]))])

    idx = np.arange(b.shape[0])
    full = est(idx)
    jack = np.array([est(idx[idx // 4 != n]) for n in range(ns)])
    se = np.sqrt((ns - 1) / ns * ((jack - jack.mean(axis=0)) ** 2).sum(axis=0))
    return full, se


def test_extra_observables_are_refused_where_not_recorded(T, states):
    s, box, sr, sp, sz = states
    say("extra observables: refusals")
    with T.Context() as ctx:
        # FP64 forces run in the cell form, which records P_xy only
        mid = ctx.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=0),
                                   sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        ctx.ttcf_record_observables(True)
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_spawn_daughters(mid, N_STATES, 0, 1e-2, 10)
        assert e.value.code == T.TTCF_EINVAL
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=1),
                                   sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        # groups without the observables: P_xy works, the others are refused
        ctx.ttcf_spawn_daughters(mid, N_STATES, 0, 1e-2, 10)
        ctx.ttcf_step(10)
        ctx.ttcf_accumulate()
        ctx.ttcf_response(11, 1e-2)
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_response(11, 1e-2, observable=T.TTCF_OBS_N1)
        assert e.value.code == T.TTCF_ESTATE
        # a forced cell form cannot step daughters that record them
        ctx.ttcf_record_observables(True)
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_graph_create(mid, 4, 10, 1e-2, 10, 2)
        assert e.value.code == T.TTCF_ESTATE
        ctx.ttcf_spawn_daughters(mid, N_STATES, 0, 1e-2, 10)
        ctx.ttcf_set_step_shape(variant=1)
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_step(10)
        assert e.value.code == T.TTCF_EINVAL


def test_full_size_batch_records_the_oracle_observables(T, orc):
    """N=2048, 1024 start states x 4 mappings x 500 steps with the observables recorded, in
    one launch of the recording build; a sample of 4 daughters agrees with the oracle's own
    over the first 30 steps (the bars above)."""
    s = I.System(8)
    r, p = I.initial_state(s, 2)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    sr16, sp16 = orc.mother_sample(box, st, 400, 16, 50, s.temperature, s.dt,
                                   orc.nh_q(s.nf, s.temperature, TAU), s.nf)
    sr, sp = np.tile(sr16, (64, 1)), np.tile(sp16, (64, 1))
    nst, gd = 500, 1e-2
    say("observables, full size: 4096 daughters x 500 steps")
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=1),
                                   sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        ctx.ttcf_record_observables(True)
        first = ctx.ttcf_spawn_daughters(mid, 1024, 0, gd, nst)
        ctx.ttcf_step(nst)
        sample = [0, 1, 4 * 517 + 2, 4 * 517 + 3]
        obs = np.stack([ctx.ttcf_export_observables(first + d, 1, nst + 1)[0] for d in sample])
        assert ctx.ttcf_accumulate() == 1024
        tm, tse, dm, dse, used = ctx.ttcf_response(nst + 1, gd, observable=T.TTCF_OBS_ENERGY)
    assert used == 1024 and np.all(np.isfinite(tm))
    st_of = np.array([d // 4 for d in sample]) % 16
    mp_of = np.array([d % 4 for d in sample])
    _, oo = orc.run_daughters_obs(box, sr16, sp16, st_of, mp_of, np.full(len(sample), gd), s.dt,
                                  30, nthreads=4)
    for c in range(3):
        scale = np.std(oo[:, :, c])
        assert np.abs(obs[:, :31, c] - oo[:, :, c]).max() <= 1e-4 * scale, c
    scale = np.std(oo[:, :, 3:])
    assert np.abs(obs[:, :11, 3:] - oo[:, :11, 3:]).max() <= 1e-4 * scale
