"""GPU-vs-oracle parity of the colour-field daughters (charge +1 on even atoms, -1 on odd ones,
force charge * F_e along x; isokinetic or Nose-Hoover), run by the list form's colour build.

Bars (FP32 forces, as for shear): the series V J_x and the final states over 50 steps within
1e-4 of their spread; J_x(0) under the four mappings (+, -, -, +) to FP64 rounding; the
responses equal to the estimator on the GPU's own series to 1e-9 of its scale and within 2
combined standard errors of the oracle's estimate on its own daughters; shear daughters that
share a step call with colour daughters bit for bit as in a shear-only call.
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
    """WCA N=256 at rho=0.8442, T=0.722: 8 start states every 100 steps."""
    s = I.System(4)
    r, p = I.initial_state(s, 29)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, 1000, 2.0, s.dt, orc.nh_q(s.nf, 2.0, TAU), s.nf)
    sr, sp, sz = orc.mother_sample(box, st, 2000, N_STATES, 100, s.temperature, s.dt,
                                   orc.nh_q(s.nf, s.temperature, TAU), s.nf, with_zeta=True)
    return s, box, sr, sp, sz


def context(T, s, sr, sp, precision=1, thermostat=0, sz=None):
    ctx = T.Context()
    mid = ctx.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt,
                                             precision=precision, nh_tau=TAU,
                                             thermostat=thermostat),
                               sr[0], sp[0], n_equil=0)
    ctx.ttcf_import_states(mid, sr, sp)
    if sz is not None:
        ctx.ttcf_import_states_zeta(mid, sz)
    return ctx, mid


@pytest.mark.parametrize("thermostat", [0, 1])
@pytest.mark.parametrize("fe", [1e-3, 0.5])
def test_colour_daughters_match_oracle(T, orc, states, fe, thermostat):
    s, box, sr, sp, sz = states
    nst, nd = 50, 4 * N_STATES
    say(f"colour daughters {nd} x {nst} steps F_e={fe} thermostat={thermostat}")
    ctx, mid = context(T, s, sr, sp, thermostat=thermostat, sz=sz)
    with ctx:
        first = ctx.ttcf_spawn_colour(mid, N_STATES, 0, fe, nst)
        ctx.ttcf_step(nst)
        ser = ctx.ttcf_export_series(first, nd, nst + 1)
        fin = [ctx.ttcf_export_daughter(first + d, s.n) for d in range(nd)]
    state_of = np.repeat(np.arange(N_STATES), 4)
    map_of = np.tile(np.arange(4), N_STATES)
    q = orc.nh_q(s.nf, s.temperature, TAU)
    jo, ro, po, _ = orc.run_daughters_colour(box, sr, sp, state_of, map_of, np.full(nd, fe),
                                             s.dt, nst, nthreads=8, final_state=True,
                                             states_zeta=sz if thermostat else None,
                                             temperature=s.temperature, q=q, nf=s.nf)
    assert np.abs(ser - jo).max() / np.std(jo) <= 1e-4
    for d in range(nd):
        rg, pg, k = fin[d]
        assert k == nst
        dr = rg - ro[d]
        dr -= s.box * np.rint(dr / s.box)
        assert np.abs(dr).max() / s.box <= 1e-4
        assert np.abs(pg - po[d]).max() / np.sqrt(np.mean(po[d] ** 2)) <= 1e-4
        if not thermostat:
            k_start = 0.5 * np.sum(sp[d // 4] ** 2)
            assert 0.5 * np.sum(pg ** 2) == pytest.approx(k_start, rel=1e-13)
    j0 = ser[:, 0].reshape(N_STATES, 4)
    np.testing.assert_allclose(j0 / j0[:, :1], np.tile([1.0, -1.0, -1.0, 1.0], (N_STATES, 1)),
                               rtol=1e-12)
    np.testing.assert_allclose(ser[:, 0], jo[:, 0], rtol=1e-12)


def numpy_ttcf(b, omega, dt):
    ob = omega[:, None] * b
    integ = np.zeros_like(ob)
    integ[:, 1:] = np.cumsum(0.5 * dt * (ob[:, :-1] + ob[:, 1:]), axis=1)
    g = (b[:, :1] + integ).reshape(-1, 4, b.shape[1]).mean(axis=1)
    d = b.reshape(-1, 4, b.shape[1]).mean(axis=1)
    return g.mean(axis=0), d.mean(axis=0)


def test_colour_response(T, orc, states):
    s, box, sr, sp, sz = states
    nst, nd, fe = 100, 4 * N_STATES, 0.05
    say("colour response")
    ctx, mid = context(T, s, sr, sp)
    with ctx:
        first = ctx.ttcf_spawn_colour(mid, N_STATES, 0, fe, nst)
        ctx.ttcf_step(nst)
        ser = ctx.ttcf_export_series(first, nd, nst + 1)
        assert ctx.ttcf_accumulate() == N_STATES
        tm, tse, dm, dse, used = ctx.ttcf_response(nst + 1, fe, observable=T.TTCF_OBS_JX)
        tn, _, dn, _, _ = ctx.ttcf_response(nst + 1, 0.0, observable=T.TTCF_OBS_JX)
        mm, mse, _ = ctx.ttcf_response_modified(nst + 1, fe, T.TTCF_OBS_JX)
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_response(nst + 1, fe)  # no shear group here
        assert e.value.code == T.TTCF_ESTATE
    assert used == N_STATES
    b = ser / s.volume
    om = (fe / s.temperature) * ser[:, 0]  # Omega(0) = (V/T) F_e J_x(0)
    gm, gd = numpy_ttcf(b, om, s.dt)
    sc = np.abs(b).max()
    assert np.abs(tm - gm).max() <= 1e-9 * sc
    assert np.abs(dm - gd).max() <= 1e-9 * sc
    np.testing.assert_allclose(tn, tm / fe, rtol=1e-12, atol=1e-12 * sc / fe)
    np.testing.assert_allclose(dn, dm / fe, rtol=1e-12, atol=1e-12 * sc / fe)
    # J_x(0) flips exactly under mappings 1 and 2, so <Omega(0)> is zero state by state and
    # Eq. (corr_modified) equals the plain estimate
    assert np.abs(mm - tm).max() <= 1e-12 * sc
    # against the oracle's own daughters
    state_of = np.repeat(np.arange(N_STATES), 4)
    map_of = np.tile(np.arange(4), N_STATES)
    jo, _ = orc.run_daughters_colour(box, sr, sp, state_of, map_of, np.full(nd, fe), s.dt, nst,
                                     nthreads=8)
    ref = orc.ttcf_response(jo / s.volume, jo[:, 0], np.full(nd, fe), s.temperature, s.dt,
                            omega=orc.omega0_colour(jo[:, 0], fe, s.temperature))
    assert np.all(np.abs(tm - ref.ttcf)[1:] <= 2.0 * np.hypot(tse, ref.ttcf_se)[1:] + 1e-12 * sc)
    assert np.all(np.abs(dm - ref.dav) <= 2.0 * np.hypot(dse, ref.dav_se) + 1e-12 * sc)
    # the field drives a current along +x
    assert tm[-1] > 0


def test_shear_daughters_beside_colour_ones_are_unchanged(T, states):
    s, box, sr, sp, sz = states
    nst = 40
    say("shear daughters in the colour build")
    ctx, mid = context(T, s, sr, sp)
    with ctx:
        f_shear = ctx.ttcf_spawn_daughters(mid, N_STATES, 0, 1e-2, nst)
        f_col = ctx.ttcf_spawn_colour(mid, N_STATES, 0, 0.1, nst)
        ctx.ttcf_step(nst)
        mixed = ctx.ttcf_export_series(f_shear, 4 * N_STATES, nst + 1)
        col_mixed = ctx.ttcf_export_series(f_col, 4 * N_STATES, nst + 1)
    ctx, mid = context(T, s, sr, sp)
    with ctx:
        f_shear = ctx.ttcf_spawn_daughters(mid, N_STATES, 0, 1e-2, nst)
        ctx.ttcf_step(nst)
        alone = ctx.ttcf_export_series(f_shear, 4 * N_STATES, nst + 1)
    ctx, mid = context(T, s, sr, sp)
    with ctx:
        f_col = ctx.ttcf_spawn_colour(mid, N_STATES, 0, 0.1, nst)
        ctx.ttcf_step(nst)
        col_alone = ctx.ttcf_export_series(f_col, 4 * N_STATES, nst + 1)
    np.testing.assert_array_equal(mixed, alone)
    np.testing.assert_array_equal(col_mixed, col_alone)


def test_colour_daughters_are_refused_where_not_supported(T, states):
    s, box, sr, sp, sz = states
    say("colour daughters: refusals")
    ctx, mid = context(T, s, sr, sp, precision=0)
    with ctx:
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_spawn_colour(mid, N_STATES, 0, 0.1, 10)
        assert e.value.code == T.TTCF_EINVAL
    ctx, mid = context(T, s, sr, sp)
    with ctx:
        ctx.ttcf_record_observables(True)
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_spawn_colour(mid, N_STATES, 0, 0.1, 10)
        assert e.value.code == T.TTCF_EINVAL
        ctx.ttcf_record_observables(False)
        ctx.ttcf_spawn_colour(mid, N_STATES, 0, 0.1, 10)
        ctx.ttcf_set_step_shape(variant=1)
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_step(10)
        assert e.value.code == T.TTCF_EINVAL


def test_full_size_colour_batch_matches_oracle_sample(T, orc):
    """N=2048, 1024 start states x 4 mappings x 500 steps under the colour field in one
    launch; a sample of 4 daughters agrees with the oracle's own over the first 50 steps, and
    J_x(0) cancels over each state's mappings."""
    s = I.System(8)
    r, p = I.initial_state(s, 2)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    sr16, sp16 = orc.mother_sample(box, st, 400, 16, 50, s.temperature, s.dt,
                                   orc.nh_q(s.nf, s.temperature, TAU), s.nf)
    sr, sp = np.tile(sr16, (64, 1)), np.tile(sp16, (64, 1))
    nst, fe = 500, 1e-2
    say("colour, full size: 4096 daughters x 500 steps")
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=1),
                                   sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        first = ctx.ttcf_spawn_colour(mid, 1024, 0, fe, nst)
        ctx.ttcf_step(nst)
        sample = [0, 1, 4 * 517 + 2, 4 * 517 + 3]
        ser = np.stack([ctx.ttcf_export_series(first + d, 1, nst + 1)[0] for d in sample])
        j0 = ctx.ttcf_export_series(first, 4096, 1)[:, 0]
        assert ctx.ttcf_accumulate() == 1024
        tm, tse, dm, dse, used = ctx.ttcf_response(nst + 1, fe, observable=T.TTCF_OBS_JX)
    assert used == 1024 and np.all(np.isfinite(tm))
    np.testing.assert_allclose(j0.reshape(1024, 4).sum(axis=1), 0.0,
                               atol=1e-12 * np.abs(j0).max())
    st_of = np.array([d // 4 for d in sample]) % 16
    mp_of = np.array([d % 4 for d in sample])
    jo, _ = orc.run_daughters_colour(box, sr16, sp16, st_of, mp_of, np.full(len(sample), fe),
                                     s.dt, 50, nthreads=4)
    assert np.abs(ser[:, :51] - jo).max() / np.std(jo) <= 1e-4
