"""The list form with its neighbour lists in global scratch (systems whose lists do not fit
in LDS, e.g. N = 4000): bit for bit the LDS-list form where both fit (same lists, same order,
same arithmetic), the oracle's trajectories at N = 4000, and captured cycles that replay the
eager ones exactly."""
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


def oracle_states(orc, s, seed, n_states, between=100, n_equil=1000, n_melt=500):
    r, p = I.initial_state(s, seed)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, n_melt, 2.0, s.dt, orc.nh_q(s.nf, 2.0, TAU), s.nf)
    sr, sp, sz = orc.mother_sample(box, st, n_equil, n_states, between, s.temperature, s.dt,
                                   orc.nh_q(s.nf, s.temperature, TAU), s.nf, with_zeta=True)
    return box, sr, sp, sz


def run(T, s, sr, sp, sz, variant, thermostat, gd, nst, n_states, threads=0):
    with T.Context() as ctx:
        sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1, nh_tau=TAU,
                             thermostat=thermostat)
        mid = ctx.ttcf_init_mother(sysd, sr[0], sp[0], n_equil=0)
        ctx.ttcf_set_step_shape(variant=variant, threads=threads)
        ctx.ttcf_import_states(mid, sr, sp)
        ctx.ttcf_import_states_zeta(mid, sz)
        first = ctx.ttcf_spawn_daughters(mid, n_states, 0, gd, nst)
        ctx.ttcf_step(nst // 3)
        ctx.ttcf_step(nst)
        nd = 4 * n_states
        ser = ctx.ttcf_export_series(first, nd, nst + 1)
        fin = [ctx.ttcf_export_daughter(first + d, s.n) for d in range(nd)]
    return ser, fin


@pytest.mark.parametrize("thermostat", [0, 1])
def test_global_lists_equal_lds_lists(T, orc, thermostat):
    s = I.System(4)
    box, sr, sp, sz = oracle_states(orc, s, 61, 8)
    say(f"global vs LDS lists, thermostat={thermostat}")
    a, fa = run(T, s, sr, sp, sz, 2, thermostat, 1.0, 60, 8)
    b, fb = run(T, s, sr, sp, sz, 3, thermostat, 1.0, 60, 8)
    np.testing.assert_array_equal(a, b)
    for x, y in zip(fa, fb):
        np.testing.assert_array_equal(x[0], y[0])
        np.testing.assert_array_equal(x[1], y[1])


def test_n4000_list_form_matches_oracle(T, orc):
    """N = 4000: its lists exceed the LDS, so the list form keeps them in global scratch."""
    s = I.System(10)
    n_states, nst, gd = 4, 40, 0.5
    box, sr, sp, sz = oracle_states(orc, s, 62, n_states, n_equil=600, n_melt=300)
    say("N=4000 list form vs oracle")
    ser, fin = run(T, s, sr, sp, sz, 2, 0, gd, nst, n_states)
    state_of = np.repeat(np.arange(n_states), 4)
    map_of = np.tile(np.arange(4), n_states)
    vo, ro, po, _ = orc.run_daughters(box, sr, sp, state_of, map_of, np.full(4 * n_states, gd),
                                      s.dt, nst, nthreads=8, final_state=True)
    assert np.abs(ser - vo).max() / np.std(vo) <= 1e-4
    for d in range(4 * n_states):
        rg, pg, k = fin[d]
        assert k == nst
        dr = rg - ro[d]
        dr -= s.box * np.rint(dr / s.box)
        assert np.abs(dr).max() / s.box <= 1e-4
        assert np.abs(pg - po[d]).max() / np.sqrt(np.mean(po[d] ** 2)) <= 1e-4


def test_graph_with_global_lists_replays_eager_cycles(T):
    s = I.System(4)
    r0, p0 = I.initial_state(s, 63)
    ns, sb, nst, reps = 6, 30, 25, 2
    gam = I.log_uniform_rates(ns, 1e-3, 1e-1, 64)
    say("graph with global lists vs eager")
    eager = []
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=1),
                                   r0, p0, n_equil=100)
        ctx.ttcf_set_step_shape(variant=3)
        for _ in range(reps):
            ctx.ttcf_spawn_daughters(mid, ns, sb, gam, nst)
            ctx.ttcf_step(nst)
            ctx.ttcf_accumulate()
            eager.append(ctx.ttcf_response(nst + 1, 0.0))
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=1),
                                   r0, p0, n_equil=100)
        ctx.ttcf_set_step_shape(variant=3)
        g = ctx.ttcf_graph_create(mid, ns, sb, gam, nst, max_replays=reps)
        for k in range(reps):
            g.launch(1)
            got = ctx.ttcf_response(nst + 1, 0.0)
            for x, y in zip(got[:4], eager[k][:4]):
                assert np.array_equal(x, y)
            ctx.ttcf_export_mother(mid)  # eager work between replays
