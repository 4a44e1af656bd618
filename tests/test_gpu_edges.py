"""Edge and degenerate cases of the C ABI on the GPU: calls with nothing to do, single-step
daughters, a single mapping, the smallest and largest accepted system sizes, and the errors
for sizes and arguments the library does not take. Every error here is raised by the host
before any kernel runs."""
import sys

import numpy as np
import pytest

import ttcf_inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    from paper_2312_02990_amd import ttcf
    ttcf.lib()
    return ttcf


def small_context(T, seed=3):
    s = I.System(3)  # N = 108
    r, p = I.initial_state(s, seed)
    ctx = T.Context()
    mid = ctx.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=1), r, p,
                               n_equil=200)
    return s, ctx, mid


def test_calls_with_nothing_to_do(T):
    say("edges: nothing to do")
    s, ctx, mid = small_context(T)
    with ctx:
        ctx.ttcf_step(10)                  # no live daughters
        assert ctx.ttcf_accumulate() == 0  # nothing finished
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_response(5, 1e-2)     # no group yet
        assert e.value.code == T.TTCF_ESTATE
        first = ctx.ttcf_spawn_daughters(mid, 4, 20, 1e-2, 10)
        ctx.ttcf_step(0)                   # zero steps: nothing moves
        assert ctx.ttcf_accumulate() == 0
        ctx.ttcf_step(10)
        assert ctx.ttcf_accumulate() == 4
        ctx.ttcf_step(10)                  # all daughters folded: nothing left
        assert ctx.ttcf_accumulate() == 0
        with pytest.raises(T.TTCFError):
            ctx.ttcf_export_series(first, 1, 11)  # accumulated daughters are gone


def test_single_step_daughters_and_one_mapping(T):
    say("edges: one step, one mapping")
    s, ctx, mid = small_context(T, seed=4)
    with ctx:
        first = ctx.ttcf_spawn_daughters(mid, 6, 20, 1e-2, 1, mapping_mask=0x1)
        ctx.ttcf_step(5)                   # each stops at its own length
        ser = ctx.ttcf_export_series(first, 6, 2)
        assert ctx.ttcf_accumulate() == 6
        tm, tse, dm, dse, used = ctx.ttcf_response(2, 1e-2)
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_response(3, 1e-2)     # longer than the groups recorded
        assert e.value.code == T.TTCF_ESTATE
    assert used == 6
    b = ser / s.volume
    # one daughter per group: D(t) is its series, TTCF(0) is B(0)
    np.testing.assert_allclose(dm, b.mean(axis=0), rtol=1e-13, atol=1e-15)
    assert tm[0] == pytest.approx(b[:, 0].mean(), rel=1e-13)
    om = -(1e-2 / s.temperature) * ser[:, 0]
    g1 = b[:, 0] + 0.5 * s.dt * om * (b[:, 0] + b[:, 1])
    assert tm[1] == pytest.approx(g1.mean(), rel=1e-12, abs=1e-15)


def test_zero_length_daughters_and_bad_sizes_are_refused(T):
    say("edges: refusals")
    s, ctx, mid = small_context(T, seed=5)
    with ctx:
        for args in ((mid, 4, 20, 1e-2, 0), (mid, 0, 20, 1e-2, 10), (mid, 4, -1, 1e-2, 10),
                     (mid + 7, 4, 20, 1e-2, 10)):
            with pytest.raises(T.TTCFError) as e:
                ctx.ttcf_spawn_daughters(*args)
            assert e.value.code == T.TTCF_EINVAL
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_spawn_daughters(mid, 4, 20, 1e-2, 10, mapping_mask=0x10)
        assert e.value.code == T.TTCF_EINVAL
        with pytest.raises(T.TTCFError) as e:
            ctx.ttcf_spawn_daughters(mid, 4, 20, float("nan"), 10)
        assert e.value.code == T.TTCF_EINVAL
    # systems: fewer than 2 atoms, or more than 65535 (ids are 16-bit)
    for n in (1, 65536):
        box = (n / 0.8442) ** (1.0 / 3.0)
        r = np.random.default_rng(1).uniform(0, box, (3, n))
        with pytest.raises(T.TTCFError) as e:
            with T.Context() as ctx:
                ctx.ttcf_init_mother(T.make_system(n, box, 0.722, 0.0025, precision=1), r,
                                     np.zeros((3, n)), n_equil=0)
        assert e.value.code == T.TTCF_EINVAL


def test_largest_list_form_system_steps(T):
    """N = 4096, the most atoms one workgroup of 1024 threads holds at four per thread,
    steps in the list form with its lists in global scratch and keeps its kinetic energy."""
    say("edges: N = 4096")
    s = I.System(4, density=0.8442)
    n = 4096
    box = (n / 0.8442) ** (1.0 / 3.0)
    g = np.arange(16) * (box / 16)
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    r = np.stack([x.ravel(), y.ravel(), z.ravel()]) + 0.01
    p = I.maxwell_boltzmann(n, 0.722, 6)
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(T.make_system(n, box, 0.722, 0.0025, precision=1), r, p,
                                   n_equil=0, n_melt=300, t_melt=2.0)
        ctx.ttcf_set_step_shape(variant=2)
        first = ctx.ttcf_spawn_daughters(mid, 2, 10, 1e-2, 20)
        ctx.ttcf_step(20)
        rg, pg, k = ctx.ttcf_export_daughter(first, n)
        r0, p0 = ctx.ttcf_export_states(mid, 1)
        assert ctx.ttcf_accumulate() == 2
    assert k == 20
    assert 0.5 * np.sum(pg ** 2) == pytest.approx(0.5 * np.sum(p0[0] ** 2), rel=1e-13)
    assert np.all(np.isfinite(rg))
    del s
