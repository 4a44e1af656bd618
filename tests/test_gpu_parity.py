"""GPU-vs-oracle parity through the C ABI (runs on an MI355X).

Inputs are seeded (ttcf_inputs) or produced by the FP64 oracle; nothing the GPU computes is
fed into the oracle. Bars:
  * cell lists and neighbour pairs: bit-exact on identical FP64 positions;
  * forces: max_i |dF_i| / rms_i |F_i| <= 1e-12 (FP64 form), <= 1e-5 (FP32 form);
  * trajectories over 50 steps: max |dr|/L and max |dp|/rms(p) <= 1e-4 (FP32 forms),
    <= 1e-9 (FP64 form);
  * accumulate/response kernels with FP64 forces: the oracle's own daughters through its own
    estimator agree to 1e-7 of the per-state series' scale (the trajectories agree to ~1e-9);
    with FP32 forces, TTCF and direct average within 2 combined standard errors.
"""
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


def gsys(T, s: I.System, precision):
    return T.make_system(s.n, s.box, s.temperature, s.dt, precision=precision)


def oracle_states(orc, s: I.System, seed: int, n_states: int, between: int = 100,
                  n_equil: int = 2000, n_melt: int = 1000):
    """Mother of the paper's algorithm on the oracle: melt, equilibrate, sample."""
    r, p = I.initial_state(s, seed)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    if n_melt:
        orc.nh_run(box, st, n_melt, 2.0, s.dt, orc.nh_q(s.nf, 2.0, TAU), s.nf)
    sr, sp = orc.mother_sample(box, st, n_equil, n_states, between, s.temperature, s.dt,
                               orc.nh_q(s.nf, s.temperature, TAU), s.nf)
    return box, sr, sp


@pytest.fixture(scope="module")
def cfg1(orc):
    """Config 1: WCA N=256, rho=0.8442, T=0.722; 8 start states every 100 steps."""
    s = I.System(4)
    box, sr, sp = oracle_states(orc, s, seed=1, n_states=8)
    return s, box, sr, sp


# ----------------------------------------------------------------------------------------
# cell lists, pairs, forces
# ----------------------------------------------------------------------------------------

SIZES = [(3, 0.8442), (4, 0.8442), (5, 0.8442), (8, 0.8442), (10, 0.7), (5, 0.9)]


@pytest.mark.parametrize("n_cells,rho", SIZES)
def test_cell_list_bit_exact(T, orc, n_cells, rho):
    s = I.System(n_cells, density=rho)
    say(f"cell list N={s.n} rho={rho}")
    r = I.perturbed_positions(s, 40 + n_cells, amplitude=0.2)
    dims, cell_of, order, start = T.ttcf_debug_cell_list(gsys(T, s, 1), r)
    box = orc.make_box(s.n, s.box)
    c2, o2, s2 = orc.cell_list(box, r.ravel())
    assert np.array_equal(dims, orc.cell_dims(box))
    assert np.array_equal(cell_of, c2)
    assert np.array_equal(order, o2)
    assert np.array_equal(start, s2)


@pytest.mark.parametrize("dx_frac", [0.0, 0.37, -0.61, 0.999999])
def test_pairs_bit_exact(T, orc, cfg1, dx_frac):
    s, box, sr, sp = cfg1
    for r, sysobj, b in ((sr[3], s, box),):
        dxle = dx_frac * sysobj.box
        say(f"pairs N={sysobj.n} dx={dxle}")
        for rl in (box.rc, 0.93 * box.rc):
            gi, gj = T.ttcf_debug_pairs(gsys(T, sysobj, 0), r, dxle, rl)
            oi, oj = orc.pairs(b, r, dxle, rl)
            assert np.array_equal(gi, oi) and np.array_equal(gj, oj)
    # a larger box
    s8 = I.System(8)
    r8 = I.perturbed_positions(s8, 7, amplitude=0.15)
    b8 = orc.make_box(s8.n, s8.box)
    gi, gj = T.ttcf_debug_pairs(gsys(T, s8, 0), r8, dx_frac * s8.box)
    oi, oj = orc.pairs(b8, r8.ravel(), dx_frac * s8.box)
    assert np.array_equal(gi, oi) and np.array_equal(gj, oj)


def sheared_state(orc, n_cells, k, gd=1.0, seed=9):
    """A state evolved k steps under SLLOD from a perturbed lattice, with its own LE offset.
    (A configuration taken at one offset and evaluated at another would put image atoms on
    top of boundary atoms; only states sheared into their offset are physical.)"""
    s = I.System(n_cells)
    box = orc.make_box(s.n, s.box)
    r = I.perturbed_positions(s, seed, 0.12).ravel().copy()
    p = I.maxwell_boltzmann(s.n, s.temperature, seed).ravel().copy()
    _, _, _, kk = orc.sllod_run(box, r, p, gd, s.dt, k)
    return s, box, r, orc.le_offset(box, gd, s.dt, kk)


@pytest.fixture(scope="module")
def force_cases(orc, cfg1):
    s, box, sr, sp = cfg1
    s8 = I.System(8)
    cases = [(s, box, sr[5], 0.0),
             (s8, orc.make_box(s8.n, s8.box), I.perturbed_positions(s8, 9, 0.12).ravel(), 0.0)]
    cases.append(sheared_state(orc, 4, 200))   # offset 0.5 Lx
    cases.append(sheared_state(orc, 8, 150))   # offset 0.375 Lx
    cases.append(sheared_state(orc, 4, 290, gd=-0.7, seed=4))
    return cases


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_forces(T, orc, force_cases, precision, tol):
    for sysobj, b, r, dxle in force_cases:
        say(f"forces N={sysobj.n} precision={precision} dx={dxle}")
        f, u, w = T.ttcf_debug_forces(gsys(T, sysobj, precision), r, dxle)
        fo, uo, wo, _ = orc.forces(b, r, dxle)
        rms = np.sqrt(np.mean(np.sum(fo * fo, axis=0)))
        err = np.max(np.linalg.norm(f - fo, axis=0)) / rms
        assert err <= tol, err
        fsum = np.linalg.norm(fo, axis=0).sum()
        assert abs(w - wo) <= tol * fsum * b.rc
        assert abs(u - uo) <= tol * max(abs(uo), 1.0) * (10 if precision else 1)


@pytest.mark.parametrize("dx_frac", [0.43, -0.27])
def test_forces_fp64_any_offset(T, orc, dx_frac):
    """The FP64 form matches at any offset, including unphysical overlapping ones."""
    s8 = I.System(8)
    b8 = orc.make_box(s8.n, s8.box)
    r = I.perturbed_positions(s8, 9, 0.12).ravel()
    dxle = dx_frac * s8.box
    f, u, w = T.ttcf_debug_forces(gsys(T, s8, 0), r, dxle)
    fo, uo, wo, _ = orc.forces(b8, r, dxle)
    rms = np.sqrt(np.mean(np.sum(fo * fo, axis=0)))
    assert np.max(np.linalg.norm(f - fo, axis=0)) / rms <= 1e-12


# ----------------------------------------------------------------------------------------
# trajectories
# ----------------------------------------------------------------------------------------

@pytest.mark.parametrize("precision,tol", [(0, 1e-9), (1, 1e-4)])
def test_mother_short_trajectory(T, orc, precision, tol):
    s = I.System(4)
    r0, p0 = I.initial_state(s, 3)
    r0 = I.perturbed_positions(s, 3, 0.05)
    say(f"mother 50 steps precision={precision}")
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(gsys(T, s, precision), r0, p0, n_equil=50)
        rg, pg, zg, steps = ctx.ttcf_export_mother(mid)
    assert steps == 50
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r0.ravel().copy(), p0.ravel().copy())
    orc.nh_run(box, st, 50, s.temperature, s.dt, orc.nh_q(s.nf, s.temperature, TAU), s.nf)
    dr = rg - st.r
    dr -= s.box * np.rint(dr / s.box)
    assert np.abs(dr).max() / s.box <= tol
    assert np.abs(pg - st.p).max() / np.sqrt(np.mean(st.p ** 2)) <= tol
    assert zg == pytest.approx(st.zeta, rel=100 * tol, abs=100 * tol)


def test_replicated_sampling_matches_oracle(T, orc, cfg1):
    """Copies of the mother, each kicked by a seeded zero-sum momentum change, decorrelated and
    sampled in one launch: every stored state equals the oracle's mother run from the same
    kicked start, and the mother itself does not move."""
    s, box, sr, sp = cfg1
    n_rep, per, between, decor = 3, 4, 10, 20
    rng = np.random.Generator(np.random.PCG64(77))
    kicks = 1e-3 * rng.standard_normal((n_rep, 3, s.n))
    kicks -= kicks.mean(axis=2, keepdims=True)
    kicks = kicks.reshape(n_rep, 3 * s.n)
    say("replicated mother sampling")
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(gsys(T, s, 0), sr[0], sp[0], n_equil=0)
        ctx.ttcf_sample_states_replicated(mid, n_rep, kicks, decor, per, between)
        gr, gp = ctx.ttcf_export_states(mid, n_rep * per)
        rm, pm, _, steps = ctx.ttcf_export_mother(mid)
    assert steps == 0 and np.array_equal(rm, sr[0]) and np.array_equal(pm, sp[0])
    q = orc.nh_q(s.nf, s.temperature, TAU)
    for k in range(n_rep):
        st = orc.NHState(sr[0].copy(), sp[0] + kicks[k])
        orr, orp = orc.mother_sample(box, st, decor, per, between, s.temperature, s.dt, q, s.nf)
        for j in range(per):
            dr = gr[k * per + j] - orr[j]
            dr -= s.box * np.rint(dr / s.box)
            assert np.abs(dr).max() / s.box <= 1e-9
            assert np.abs(gp[k * per + j] - orp[j]).max() / np.sqrt(np.mean(orp[j] ** 2)) <= 1e-9


@pytest.mark.parametrize("precision,variant,tol", [(0, 1, 1e-9), (1, 1, 1e-4), (1, 2, 1e-4)])
@pytest.mark.parametrize("gd", [1e-3, 1.0])
def test_daughter_trajectories(T, orc, cfg1, precision, variant, tol, gd):
    """variant 1: cell list every step; variant 2: neighbour lists (FP32 forces)."""
    s, box, sr, sp = cfg1
    nst = 50
    say(f"daughters 32 x {nst} steps precision={precision} variant={variant} gamma={gd}")
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(gsys(T, s, precision), sr[0], sp[0], n_equil=0)
        ctx.ttcf_set_step_shape(variant=variant)
        ctx.ttcf_import_states(mid, sr, sp)
        first = ctx.ttcf_spawn_daughters(mid, 8, 0, gd, nst)
        ctx.ttcf_step(nst)
        ser = ctx.ttcf_export_series(first, 32, nst + 1)
        fin = [ctx.ttcf_export_daughter(first + d, s.n) for d in range(32)]
    state_of = np.repeat(np.arange(8), 4)
    map_of = np.tile(np.arange(4), 8)
    vo, ro, po, _ = orc.run_daughters(box, sr, sp, state_of, map_of, np.full(32, gd), s.dt, nst,
                                      nthreads=8, final_state=True)
    scale = np.std(vo)
    assert np.abs(ser - vo).max() / scale <= tol
    for d in range(32):
        rg, pg, k = fin[d]
        assert k == nst
        dr = rg - ro[d]
        dr -= s.box * np.rint(dr / s.box)
        assert np.abs(dr).max() / s.box <= tol
        assert np.abs(pg - po[d]).max() / np.sqrt(np.mean(po[d] ** 2)) <= tol
        # the isokinetic constraint holds on the GPU state
        k_start = 0.5 * np.sum(sp[d // 4] ** 2)
        assert 0.5 * np.sum(pg ** 2) == pytest.approx(k_start, rel=1e-13)
    # Eq. (mappings): P_xy(0) of the four mapped daughters is (P, P, -P, -P)
    v0 = ser[:, 0].reshape(8, 4)
    np.testing.assert_allclose(v0[:, 1], v0[:, 0], rtol=1e-12)
    np.testing.assert_allclose(v0[:, 2], -v0[:, 0], rtol=1e-5 if precision else 1e-12)
    np.testing.assert_allclose(v0[:, 3], -v0[:, 0], rtol=1e-5 if precision else 1e-12)


@pytest.fixture(scope="module")
def cfg1_nh(orc):
    """Config-1 system, 8 start states every 100 steps with their thermostat variables."""
    s = I.System(4)
    r, p = I.initial_state(s, 11)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, 1000, 2.0, s.dt, orc.nh_q(s.nf, 2.0, TAU), s.nf)
    sr, sp, sz = orc.mother_sample(box, st, 2000, 8, 100, s.temperature, s.dt,
                                   orc.nh_q(s.nf, s.temperature, TAU), s.nf, with_zeta=True)
    return s, box, sr, sp, sz


@pytest.mark.parametrize("precision,variant,tol", [(0, 1, 1e-9), (1, 1, 1e-4), (1, 2, 1e-4)])
@pytest.mark.parametrize("gd", [1e-3, 1.0])
def test_nh_daughter_trajectories(T, orc, cfg1_nh, precision, variant, tol, gd):
    """Nose-Hoover daughters (Eq. system1 as printed), zeta carried from the start state and
    reversed by mappings 1 and 3, against the oracle; the run is split over two step calls."""
    s, box, sr, sp, sz = cfg1_nh
    nst = 50
    q = orc.nh_q(s.nf, s.temperature, TAU)
    say(f"NH daughters 32 x {nst} steps precision={precision} variant={variant} gamma={gd}")
    with T.Context() as ctx:
        sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=precision, nh_tau=TAU,
                             thermostat=T.TTCF_DAUGHTER_NH)
        mid = ctx.ttcf_init_mother(sysd, sr[0], sp[0], n_equil=0)
        ctx.ttcf_set_step_shape(variant=variant)
        ctx.ttcf_import_states(mid, sr, sp)
        assert np.all(ctx.ttcf_export_states_zeta(mid, 8) == 0.0)
        ctx.ttcf_import_states_zeta(mid, sz)
        assert np.array_equal(ctx.ttcf_export_states_zeta(mid, 8), sz)
        first = ctx.ttcf_spawn_daughters(mid, 8, 0, gd, nst)
        ctx.ttcf_step(20)
        ctx.ttcf_step(nst)
        ser = ctx.ttcf_export_series(first, 32, nst + 1)
        fin = [ctx.ttcf_export_daughter(first + d, s.n) for d in range(32)]
    state_of = np.repeat(np.arange(8), 4)
    map_of = np.tile(np.arange(4), 8)
    vo, ro, po, _ = orc.run_daughters_nh(box, sr, sp, sz, state_of, map_of, np.full(32, gd), s.dt,
                                         s.temperature, q, s.nf, nst, nthreads=8,
                                         final_state=True)
    scale = np.std(vo)
    assert np.abs(ser - vo).max() / scale <= tol
    for d in range(32):
        rg, pg, k = fin[d]
        assert k == nst
        dr = rg - ro[d]
        dr -= s.box * np.rint(dr / s.box)
        assert np.abs(dr).max() / s.box <= tol
        assert np.abs(pg - po[d]).max() / np.sqrt(np.mean(po[d] ** 2)) <= tol


def test_sampled_states_carry_the_mother_thermostat(T, orc, cfg1_nh):
    """Sampling records the mother's zeta at every saved state (the last one is the mother's
    current zeta), and replicated sampling records each copy's."""
    s, box, sr, sp, sz = cfg1_nh
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(gsys(T, s, 0), sr[0], sp[0], n_equil=0)
        ctx.ttcf_sample_states(mid, 3, 40)
        z = ctx.ttcf_export_states_zeta(mid, 3)
        _, _, zm, _ = ctx.ttcf_export_mother(mid)
        assert z[-1] == zm and len(set(z.tolist())) == 3
        ctx.ttcf_sample_states_replicated(mid, 2, None, 30, 2, 20)
        zr = ctx.ttcf_export_states_zeta(mid, 4)
        # copies without kicks run the same trajectory: equal zeta, copy by copy
        assert zr[0] == zr[2] and zr[1] == zr[3] and zr[0] != zr[1]
    # the oracle mother from the same state gives the same zeta sequence
    st = orc.NHState(sr[0].copy(), sp[0].copy(), 0.0)
    _, _, oz = orc.mother_sample(box, st, 0, 3, 40, s.temperature, s.dt,
                                 orc.nh_q(s.nf, s.temperature, TAU), s.nf, with_zeta=True)
    np.testing.assert_allclose(z, oz, rtol=1e-9, atol=1e-12)


def test_neighbour_lists_are_skin_invariant(T, orc, cfg1):
    """Lists are sorted by atom id and pairs beyond the cutoff add nothing, so the results
    are bit-identical for any skin (and any rebuild schedule), at strong shear too."""
    s, box, sr, sp = cfg1
    nst = 200
    out = []
    for skin, kmax in ((0.15, 20), (0.25, 24), (0.4, 32)):
        say(f"skin {skin}")
        with T.Context() as ctx:
            mid = ctx.ttcf_init_mother(gsys(T, s, 1), sr[0], sp[0], n_equil=0)
            ctx.ttcf_import_states(mid, sr[:2], sp[:2])
            ctx.ttcf_set_step_shape(variant=2, skin=skin, kmax=kmax)
            first = ctx.ttcf_spawn_daughters(mid, 2, 0, [1e-3, 2.0], nst)
            ctx.ttcf_step(nst)
            out.append(ctx.ttcf_export_series(first, 8, nst + 1))
            assert all(ctx.ttcf_daughter_health(first + d) == 0 for d in range(8))
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[1], out[2])


def test_neighbour_list_form_matches_cell_form(T, cfg1):
    """The two FP32 kernel forms agree to FP32 accuracy over 100 steps."""
    s, box, sr, sp = cfg1
    nst = 100
    out = []
    for variant in (1, 2):
        with T.Context() as ctx:
            mid = ctx.ttcf_init_mother(gsys(T, s, 1), sr[0], sp[0], n_equil=0)
            ctx.ttcf_import_states(mid, sr, sp)
            ctx.ttcf_set_step_shape(variant=variant)
            first = ctx.ttcf_spawn_daughters(mid, 8, 0, 0.5, nst)
            ctx.ttcf_step(nst)
            out.append(ctx.ttcf_export_series(first, 32, nst + 1))
    assert np.abs(out[0] - out[1]).max() / np.std(out[0]) < 1e-3


# ----------------------------------------------------------------------------------------
# accumulate and response
# ----------------------------------------------------------------------------------------

@pytest.mark.parametrize("precision", [0, 1])
def test_config1_ttcf_matches_oracle(T, orc, cfg1, precision):
    """Config 1 end to end: 8 states x 4 mappings = 32 daughters x 100 steps at 1e-3."""
    s, box, sr, sp = cfg1
    nst, gd = 100, 1e-3
    say(f"config 1 TTCF precision={precision}")
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(gsys(T, s, precision), sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        first = ctx.ttcf_spawn_daughters(mid, 8, 0, gd, nst)
        ctx.ttcf_step(40)
        ctx.ttcf_step(100)  # continues to each daughter's own length
        assert ctx.ttcf_accumulate() == 8
        tm, tse, dm, dse, used = ctx.ttcf_response(nst + 1, gd)
    assert used == 8
    # the oracle's own daughters from the same start states, through its own estimator
    state_of = np.repeat(np.arange(8), 4)
    map_of = np.tile(np.arange(4), 8)
    vo, _ = orc.run_daughters(box, sr, sp, state_of, map_of, np.full(32, gd), s.dt, nst,
                              nthreads=8)
    oref = orc.ttcf_response(vo / s.volume, vo[:, 0], np.full(32, gd), s.temperature, s.dt)
    if precision == 0:
        # FP64 forces: the trajectories agree to ~1e-9 of their spread over 100 steps, so the
        # estimates agree to that accuracy (relative to the spread of the per-state series)
        for got, ref, per in ((tm, oref.ttcf, oref.g), (dm, oref.dav, oref.d)):
            assert np.abs(got - ref).max() <= 1e-7 * np.abs(per).max()
        np.testing.assert_allclose(tse, oref.ttcf_se, rtol=1e-6, atol=1e-7 * np.abs(oref.g).max())
        np.testing.assert_allclose(dse, oref.dav_se, rtol=1e-6, atol=1e-7 * np.abs(oref.d).max())
    # both forms: within 2 combined standard errors at every time point
    comb = np.hypot(tse, oref.ttcf_se)
    assert np.all(np.abs(tm - oref.ttcf)[1:] <= 2.0 * comb[1:])
    assert np.all(np.abs(dm - oref.dav) <= 2.0 * np.hypot(dse, oref.dav_se) + 1e-15)


@pytest.mark.parametrize("mask", [0xF, 0x5, 0x1, 0x3])
def test_modified_integrand_matches_oracle(T, orc, cfg1, mask):
    """Eq. (corr_modified) from the accumulator rows against the oracle's definition and
    jackknife on its own daughters (FP64 forces). Where a state's mappings hold as many
    Omega-keeping (0, 1) as Omega-reversing (2, 3) ones, <Omega(0)> vanishes state by state
    and it equals the plain estimate; otherwise (mappings {0} or {0, 1}) the sample
    <Omega(0)> is not zero and the correction acts."""
    s, box, sr, sp = cfg1
    nst, gd = 100, 1e-2
    maps = [m for m in range(4) if mask >> m & 1]
    say(f"modified integrand, mappings {maps}")
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(gsys(T, s, 0), sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        ctx.ttcf_spawn_daughters(mid, 8, 0, gd, nst, mapping_mask=mask)
        ctx.ttcf_step(nst)
        assert ctx.ttcf_accumulate() == 8
        mm, mse, used = ctx.ttcf_response_modified(nst + 1, gd)
        tm, tse, _, _, _ = ctx.ttcf_response(nst + 1, gd)
    assert used == 8
    nm = len(maps)
    vo, _ = orc.run_daughters(box, sr, sp, np.repeat(np.arange(8), nm), np.tile(maps, 8),
                              np.full(8 * nm, gd), s.dt, nst, nthreads=8)
    om, ose = orc.ttcf_response_modified(vo / s.volume, vo[:, 0], np.full(8 * nm, gd),
                                         s.temperature, s.dt, n_maps=nm)
    scale = np.abs(vo / s.volume).max()
    assert np.abs(mm - om).max() <= 1e-7 * scale
    np.testing.assert_allclose(mse[1:], ose[1:], rtol=1e-5, atol=1e-9 * scale)
    if sum(m < 2 for m in maps) == sum(m >= 2 for m in maps):
        assert np.abs(mm - tm).max() <= 1e-12 * scale
        np.testing.assert_allclose(mse[1:], tse[1:], rtol=1e-8)
    else:
        assert np.abs(mm - tm).max() > 1e-6 * scale


def oracle_group_response(orc, s, box, sr, sp, states, gd, nst):
    """The oracle's own four mapped daughters of each listed start state, through its
    estimator."""
    states = np.asarray(states)
    state_of = np.repeat(states, 4)
    map_of = np.tile(np.arange(4), len(states))
    vo, _ = orc.run_daughters(box, sr, sp, state_of, map_of, np.full(len(state_of), gd), s.dt,
                              nst, nthreads=8)
    return orc.ttcf_response(vo / s.volume, vo[:, 0], np.full(len(state_of), gd),
                             s.temperature, s.dt)


def close_to(got, ref, per, rel=1e-7):
    """FP64 forces against the oracle: agreement to rel of the per-state series' scale."""
    assert np.abs(got - ref).max() <= rel * np.abs(per).max()


def test_response_filters_and_normalisation(T, orc, cfg1):
    s, box, sr, sp = cfg1
    nst = 30
    say("response filters")
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(gsys(T, s, 0), sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        ctx.ttcf_spawn_daughters(mid, 8, 0, 1e-2, nst)
        ctx.ttcf_spawn_daughters(mid, 8, 0, 1e-4, nst)
        ctx.ttcf_step(nst)
        assert ctx.ttcf_accumulate() == 16
        a = ctx.ttcf_response(nst + 1, 1e-2)
        b = ctx.ttcf_response(nst + 1, 1e-4)
        c = ctx.ttcf_response(nst + 1, 0.0)
        with pytest.raises(T.TTCFError):
            ctx.ttcf_response(nst + 1, 3e-3)
        with pytest.raises(T.TTCFError):
            ctx.ttcf_response(nst + 2, 1e-2)
    ra = oracle_group_response(orc, s, box, sr, sp, range(8), 1e-2, nst)
    rb = oracle_group_response(orc, s, box, sr, sp, range(8), 1e-4, nst)
    close_to(a[0], ra.ttcf, ra.g)
    close_to(b[0], rb.ttcf, rb.g)
    assert a[4] == 8 and b[4] == 8
    # per-unit-rate response over both batches: mean of the 16 normalised groups
    g = np.concatenate([ra.g / 1e-2, rb.g / 1e-4])
    close_to(c[0], g.mean(axis=0), g)
    assert c[4] == 16


@pytest.mark.parametrize("nst", [1, 63, 64, 200])
def test_accumulate_and_response_on_the_gpu_series(T, orc, cfg1, nst):
    """The accumulator (per group, a compensated prefix scan of the trapezoid terms over
    blocks of 64 time points) and the response kernels, applied to the GPU's own exported
    daughter series, against the oracle's estimator on those series: 2, 64 (one full block),
    65 (a block and one point) and 201 time points (three full blocks and a ragged tail), two
    shear rates, the per-rate filters and the per-unit-rate normalisation, to rounding
    (1e-12 of the per-state scale for the means, 1e-9 relative for the block standard
    errors)."""
    s, box, sr, sp = cfg1
    say(f"accumulate/response on the GPU's own series, {nst + 1} points")
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(gsys(T, s, 1), sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        fa = ctx.ttcf_spawn_daughters(mid, 8, 0, 1e-2, nst)
        fb = ctx.ttcf_spawn_daughters(mid, 8, 0, 0.5, nst)
        ctx.ttcf_step(nst)
        sa = ctx.ttcf_export_series(fa, 32, nst + 1)
        sb = ctx.ttcf_export_series(fb, 32, nst + 1)
        assert ctx.ttcf_accumulate() == 16
        ra = ctx.ttcf_response(nst + 1, 1e-2)
        rb = ctx.ttcf_response(nst + 1, 0.5)
        rn = ctx.ttcf_response(nst + 1, 0.0)
    refs = []
    for got, ser, gd in ((ra, sa, 1e-2), (rb, sb, 0.5)):
        ref = orc.ttcf_response(ser / s.volume, ser[:, 0], np.full(32, gd), s.temperature, s.dt)
        refs.append((ref, gd))
        assert got[4] == 8
        sc = np.abs(ref.g).max()
        assert np.abs(got[0] - ref.ttcf).max() <= 1e-12 * sc
        assert np.abs(got[2] - ref.dav).max() <= 1e-12 * np.abs(ref.d).max()
        np.testing.assert_allclose(got[1], ref.ttcf_se, rtol=1e-9, atol=1e-14 * sc)
        np.testing.assert_allclose(got[3], ref.dav_se, rtol=1e-9,
                                   atol=1e-14 * np.abs(ref.d).max())
    # per unit rate: the 16 groups, each divided by its own rate
    g = np.concatenate([ref.g / gd for ref, gd in refs])
    d = np.concatenate([ref.d / gd for ref, gd in refs])
    assert rn[4] == 16
    sq = np.sqrt(16)
    assert np.abs(rn[0] - g.mean(axis=0)).max() <= 1e-12 * np.abs(g).max()
    assert np.abs(rn[2] - d.mean(axis=0)).max() <= 1e-12 * np.abs(d).max()
    np.testing.assert_allclose(rn[1], g.std(axis=0, ddof=1) / sq, rtol=1e-9,
                               atol=1e-14 * np.abs(g).max())
    np.testing.assert_allclose(rn[3], d.std(axis=0, ddof=1) / sq, rtol=1e-9,
                               atol=1e-14 * np.abs(d).max())


def test_health_check_excludes_whole_group(T, orc, cfg1):
    s, box, sr, sp = cfg1
    nst = 20
    say("health / failure injection")
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(gsys(T, s, 0), sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        first = ctx.ttcf_spawn_daughters(mid, 8, 0, 1e-3, nst)
        ctx.ttcf_step(5)
        ctx.ttcf_debug_poison(first + 13)  # state 3, mapping 1
        ctx.ttcf_step(nst)
        assert ctx.ttcf_daughter_health(first + 13) != 0
        assert ctx.ttcf_daughter_health(first + 12) == 0
        assert ctx.ttcf_accumulate() == 7
        tm, tse, dm, dse, used = ctx.ttcf_response(nst + 1, 1e-3)
    assert used == 7
    ref = oracle_group_response(orc, s, box, sr, sp, [0, 1, 2, 4, 5, 6, 7], 1e-3, nst)
    close_to(tm, ref.ttcf, ref.g)
    close_to(dm, ref.dav, ref.d)


def test_uneven_batch_is_invariant_and_deterministic(T, orc, cfg1):
    """Daughters of two system sizes in one launch give bit-identical series to each size
    run alone, and repeated runs are bit-identical."""
    s, box, sr, sp = cfg1
    s5 = I.System(5)
    r5, p5 = I.initial_state(s5, 8)
    r5 = I.perturbed_positions(s5, 8, 0.1)
    nst = 25
    say("uneven batch invariance")

    def run(with256, with500):
        out = {}
        with T.Context() as ctx:
            if with256:
                m1 = ctx.ttcf_init_mother(gsys(T, s, 1), sr[0], sp[0], n_equil=0)
                ctx.ttcf_import_states(m1, sr[:2], sp[:2])
            if with500:
                m2 = ctx.ttcf_init_mother(
                    T.make_system(s5.n, s5.box, block_threads=512, precision=1), r5, p5,
                    n_equil=0)
                ctx.ttcf_import_states(m2, r5.reshape(1, -1), p5.reshape(1, -1))
            if with256:
                f1 = ctx.ttcf_spawn_daughters(m1, 2, 0, 0.1, nst)
            if with500:
                f2 = ctx.ttcf_spawn_daughters(m2, 1, 0, 0.1, nst)
            ctx.ttcf_step(nst)
            if with256:
                out[256] = ctx.ttcf_export_series(f1, 8, nst + 1)
            if with500:
                out[500] = ctx.ttcf_export_series(f2, 4, nst + 1)
        return out

    both = run(True, True)
    both2 = run(True, True)
    a = run(True, False)
    b = run(False, True)
    assert np.array_equal(both[256], both2[256]) and np.array_equal(both[500], both2[500])
    # the 256-atom daughters ran with 512-thread workgroups in the mixed launch and with
    # 256-thread ones alone; their per-atom work is identical, so are their results
    np.testing.assert_allclose(both[256], a[256], rtol=0, atol=0)
    np.testing.assert_allclose(both[500], b[500], rtol=0, atol=0)


def test_mixed_forms_in_one_step_call(T):
    """N = 4000 (its lists do not fit in LDS: cell form) and N = 500 (neighbour-list form)
    live together: one ttcf_step call launches both forms, and each size's series equal the
    ones it gives alone."""
    s_big = I.System(10, density=0.7)
    s_small = I.System(5)
    rb = I.perturbed_positions(s_big, 21, 0.1)
    pb = I.maxwell_boltzmann(s_big.n, s_big.temperature, 21)
    rs = I.perturbed_positions(s_small, 22, 0.1)
    ps = I.maxwell_boltzmann(s_small.n, s_small.temperature, 22)
    nst = 20
    say("mixed kernel forms")

    def run(big, small):
        out = {}
        with T.Context() as ctx:
            if big:
                mb = ctx.ttcf_init_mother(gsys(T, s_big, 1), rb, pb, n_equil=0)
                ctx.ttcf_import_states(mb, rb.reshape(1, -1), pb.reshape(1, -1))
                fb = ctx.ttcf_spawn_daughters(mb, 1, 0, 0.05, nst)
            if small:
                ms = ctx.ttcf_init_mother(gsys(T, s_small, 1), rs, ps, n_equil=0)
                ctx.ttcf_import_states(ms, rs.reshape(1, -1), ps.reshape(1, -1))
                fs = ctx.ttcf_spawn_daughters(ms, 1, 0, 0.05, nst)
            ctx.ttcf_step(nst)
            if big:
                out["big"] = ctx.ttcf_export_series(fb, 4, nst + 1)
            if small:
                out["small"] = ctx.ttcf_export_series(fs, 4, nst + 1)
        return out

    both = run(True, True)
    assert np.array_equal(both["big"], run(True, False)["big"])
    assert np.array_equal(both["small"], run(False, True)["small"])
    assert np.all(np.isfinite(both["big"])) and np.all(np.isfinite(both["small"]))


def test_autotuned_shape_is_the_one_used(T):
    """The autotuner leaves live daughters alone, caches its pick for the system, and
    ttcf_step then runs exactly that shape: series equal bit for bit to the same shape set
    explicitly or imported from the exported cache text, and to the default shape within
    FP32 rounding."""
    s = I.System(5)
    r0, p0 = I.initial_state(s, 41)
    nst = 30
    say("autotune")

    def run(setup):
        with T.Context() as ctx:
            mid = ctx.ttcf_init_mother(gsys(T, s, 1), r0, p0, n_equil=200, n_melt=200, t_melt=2.0)
            ctx.ttcf_sample_states(mid, 8, 20)
            first = ctx.ttcf_spawn_daughters(mid, 8, 0, 0.05, nst)
            info = setup(ctx, mid)
            ctx.ttcf_step(nst)
            series = ctx.ttcf_export_series(first, 32, nst + 1)
            assert ctx.ttcf_accumulate() == 8
            return series, info

    tuned, (shape, text) = run(lambda ctx, mid: (ctx.ttcf_autotune(mid, 0, 0.05, 20),
                                                 ctx.ttcf_autotune_export()))
    say("tuned shape", shape)
    # the cell form at one of its three sizes; the pair form at four atoms per thread
    assert shape["variant"] in (1, 2)
    assert shape["threads"] in ((256, 512, 1024) if shape["variant"] == 1 else
                                (64 * ((s.n + 255) // 256),))
    assert shape["candidates"] >= 3 and shape["ms_per_step"] > 0.0
    assert '"n": 500' in text
    nl = shape["variant"] == 2
    explicit, _ = run(lambda ctx, mid: ctx.ttcf_set_step_shape(
        shape["variant"], shape["threads"], shape["skin"] if nl else 0.0,
        shape["kmax"] if nl else 0))
    imported, _ = run(lambda ctx, mid: ctx.ttcf_autotune_import(text))
    default, _ = run(lambda ctx, mid: None)
    assert np.array_equal(tuned, explicit)
    assert np.array_equal(tuned, imported)
    assert np.abs(tuned - default).max() <= 1e-4 * np.abs(default).max()
    assert np.all(np.isfinite(tuned))


def test_autotune_cache_text_is_validated(T):
    s = I.System(4)
    r0, p0 = I.initial_state(s, 3)
    with T.Context() as ctx:
        ctx.ttcf_init_mother(gsys(T, s, 1), r0, p0, n_equil=0)
        assert ctx.ttcf_autotune_export().strip() == "[\n]".strip()
        with pytest.raises(T.TTCFError):
            ctx.ttcf_autotune_import('[{"arch": "x", "n": 256}]')
        with pytest.raises(T.TTCFError):
            ctx.ttcf_autotune(0)  # no stored start states yet
        good = ('[{"arch": "gfx000", "n": 256, "rho_key": 844, "rc_key": 11225, "precision": 1, '
                '"variant": 2, "threads": 256, "kmax": 20, "skin": 0.4, "ms_per_step": 1}]')
        ctx.ttcf_autotune_import(good)
        assert '"arch": "gfx000"' in ctx.ttcf_autotune_export()


def test_autocorrelation_matches_oracle(T, orc):
    """The autocorrelation used to choose T_s: a seeded AR(1) series against the oracle's
    definition, and the mother's recorded V*P_xy series through both entry points."""
    x = I.ar1_series(20000, 0.95, 9)
    s = I.System(4)
    r0, p0 = I.initial_state(s, 1)
    say("autocorrelation")
    with T.Context() as ctx:
        # melted first: an fcc start at this state point stays crystalline for a while
        mid = ctx.ttcf_init_mother(gsys(T, s, 0), r0, p0, n_equil=1000, n_melt=1000, t_melt=2.0)
        a, fb, tau = ctx.ttcf_acf(x, 300, 0.05)
        ctx.ttcf_record_mother(mid, 4000)
        ctx.ttcf_sample_states(mid, 40, 100)
        am, fbm, taum = ctx.ttcf_mother_acf(mid, 400, 0.05)
        series = ctx.ttcf_export_mother_series(mid, 4000)
        a2, fb2, tau2 = ctx.ttcf_acf(series, 400, 0.05)
        with pytest.raises(T.TTCFError):
            ctx.ttcf_acf(x[:10], 20)  # max_lag beyond the series
    oa = orc.acf(x, 300)
    ofb, otau = orc.acf_summary(oa, 0.05)
    np.testing.assert_allclose(a, oa, rtol=0, atol=1e-12)
    assert fb == ofb and tau == pytest.approx(otau, rel=1e-12)
    assert len(series) == 4000
    np.testing.assert_array_equal(am, a2)
    assert (fbm, taum) == (fb2, tau2)
    say("mother acf: first lag below 0.05", fbm, "integrated time", taum)
    assert am[0] == pytest.approx(1.0, abs=1e-15) and 0 < fbm < 400


# ----------------------------------------------------------------------------------------
# captured batch cycles: every replay equals the same cycle run through the eager calls
# ----------------------------------------------------------------------------------------
def _same_response(a, b):
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)
    assert a[4] == b[4]


@pytest.mark.parametrize("precision,thermostat", [(0, 0), (1, 0), (1, 1)])
def test_graph_replays_equal_eager_cycles(T, precision, thermostat):
    """A mother that saves 6 states 30 steps apart, per-state shear rates, 25-step daughters:
    after each replay (eager work and synchronisation in between) the response and the
    mother equal those of the same number of eager cycles, bit for bit."""
    s = I.System(4)
    r0, p0 = I.initial_state(s, 51)
    ns, sb, nst, reps = 6, 30, 25, 3
    gam = I.log_uniform_rates(ns, 1e-3, 1e-1, 52)
    say("graph vs eager, precision", precision)
    eager, eager_mother = [], None
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=precision, thermostat=thermostat), r0, p0, n_equil=100)
        for _ in range(reps):
            ctx.ttcf_spawn_daughters(mid, ns, sb, gam, nst)
            ctx.ttcf_step(nst)
            ctx.ttcf_accumulate()
            eager.append(ctx.ttcf_response(nst + 1, 0.0))
        eager_mother = ctx.ttcf_export_mother(mid)
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=precision, thermostat=thermostat), r0, p0, n_equil=100)
        g = ctx.ttcf_graph_create(mid, ns, sb, gam, nst, max_replays=reps)
        with pytest.raises(T.TTCFError):
            ctx.ttcf_response(nst + 1, 0.0)  # reserved rows are not counted before a replay
        for k in range(reps):
            g.launch(1)
            got = ctx.ttcf_response(nst + 1, 0.0)
            _same_response(got, eager[k])
            ctx.ttcf_export_mother(mid)  # eager work between replays
        assert g.replays == reps
        with pytest.raises(T.TTCFError):
            g.launch(1)
        r, p, z, steps = ctx.ttcf_export_mother(mid)
        assert np.array_equal(r, eager_mother[0]) and np.array_equal(p, eager_mother[1])
        assert z == eager_mother[2] and steps == eager_mother[3]
        # ordinary daughters accumulate beside the graph's rows
        ctx.ttcf_spawn_daughters(mid, ns, sb, gam, nst)
        ctx.ttcf_step(nst)
        assert ctx.ttcf_accumulate() == ns
        assert ctx.ttcf_response(nst + 1, 0.0)[4] == (reps + 1) * ns


@pytest.mark.parametrize("precision,thermostat", [(0, 0), (1, 0), (1, 1)])
def test_graph_of_uneven_mothers_equals_eager_cycles(T, precision, thermostat):
    """One captured cycle over two mothers of different N (256 and 500), each saving 3 states
    30 steps apart at per-state rates, 25-step daughters stepped together: after each replay
    the response over all groups and both mothers equal those of the eager cycles (each
    mother's spawn in order, one step call, one accumulation) bit for bit."""
    systems = [I.System(4), I.System(5)]
    starts = [I.initial_state(sy, 71 + k) for k, sy in enumerate(systems)]
    ns, sb, nst, reps = 3, 30, 25, 3
    gams = [I.log_uniform_rates(ns, 1e-3, 1e-1, 72 + k) for k in range(2)]
    say("uneven graph vs eager, precision", precision, "thermostat", thermostat)

    def mothers(ctx):
        return [ctx.ttcf_init_mother(T.make_system(sy.n, sy.box, sy.temperature, sy.dt,
                                                   precision=precision, thermostat=thermostat),
                                     r0, p0, n_equil=100)
                for sy, (r0, p0) in zip(systems, starts)]

    eager = []
    with T.Context() as ctx:
        mids = mothers(ctx)
        for _ in range(reps):
            for mid, g in zip(mids, gams):
                ctx.ttcf_spawn_daughters(mid, ns, sb, g, nst)
            ctx.ttcf_step(nst)
            assert ctx.ttcf_accumulate() == 2 * ns
            eager.append(ctx.ttcf_response(nst + 1, 0.0))
        eager_mothers = [ctx.ttcf_export_mother(mid) for mid in mids]
    with T.Context() as ctx:
        mids = mothers(ctx)
        gr = ctx.ttcf_graph_create_multi(
            [{"mother": mid, "states_per_replica": ns, "steps_between": sb, "gamma_dot": g}
             for mid, g in zip(mids, gams)], nst, reps)
        for k in range(reps):
            gr.launch(1)
            _same_response(ctx.ttcf_response(nst + 1, 0.0), eager[k])
            ctx.ttcf_export_mother(mids[0])  # eager work between replays
        assert gr.replays == reps
        for mid, em in zip(mids, eager_mothers):
            r, p, z, steps = ctx.ttcf_export_mother(mid)
            assert np.array_equal(r, em[0]) and np.array_equal(p, em[1])
            assert z == em[2] and steps == em[3]
        part = {"mother": mids[0], "states_per_replica": 1, "steps_between": 5, "gamma_dot": 0.1}
        with pytest.raises(T.TTCFError) as e:  # one mother in two parts
            ctx.ttcf_graph_create_multi([part, dict(part)], nst, 1)
        assert e.value.code == T.TTCF_EINVAL


def test_graph_with_parallel_mother_copies(T):
    """Mother copies (kicked, decorrelated) persist across replays: the first replay equals
    eager replicated sampling bit for bit, and two replays of 2 states per copy equal one
    replay of 4 states per copy (the same start states; rows in another order)."""
    s = I.System(4)
    r0, p0 = I.initial_state(s, 61)
    n_rep, per, sb, nst, dec = 4, 2, 20, 25, 50
    rng = np.random.Generator(np.random.PCG64(62))
    kicks = 0.05 * rng.standard_normal((n_rep, 3, s.n))
    kicks -= kicks.mean(axis=2, keepdims=True)
    kicks = kicks.reshape(n_rep, -1)
    say("graph with mother copies")

    def mother(ctx):
        return ctx.ttcf_init_mother(gsys(T, s, 1), r0, p0, n_equil=100)

    with T.Context() as ctx:
        mid = mother(ctx)
        ctx.ttcf_sample_states_replicated(mid, n_rep, kicks, dec, per, sb)
        ctx.ttcf_spawn_daughters(mid, n_rep * per, 0, 0.02, nst)
        ctx.ttcf_step(nst)
        ctx.ttcf_accumulate()
        eager = ctx.ttcf_response(nst + 1, 0.02)
    with T.Context() as ctx:
        mid = mother(ctx)
        g = ctx.ttcf_graph_create(mid, per, sb, 0.02, nst, max_replays=2, n_replicas=n_rep,
                                  kicks=kicks, decorrelate_steps=dec)
        g.launch(1)
        _same_response(ctx.ttcf_response(nst + 1, 0.02), eager)
        g.launch(1)
        two = ctx.ttcf_response(nst + 1, 0.02)
        m_after = ctx.ttcf_export_mother(mid)
    with T.Context() as ctx:
        mid = mother(ctx)
        g = ctx.ttcf_graph_create(mid, 2 * per, sb, 0.02, nst, max_replays=1, n_replicas=n_rep,
                                  kicks=kicks, decorrelate_steps=dec)
        g.launch(1)
        one = ctx.ttcf_response(nst + 1, 0.02)
        m_before = ctx.ttcf_export_mother(mid)
    assert two[4] == one[4] == 2 * n_rep * per
    for x, y in zip(two[:4], one[:4]):
        np.testing.assert_allclose(x, y, rtol=1e-9, atol=1e-12 * np.abs(y).max())
    # the copies ran, not the context's mother
    assert m_after[3] == m_before[3] and np.array_equal(m_after[0], m_before[0])


# ----------------------------------------------------------------------------------------
# the mother on the GPU
# ----------------------------------------------------------------------------------------

def test_gpu_mother_is_canonical_at_T(T):
    """A long GPU mother run holds the target temperature and samples states with zero-mean
    P_xy (<Omega(0)> = 0)."""
    s = I.System(4)
    r0, p0 = I.initial_state(s, 11)
    say("gpu mother statistics")
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(gsys(T, s, 1), r0, p0, n_equil=2000, n_melt=1000, t_melt=2.0)
        ctx.ttcf_record_mother(mid, 200000)
        ctx.ttcf_sample_states(mid, 2000, 100)
        vp = ctx.ttcf_export_mother_series(mid, 200000)
        r, p = ctx.ttcf_export_states(mid, 2000)
    assert len(vp) == 200000
    ke = 0.5 * np.sum(p * p, axis=1)
    temp = 2 * ke / s.nf
    assert temp.mean() == pytest.approx(s.temperature, rel=0.01)
    blocks = vp.reshape(50, -1).mean(axis=1)
    se = blocks.std(ddof=1) / np.sqrt(50)
    assert abs(blocks.mean()) < 3 * se
    # every stored state is inside the box
    rr = r.reshape(2000, 3, s.n)
    assert np.all(rr >= 0) and np.all(rr < s.box)


# ----------------------------------------------------------------------------------------
# the headline workload at full size, in the benchmark's launch configuration
# ----------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def cfg2(orc):
    """Config 2's system, N=2048: 16 start states of an oracle mother (400 steps, then every
    50), the benchmark's batch made by tiling them to 1024."""
    s = I.System(8)
    box, sr16, sp16 = oracle_states(orc, s, seed=2, n_states=16, n_melt=0, n_equil=400,
                                    between=50)
    return s, box, sr16, sp16


@pytest.mark.parametrize("gd", [1e-2, 1.0])
def test_config2_full_size_sampled(T, orc, cfg2, gd):
    """N=2048, 1024 start states x 4 mappings = 4096 daughters x 500 steps, FP32 forces, in
    one persistent launch, at a shear rate of the sweep (at 1.0 the Lees-Edwards offset passes
    L_x, 1.25 L_x at the end). The oracle recomputes a sample of 8 daughters; their first 50
    steps agree element by element to 1e-4; every daughter keeps its kinetic energy, the mapped
    P_xy(0) cancel, and every group stays healthy."""
    s, box, sr16, sp16 = cfg2
    reps = 64
    sr = np.tile(sr16, (reps, 1))
    sp = np.tile(sp16, (reps, 1))
    nst = 500
    say(f"config 2 full size: 4096 daughters x 500 steps at {gd}")
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(gsys(T, s, 1), sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        first = ctx.ttcf_spawn_daughters(mid, 1024, 0, gd, nst)
        ctx.ttcf_step(nst)
        sample = [0, 1, 2, 3, 4 * 517 + 0, 4 * 517 + 1, 4 * 517 + 2, 4 * 517 + 3]
        ser = np.stack([ctx.ttcf_export_series(first + d, 1, nst + 1)[0] for d in sample])
        allv0 = ctx.ttcf_export_series(first, 4096, 1)[:, 0]
        fin = [ctx.ttcf_export_daughter(first + d, s.n) for d in (0, 4095)]
        assert ctx.ttcf_accumulate() == 1024
        tm, tse, dm, dse, used = ctx.ttcf_response(nst + 1, gd)
    assert used == 1024 and np.all(np.isfinite(tm)) and np.all(np.isfinite(dm))
    st_of = np.array([d // 4 for d in sample]) % 16
    mp_of = np.array([d % 4 for d in sample])
    vo, _ = orc.run_daughters(box, sr16, sp16, st_of, mp_of, np.full(len(sample), gd), s.dt, 50,
                              nthreads=8)
    scale = np.std(vo)
    assert np.abs(ser[:, :51] - vo).max() / scale <= 1e-4
    v0 = allv0.reshape(1024, 4)
    np.testing.assert_allclose(v0.sum(axis=1), 0.0, atol=1e-5 * np.abs(v0).max())
    for (rg, pg, k), d in zip(fin, (0, 4095)):
        assert k == nst
        k_start = 0.5 * np.sum(sp[d // 4] ** 2)
        assert 0.5 * np.sum(pg ** 2) == pytest.approx(k_start, rel=1e-13)


def test_config2_response_of_16_states_matches_oracle(T, orc, cfg2):
    """The full 500 steps of config 2's system at 1e-2 from 16 start states (64 daughters):
    the GPU's TTCF and direct average (FP32 forces) against the oracle's own daughters and
    estimator (FP64), within 2 combined standard errors at every time point (Eq. TTCF)."""
    s, box, sr16, sp16 = cfg2
    nst, gd = 500, 1e-2
    say("config 2, 16 states x 4 mappings x 500 steps")
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(gsys(T, s, 1), sr16[0], sp16[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr16, sp16)
        ctx.ttcf_spawn_daughters(mid, 16, 0, gd, nst)
        ctx.ttcf_step(nst)
        assert ctx.ttcf_accumulate() == 16
        tm, tse, dm, dse, used = ctx.ttcf_response(nst + 1, gd)
    assert used == 16
    state_of = np.repeat(np.arange(16), 4)
    map_of = np.tile(np.arange(4), 16)
    vo, _ = orc.run_daughters(box, sr16, sp16, state_of, map_of, np.full(64, gd), s.dt, nst,
                              nthreads=16)
    oref = orc.ttcf_response(vo / s.volume, vo[:, 0], np.full(64, gd), s.temperature, s.dt)
    comb = np.hypot(tse, oref.ttcf_se)
    assert np.all(np.abs(tm - oref.ttcf)[1:] <= 2.0 * comb[1:])
    assert np.all(np.abs(dm - oref.dav) <= 2.0 * np.hypot(dse, oref.dav_se) + 1e-15)
    # the same start states: over the first 50 steps (trajectories equal to 1e-4) the two
    # estimates agree to 1e-3 of the per-state responses' scale
    assert np.all(np.abs(tm - oref.ttcf)[:51] <= 1e-3 * np.abs(oref.g).max())
