"""Pins of the oracle's observables beyond P_xy (normal-stress differences, energy per atom and
the bulk momentum profile by y slab), by checks that do not reuse its formulas: the closed
form of one WCA pair at r = sigma (phi = epsilon, |F| = 24 epsilon / sigma), the pair's
orientation (which fixes every index of the diagonal), the virial as the strain derivative of
the potential energy, the kinetic parts of a non-interacting gas, the slab assignment of atoms
placed by hand, and the parities of Eq. (mappings)."""
import numpy as np
import pytest

import ttcf_inputs as I

L = 10.0


def pair_along(orc, axis):
    box = orc.make_box(2, [L, L, L])
    r = np.full((3, 2), 5.0)
    r[axis, 0] = 4.5
    r[axis, 1] = 5.5  # separation exactly 1 (sigma)
    return box, r.ravel(), np.zeros(6)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_one_pair_at_sigma(orc, axis):
    box, r, p = pair_along(orc, axis)
    out = orc.observables(box, r, p)
    w = np.zeros(3)
    w[axis] = 24.0  # r_a F_a for the pair: |r| = 1, |F| = 24
    vol = L ** 3
    assert out[0] == pytest.approx((w[0] - w[1]) / vol, abs=1e-15)
    assert out[1] == pytest.approx((w[1] - w[2]) / vol, abs=1e-15)
    assert out[2] == pytest.approx(1.0 / 2, abs=1e-15)  # U = phi(sigma) = 1 over N = 2
    assert np.all(out[3:] == 0.0)


def test_kinetic_parts_of_a_free_gas(orc):
    # 27 atoms on a 3x3x3 grid of spacing 3 > r_c: no pair interacts
    g = np.arange(3) * 3.0 + 0.5
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    box = orc.make_box(27, [9.0, 9.0, 9.0])
    r = np.concatenate([x.ravel(), y.ravel(), z.ravel()])
    p = np.random.default_rng(3).normal(size=81)
    out = orc.observables(box, r, p, n_slabs=3)
    px, py, pz = p[:27], p[27:54], p[54:]
    vol = 729.0
    assert out[0] == pytest.approx((px @ px - py @ py) / vol, rel=1e-13)
    assert out[1] == pytest.approx((py @ py - pz @ pz) / vol, rel=1e-13)
    assert out[2] == pytest.approx(0.5 * (p @ p) / 27, rel=1e-13)
    # slab s holds the atoms with y = 3 s + 0.5
    for s in range(3):
        sel = np.isclose(y.ravel(), 3 * s + 0.5)
        assert out[3 + s] == pytest.approx(px[sel].sum() / (vol / 3), rel=1e-13)


def test_slab_sums_add_up_to_the_total_momentum(orc):
    s = I.System(4)
    r, p = I.initial_state(s, 7)
    box = orc.make_box(s.n, s.box)
    out = orc.observables(box, r.ravel(), p.ravel())
    vol = s.volume
    total = out[3:].sum() * vol / len(out[3:])
    assert total == pytest.approx(p.ravel()[: s.n].sum(), abs=1e-11)


@pytest.mark.parametrize("dxle", [0.0, 1.7])
def test_virial_is_the_strain_derivative_of_the_energy(orc, dxle):
    # W_aa = sum_pairs r_a F_a = -dU/d lambda for the affine stretch r_a -> lambda r_a,
    # L_a -> lambda L_a (a stretch along x stretches the Lees-Edwards offset as well); U from
    # the brute-force pair sum over all pairs
    s = I.System(4)
    r = I.perturbed_positions(s, 11).ravel()
    n = s.n
    h = 1e-6

    def energy(axis, lam):
        edges = np.full(3, s.box)
        edges[axis] *= lam
        rr = r.copy()
        rr[axis * n:(axis + 1) * n] *= lam
        return orc.forces(orc.make_box(n, edges), rr, dxle=dxle * (lam if axis == 0 else 1.0),
                          brute=True)[1]

    w = [-(energy(a, 1 + h) - energy(a, 1 - h)) / (2 * h) for a in range(3)]
    out = orc.observables(orc.make_box(n, s.box), r, np.zeros(3 * n), dxle=dxle)
    vol = s.volume
    scale = max(abs(v) for v in w)
    assert scale > 1.0
    assert out[0] * vol == pytest.approx(w[0] - w[1], abs=1e-6 * scale)
    assert out[1] * vol == pytest.approx(w[1] - w[2], abs=1e-6 * scale)


def test_energy_is_kinetic_plus_the_brute_force_pair_sum(orc):
    s = I.System(4)
    r = I.perturbed_positions(s, 5).ravel()
    p = I.maxwell_boltzmann(s.n, s.temperature, 6).ravel()
    box = orc.make_box(s.n, s.box)
    u = orc.forces(box, r, dxle=0.9, brute=True)[1]
    out = orc.observables(box, r, p, dxle=0.9)
    assert out[2] * s.n == pytest.approx(0.5 * (p @ p) + u, rel=1e-13)


def test_mapping_parities(orc):
    s = I.System(4)
    r = I.perturbed_positions(s, 21).ravel()
    p = I.maxwell_boltzmann(s.n, s.temperature, 22).ravel()
    box = orc.make_box(s.n, s.box)
    base = orc.observables(box, r, p)
    for m in range(4):
        rm, pm = orc.apply_mapping(box, m, r, p)
        out = orc.observables(box, rm, pm)
        # the normal-stress differences and the energy are even under every mapping
        np.testing.assert_allclose(out[:3], base[:3], rtol=1e-12, atol=1e-14)
        # p_x keeps its sign under mappings 0 and 3 and flips under 1 and 2; y is untouched
        sign = 1.0 if m in (0, 3) else -1.0
        np.testing.assert_allclose(out[3:], sign * base[3:], rtol=1e-12, atol=1e-14)


def test_recorded_observables_follow_the_trajectory(orc):
    s = I.System(4)
    r, p = I.initial_state(s, 41)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    q = orc.nh_q(s.nf, s.temperature, 0.25)
    orc.nh_run(box, st, 300, s.temperature, s.dt, q, s.nf)
    sr, sp = st.r[None, :].copy(), st.p[None, :].copy()
    state_of = np.zeros(4, np.int32)
    map_of = np.arange(4, dtype=np.int32)
    gam = np.full(4, 0.5)
    vp, ob = orc.run_daughters_obs(box, sr, sp, state_of, map_of, gam, s.dt, 20, nthreads=4)
    vp_plain, _ = orc.run_daughters(box, sr, sp, state_of, map_of, gam, s.dt, 20, nthreads=4)
    np.testing.assert_array_equal(vp, vp_plain)
    # the first row is the observables of the mapped start state
    for m in range(4):
        rm, pm = orc.apply_mapping(box, m, st.r, st.p)
        np.testing.assert_allclose(ob[m, 0], orc.observables(box, rm, pm), rtol=1e-13,
                                   atol=1e-15)
    # the last row is the observables of the final state
    vp2, rf, pf, _ = orc.run_daughters(box, sr, sp, state_of[:1], map_of[:1], gam[:1], s.dt, 20,
                                       nthreads=1, final_state=True)
    dxle = orc.le_offset(box, 0.5, s.dt, 20)
    np.testing.assert_allclose(ob[0, -1], orc.observables(box, rf[0], pf[0], dxle=dxle),
                               rtol=1e-13, atol=1e-15)
