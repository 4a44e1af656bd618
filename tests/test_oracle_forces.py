"""Pins of the oracle's pair forces, cell lists and pair lists against independent checks:
closed-form two-body values, an O(N^2) sum over explicit images, finite differences of the
energy (force and strain derivative) and exact invariants."""
import os

import numpy as np
import pytest

import ttcf_inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _liquid(orc, n_cells=4, steps=300, seed=11):
    """A short Nose-Hoover run from the fcc lattice: a disordered configuration."""
    s = I.System(n_cells)
    r, p = I.initial_state(s, seed)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, steps, s.temperature, s.dt, orc.nh_q(s.nf, s.temperature, 0.25), s.nf)
    return s, box, st.r.copy(), st.p.copy()


def test_two_body_closed_forms(orc):
    rows = np.loadtxt(os.path.join(GOLDEN, "wca_pair.txt"))
    box = orc.make_box(2, 10.0)
    assert box.u_shift == pytest.approx(1.0, abs=1e-15)
    for r, phi, fmag in rows:
        for direction in (np.array([1.0, 0, 0]), np.array([0, 1.0, 0]),
                          np.array([1.0, -1.0, 1.0]) / np.sqrt(3.0)):
            pos = np.array([[5.0, 5.0, 5.0], [5.0, 5.0, 5.0]]).T.copy()
            pos[:, 1] = pos[:, 0] + r * direction
            f, u, w, npair = orc.forces(box, pos)
            assert u == pytest.approx(phi, abs=1e-13)
            # force on atom 0 points away from atom 1 (repulsive)
            np.testing.assert_allclose(f[:, 0], -fmag * direction, atol=1e-12)
            np.testing.assert_allclose(f[:, 0] + f[:, 1], 0.0, atol=1e-12)
            # virial x_01 F_y,01 for the pair
            assert w == pytest.approx((-r * direction[0]) * (-fmag * direction[1]), abs=1e-12)


@pytest.mark.parametrize("n_cells,dx_frac", [(3, 0.0), (3, 0.31), (4, 0.0), (4, -0.77),
                                              (4, 0.5), (5, 0.123)])
def test_cells_match_brute_force(orc, n_cells, dx_frac):
    s = I.System(n_cells)
    box = orc.make_box(s.n, s.box)
    r = I.perturbed_positions(s, 100 + n_cells, amplitude=0.12)
    dxle = dx_frac * s.box
    f1, u1, w1, n1 = orc.forces(box, r, dxle)
    f2, u2, w2, n2 = orc.forces(box, r, dxle, brute=True)
    assert n1 == n2
    scale = np.abs(f2).max()
    assert np.abs(f1 - f2).max() <= 1e-13 * scale
    assert abs(u1 - u2) <= 1e-13 * abs(u2)
    assert abs(w1 - w2) <= 1e-12 * (np.abs(f2).sum() * s.box / s.n)


def test_liquid_brute_force_and_net_force(orc):
    s, box, r, _ = _liquid(orc)
    for dxle in (0.0, 2.71, s.box - 1e-9):
        f1, u1, w1, _ = orc.forces(box, r, dxle)
        f2, u2, w2, _ = orc.forces(box, r, dxle, brute=True)
        assert np.abs(f1 - f2).max() <= 1e-13 * np.abs(f2).max()
        # Newton's third law: zero net force
        assert np.abs(f1.sum(axis=1)).max() <= 1e-12 * np.linalg.norm(f1, axis=0).sum()


def test_force_is_minus_energy_gradient(orc):
    s, box, r, _ = _liquid(orc, n_cells=3, steps=200)
    rng = np.random.Generator(np.random.PCG64(5))
    dxle = 1.3
    f, _, _, _ = orc.forces(box, r, dxle)
    h = 1e-6
    for _ in range(12):
        a = int(rng.integers(s.n))
        c = int(rng.integers(3))
        rp = r.copy()
        rm = r.copy()
        rp[c * s.n + a] += h
        rm[c * s.n + a] -= h
        up = orc.forces(box, rp, dxle)[1]
        um = orc.forces(box, rm, dxle)[1]
        fd = -(up - um) / (2 * h)
        assert fd == pytest.approx(f[c, a], rel=1e-6, abs=1e-6)


def test_virial_is_minus_strain_derivative(orc):
    """Under an affine shear x -> x + eps*y (with the sliding-brick offset moving by eps*Ly)
    the energy changes at rate -W_xy: the virial that enters P_xy."""
    s, box, r, _ = _liquid(orc, n_cells=3, steps=200)
    dxle = 0.9
    w = orc.forces(box, r, dxle)[2]

    def energy(eps):
        rr = r.reshape(3, s.n).copy()
        rr[0] = rr[0] + eps * rr[1]
        return orc.forces(box, rr.ravel(), dxle + eps * s.box)[1]

    h = 1e-6
    dudeps = (energy(h) - energy(-h)) / (2 * h)
    assert -dudeps == pytest.approx(w, rel=1e-6)


@pytest.mark.parametrize("dx_frac", [0.0, 0.37, -0.61, 0.999999])
def test_pair_lists_equal_brute_force(orc, dx_frac):
    s, box, r, _ = _liquid(orc, n_cells=4, steps=100, seed=3)
    dxle = dx_frac * s.box
    for rlist in (box.rc, 0.9 * box.rc):
        a = orc.pairs(box, r, dxle, rlist)
        b = orc.pairs(box, r, dxle, rlist, brute=True)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_cell_list_is_canonical_and_geometric(orc):
    s, box, r, _ = _liquid(orc, n_cells=4, steps=100, seed=4)
    d = orc.cell_dims(box)
    cell_of, order, start = orc.cell_list(box, r)
    assert start[0] == 0 and start[-1] == s.n and np.all(np.diff(start) >= 0)
    # order lists every atom once, sorted by (cell, id)
    assert sorted(order.tolist()) == list(range(s.n))
    keys = cell_of[order].astype(np.int64) * s.n + order
    assert np.all(np.diff(keys) > 0)
    for c in range(int(d.prod())):
        assert np.all(cell_of[order[start[c]:start[c + 1]]] == c)
    # every atom lies inside its cell's box (up to rounding of the cell index)
    rr = r.reshape(3, s.n)
    cx = cell_of % d[0]
    cy = (cell_of // d[0]) % d[1]
    cz = cell_of // (d[0] * d[1])
    for comp, cc, nn in ((0, cx, d[0]), (1, cy, d[1]), (2, cz, d[2])):
        w = s.box / nn
        assert np.all(rr[comp] >= cc * w - 1e-12) and np.all(rr[comp] < (cc + 1) * w + 1e-12)


@pytest.mark.parametrize("n_cells,dx_frac", [(4, 0.0), (4, 0.4), (4, -0.4), (5, 0.999999),
                                              (6, 0.25)])
def test_verlet_lists_equal_brute_force(orc, n_cells, dx_frac):
    """Verlet lists of radius rc + skin (walked through the grid of cells at least that wide)
    hold exactly the pairs that an all-pairs test over the sliding-brick images finds, at
    several skins and Lees-Edwards offsets; the per-atom view lists both directions in
    ascending order."""
    s, box, r, _ = _liquid(orc, n_cells=n_cells, steps=100, seed=30 + n_cells)
    dxle = dx_frac * s.box
    for skin in (0.1, 0.25, 0.37, 0.6):
        rl = box.rc + skin
        if s.box / rl < 4:
            continue
        a = orc.pairs(box, r, dxle, rl)
        b = orc.pairs(box, r, dxle, rl, brute=True)
        assert len(a[0]) > 0
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        lists = orc.verlet_lists(box, r, rl, dxle)
        assert sum(len(x) for x in lists) == 2 * len(a[0])
        for i in (0, s.n // 2, s.n - 1):
            assert np.all(np.diff(lists[i]) > 0) and i not in lists[i]
            for j in lists[i]:
                assert i in lists[j]
        # nested radii: the list of a larger skin contains that of a smaller one
        inner = set(zip(*orc.pairs(box, r, dxle, box.rc)))
        assert inner <= set(zip(a[0].tolist(), a[1].tolist()))


def test_list_grid_cell_list(orc):
    """The cell list on the grid of a list radius: floor(L / (rc + skin)) cells per edge,
    canonical (cell, id) order, every atom inside its cell, and a radius whose grid would have
    fewer than 4 x 3 x 3 cells is refused."""
    s, box, r, _ = _liquid(orc, n_cells=5, steps=100, seed=6)
    rl = box.rc + 0.37
    d = orc.grid_dims(box, rl)
    assert np.array_equal(d, np.floor(s.box / rl).astype(np.int32) * np.ones(3, np.int32))
    cell_of, order, start = orc.cell_list(box, r, d)
    keys = cell_of[order].astype(np.int64) * s.n + order
    assert np.all(np.diff(keys) > 0) and start[-1] == s.n
    rr = r.reshape(3, s.n)
    w = s.box / d[0]
    for comp, cc in ((0, cell_of % d[0]), (1, (cell_of // d[0]) % d[1]),
                     (2, cell_of // (d[0] * d[1]))):
        assert np.all(rr[comp] >= cc * w - 1e-12) and np.all(rr[comp] < (cc + 1) * w + 1e-12)
    with pytest.raises(ValueError):
        orc.grid_dims(box, s.box / 3.5)
