"""Parity of the pair-list step kernel's own list build and force pass (the device functions
that ttcf_step runs for FP32 forces, reached through ttcf_debug_pair_form) against the FP64
oracle, on liquid configurations of N = 256, 2048 and 4000 at Lees-Edwards offsets 0,
+-0.4 L_x and one reached after the strain passed L_x (Example 1's sliding brick):

  * the list grid, every atom's cell, the build's order and the cell starts are bit-exact
    against the oracle's canonical cell list on the same grid;
  * the offset the kernel used equals the oracle's fmod(gamma_dot L_y k dt, L_x) bit for bit;
  * the listed pairs closer than r_c are exactly the oracle's pair set; every oracle pair
    closer than r_list - eps is listed, and none farther than r_list + eps (eps covers the
    FP32 fixed-point separation), in cubic boxes and in one whose sides differ;
  * forces within max_i |dF_i| / rms_i |F_i| <= 1e-5 of the oracle's, W_xy within 1e-5 of
    the sum of |x_ij F_y,ij|, and the total force zero;
  * forces and W_xy do not depend on the skin or the pair capacity (bit for bit);
  * a capacity that is too small is reported, never overrun.
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


def liquid(orc, s, seed, steps):
    """Nose-Hoover runs of the oracle from the fcc lattice, melted at T = 2 and equilibrated
    at T (as the workloads' mothers are): a liquid, positions inside the box."""
    r, p = I.initial_state(s, seed)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, steps, 2.0, s.dt, orc.nh_q(s.nf, 2.0, TAU), s.nf)
    orc.nh_run(box, st, steps, s.temperature, s.dt, orc.nh_q(s.nf, s.temperature, TAU), s.nf)
    return box, st.r.copy(), st.p.copy()


# (gamma_dot, strain step k): offsets 0, +0.4 L, -0.4 L, and 1.25 L reduced to 0.25 L
def offsets(s):
    k40 = int(round(0.4 / s.dt))
    return [(0.0, 0), (1.0, k40), (-1.0, k40), (1.0, 500)]


@pytest.fixture(scope="module")
def states(orc):
    """Per system and offset, the positions of an oracle SLLOD daughter after k steps at
    gamma_dot from the liquid: a sheared configuration that carries that offset."""
    out = {}
    for name, s, seed, steps in (("n256", I.System(4), 71, 1000),
                                 ("n2048", I.System(8), 72, 1000),
                                 ("n4000", I.System(10, density=0.7), 73, 800)):
        box, r0, p0 = liquid(orc, s, seed, steps)
        for gd, k in offsets(s):
            r, p = r0.copy(), p0.copy()
            if k:
                orc.sllod_run(box, r, p, gd, s.dt, k)
            out[name, gd, k] = (s, box, r)
    return out


@pytest.mark.parametrize("name", ["n256", "n2048", "n4000"])
def test_list_grid_cells_and_order_bit_exact(T, orc, states, name):
    for gd, k in offsets(states[name, 0.0, 0][0]):
        s, box, r = states[name, gd, k]
        sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1)
        say(f"{name} grid/order at gamma_dot={gd}, k={k}")
        out = T.ttcf_debug_pair_form(sysd, r, gd, k)
        d = orc.grid_dims(box, out["rlist"])
        assert np.array_equal(out["dims"], d)
        cell_of, order, start = orc.cell_list(box, r, d)
        assert np.array_equal(out["cell_of"], cell_of)
        assert np.array_equal(out["order"], order)
        assert np.array_equal(out["start"], start)
        assert out["dxle"] == orc.le_offset(box, gd, s.dt, k)
        assert not out["overflow"] and not out["close"]


def check_pairs_and_forces(T, orc, s, box, r, gd, k, lbox):
    """The pair and force checks of the module docstring for one configuration in the box
    lbox = (L_x, L_y, L_z); returns the listed pair count."""
    sysd = T.make_system(s.n, lbox, s.temperature, s.dt, precision=1)
    rr = r.reshape(3, s.n)
    out = T.ttcf_debug_pair_form(sysd, r, gd, k)
    dxle, rl = out["dxle"], out["rlist"]
    gpu = set(zip(out["pairs"][0].tolist(), out["pairs"][1].tolist()))
    assert len(gpu) == len(out["pairs"][0])  # every pair listed once
    # oracle FP64 distance of every GPU pair
    pi, pj = np.array(sorted(gpu)).T
    dx = rr[:, pi] - rr[:, pj]
    ny = np.rint(dx[1] / lbox[1])
    dx[1] -= ny * lbox[1]
    dx[0] -= ny * dxle
    dx[0] -= lbox[0] * np.rint(dx[0] / lbox[0])
    dx[2] -= lbox[2] * np.rint(dx[2] / lbox[2])
    dist = np.sqrt((dx * dx).sum(0))
    eps = 1e-5 * rl
    assert dist.max() < rl + eps
    # inside the cutoff: exactly the oracle's pair set
    inside = {(a, b) for a, b, q in zip(pi.tolist(), pj.tolist(), dist) if q < box.rc}
    oi, oj = orc.pairs(box, r, dxle, box.rc)
    assert inside == set(zip(oi.tolist(), oj.tolist()))
    # every oracle pair within r_list - eps is listed
    vi, vj = orc.pairs(box, r, dxle, rl - eps)
    assert set(zip(vi.tolist(), vj.tolist())) <= gpu
    # forces and virial
    fo, _, wo, _ = orc.forces(box, r, dxle)
    fg = out["f"]
    rms = np.sqrt((fo * fo).sum(0).mean())
    err = np.sqrt(((fg - fo) ** 2).sum(0)).max() / rms
    say(f"   {len(gpu)} pairs, force error {err:.2e} of rms {rms:.2f}, "
        f"W {out['w_xy']:.6f} vs {wo:.6f}")
    assert err <= 1e-5
    wscale = np.abs(fo).sum() * box.rc
    assert abs(out["w_xy"] - wo) <= 1e-5 * wscale
    assert np.abs(fg.sum(axis=1)).max() <= 1e-6 * np.abs(fg).sum()
    return len(gpu)


@pytest.mark.parametrize("name", ["n256", "n2048", "n4000"])
def test_pairs_and_forces_match_oracle(T, orc, states, name):
    for gd, k in offsets(states[name, 0.0, 0][0]):
        s, box, r = states[name, gd, k]
        say(f"{name} pairs/forces at gamma_dot={gd}, k={k}")
        check_pairs_and_forces(T, orc, s, box, r, gd, k, (s.box,) * 3)


def test_pairs_and_forces_in_a_non_cubic_box(T, orc, states):
    """Fixed-point units that differ by axis: the N = 2048 configurations stretched by 1.05
    in x and y (so that the image offset, which scales with L_y and wraps at L_x,
    still matches the stretched positions; no pair comes closer), checked as above."""
    for gd, k in offsets(states["n2048", 0.0, 0][0]):
        s, _, r = states["n2048", gd, k]
        lbox = (s.box * 1.05, s.box * 1.05, s.box)
        rs = r.reshape(3, s.n) * np.array(lbox)[:, None] / s.box
        box = orc.make_box(s.n, lbox)
        say(f"n2048 non-cubic pairs/forces at gamma_dot={gd}, k={k}")
        check_pairs_and_forces(T, orc, s, box, np.ascontiguousarray(rs).ravel(), gd, k, lbox)


def test_forces_do_not_depend_on_skin_or_capacity(T, states):
    """Integer force sums: the same forces and W_xy bit for bit at every skin and capacity."""
    s, box, r = states["n2048", 1.0, 500]
    sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1)
    ref = T.ttcf_debug_pair_form(sysd, r, 1.0, 500)
    for skin, kcap in ((0.1, 0), (0.25, 12), (0.37, 0), (0.5, 30)):
        out = T.ttcf_debug_pair_form(sysd, r, 1.0, 500, skin=skin, kcap=kcap)
        assert not out["overflow"]
        assert np.array_equal(out["f"], ref["f"]) and out["w_xy"] == ref["w_xy"]


def test_capacity_overflow_is_reported(T, states):
    s, box, r = states["n256", 0.0, 0]
    sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1)
    out = T.ttcf_debug_pair_form(sysd, r, 0.0, 0, kcap=1)
    assert out["overflow"]
