"""Pins of the learned-control-variate oracle: closed-form bfloat16 rounding and GELU
identities, gradients against central finite differences, Adam's first step, the exact
g = 0 reduction to plain TTCF, unbiasedness for a fixed control variate, and the sign
flips of the start-state features under the phase-space mappings."""
import numpy as np
import pytest

import ttcf_inputs as I
from oracle import mlp as M


def test_bf16_rounding_closed_forms():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -2.5, 1.0 + 2.0 ** -7 + 2.0 ** -8])
    got = M.bf16_round(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa wins (1); 1 + 0.75 ulp rounds up;
    # 1 + 1.5 ulp is a tie between 1 + ulp (odd) and 1 + 2 ulp (even)
    np.testing.assert_array_equal(got, [1.0, 1.0, 1.0 + 2.0 ** -7, -2.5, 1.0 + 2.0 ** -6])


def test_gelu_identities():
    z = np.linspace(-4, 4, 41)
    # erf is odd: gelu(z) - gelu(-z) = z; gelu(0) = 0; gelu'(0) = 1/2
    np.testing.assert_allclose(M.gelu(z) - M.gelu(-z), z, atol=1e-15)
    assert M.gelu(np.array([0.0]))[0] == 0.0
    assert M.gelu_grad(np.array([0.0]))[0] == pytest.approx(0.5, abs=1e-15)
    h = 1e-6
    np.testing.assert_allclose(M.gelu_grad(z), (M.gelu(z + h) - M.gelu(z - h)) / (2 * h),
                               rtol=1e-8, atol=1e-9)


def test_gradients_match_finite_differences():
    rng = np.random.Generator(np.random.PCG64(1))
    net = M.init_weights(8, 16, 5, seed=2)
    for p in net.params():
        p += 0.1 * rng.standard_normal(p.shape)
    x = rng.standard_normal((12, 8))
    t = rng.standard_normal((12, 5))
    y, cache = M.forward(net, x)
    g = M.backward(net, cache, y, t)
    h = 1e-6
    for pa, ga in zip(net.params(), g.params()):
        flat = pa.reshape(-1)
        gflat = ga.reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = M.mse_loss(M.forward(net, x)[0], t)
            flat[idx] = old - h
            lm = M.mse_loss(M.forward(net, x)[0], t)
            flat[idx] = old
            assert gflat[idx] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-10)


def test_adam_first_step_is_signed_learning_rate():
    net = M.init_weights(4, 6, 3, seed=3)
    before = net.flat().copy()
    grad = M.MLP(*[np.where(np.arange(p.size).reshape(p.shape) % 2, 1.0, -2.0)
                   for p in net.params()])
    opt = M.Adam(lr=0.01)
    opt.step(net, grad)
    # bias-corrected m/sqrt(v) = g/|g| on the first step (up to eps)
    np.testing.assert_allclose(net.flat() - before, -0.01 * np.sign(grad.flat()), rtol=1e-6)


def test_zero_network_reduces_to_plain_ttcf():
    import oracle as orc
    rng = np.random.Generator(np.random.PCG64(4))
    nd, nt, dt, temp = 16, 11, 0.01, 0.72
    b = rng.standard_normal((nd, nt))
    vp0 = rng.standard_normal(nd) * 5
    gam = np.full(nd, 1e-2)
    res = orc.ttcf_response(b, vp0, gam, temp, dt)
    om = orc.omega0(vp0, gam, temp)
    h = M.cv_h(np.zeros((nd, nt - 1)), np.zeros(nd), om, dt)
    est, se, _ = M.cv_estimate(res.g, h, np.zeros(nt))
    np.testing.assert_array_equal(est, res.ttcf)
    np.testing.assert_allclose(se, res.ttcf_se, rtol=1e-12)


def test_fixed_control_variate_is_unbiased_and_reduces_variance():
    """G = a + c z + e, H = c z with E[z] = mu known: the CV estimate of a is unbiased and
    its spread over repeated samples is that of e alone."""
    rng = np.random.Generator(np.random.PCG64(5))
    a, c, mu = 0.3, 2.0, 0.7
    plain, cv = [], []
    for _ in range(400):
        z = mu + rng.standard_normal(64)
        e = 0.1 * rng.standard_normal(64)
        g = (a + c * z + e)[:, None]
        h = np.repeat((c * z)[:, None], 4, axis=0)  # four identical "mappings" per state
        est, _, _ = M.cv_estimate(g, h, np.array([c * mu]))
        cv.append(est[0])
        plain.append(g.mean())
    cv = np.array(cv)
    plain = np.array(plain)
    assert abs(cv.mean() - (a + c * mu)) < 3 * cv.std() / np.sqrt(len(cv))
    assert cv.std() == pytest.approx(0.1 / 8, rel=0.15)
    assert plain.std() > 10 * cv.std()


def test_features_flip_sign_under_mappings(orc):
    """Eq. (mappings) on every feature block, and the slab sums against totals from the C
    oracle (its own cell-list forces and W_xy, a separate implementation)."""
    s = I.System(3)
    r = I.perturbed_positions(s, 2, 0.1).ravel()
    p = I.maxwell_boltzmann(s.n, s.temperature, 2).ravel()
    box = orc.make_box(s.n, s.box)
    gd, T, V = 1e-4, s.temperature, s.volume
    f = []
    for m in range(4):
        rm, pm = orc.apply_mapping(box, m, r, p)
        f.append(M.features(rm, pm, (s.box,) * 3, orc.vpxy(box, rm, pm), gd, T, V))
    f0 = f[0]
    mom, st, vir = slice(2, 22), slice(22, 42), slice(42, 62)
    assert np.abs(f0[mom]).max() > 0 and np.abs(f0[st]).max() > 0 and np.abs(f0[vir]).max() > 0
    assert f0[62] != 0 and f0[63] != 0
    # p -> -p: momenta and both rates flip; kinetic and configurational stress, P_xy unchanged
    np.testing.assert_allclose(f[1][mom], -f0[mom], atol=1e-12)
    np.testing.assert_allclose(f[1][st], f0[st], atol=1e-12)
    np.testing.assert_allclose(f[1][vir], f0[vir], rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(f[1][62:], -f0[62:], rtol=1e-10)
    # (x, px) -> (-x, -px): everything flips, P_xy and Omega too
    np.testing.assert_allclose(f[2][mom], -f0[mom], atol=1e-12)
    np.testing.assert_allclose(f[2][st], -f0[st], atol=1e-12)
    np.testing.assert_allclose(f[2][vir], -f0[vir], rtol=1e-8, atol=1e-8)
    np.testing.assert_allclose(f[2][62:], -f0[62:], rtol=1e-8)
    np.testing.assert_allclose(f[2][:2], -f0[:2], rtol=1e-10)
    # (x, py, pz) -> (-x, -py, -pz): momenta and rates unchanged, both stresses flip
    np.testing.assert_allclose(f[3][mom], f0[mom], atol=1e-12)
    np.testing.assert_allclose(f[3][st], -f0[st], atol=1e-12)
    np.testing.assert_allclose(f[3][vir], -f0[vir], rtol=1e-8, atol=1e-8)
    np.testing.assert_allclose(f[3][62:], f0[62:], rtol=1e-8)
    # slab sums add up to the totals; the configurational ones to the C oracle's W_xy, and
    # the first rate to its forces
    assert f0[mom].sum() == pytest.approx(p[:s.n].sum(), abs=1e-10)
    assert f0[st].sum() == pytest.approx(np.dot(p[:s.n], p[s.n:2 * s.n]), rel=1e-12)
    F, _, w, _ = orc.forces(box, r)
    assert f0[vir].sum() == pytest.approx(w, rel=1e-10)
    pp = p.reshape(3, s.n)
    assert f0[62] == pytest.approx(np.sum(F[0] * pp[1] + pp[0] * F[1]), rel=1e-10)


def test_features_of_a_close_pair():
    """Two atoms closer than r_c in slabs 3 and 4 (the rest of the box empty): each slab holds
    half the pair virial, the first rate is sum F_x p_y + p_x F_y and the second
    (p_x,A - p_x,B) F_y on A, with the force from the C oracle."""
    import oracle as orc
    box = (5.0, 20 * 0.7, 6.0)
    V = box[0] * box[1] * box[2]
    r = np.array([1.0, 1.6, 2.45, 2.9, 3.0, 3.0])      # A in slab 3, B in slab 4
    p = np.array([0.7, -1.1, 0.3, 0.9, 0.2, -0.4])
    f = M.features(r, p, box, 0.0, 1e-3, 1.0, V)
    F, _, w, npairs = orc.forces(orc.make_box(2, box), r)
    assert npairs == 1 and F[1, 0] != 0
    vir = np.zeros(20)
    vir[3] = vir[4] = 0.5 * (r[0] - r[1]) * F[1, 0]
    np.testing.assert_allclose(f[42:62], vir, rtol=1e-12, atol=0)
    assert f[42:62].sum() == pytest.approx(w, rel=1e-12)
    d1 = sum(F[0, a] * p[2 + a] + p[a] * F[1, a] for a in range(2))
    assert f[62] == pytest.approx(d1, rel=1e-12)
    assert f[63] == pytest.approx((p[0] - p[1]) * F[1, 0], rel=1e-12)
    assert np.all(f[2:42][[0 + 3, 0 + 4]] == p[:2]) and f[22 + 3] == p[0] * p[2]


def test_features_of_a_hand_placed_state():
    """Atoms placed by hand in known slabs (centres, lower edges, the top edge of the box) with
    momenta chosen per slab: every feature entry equals its value counted by hand, so a
    slab-index, offset or component error fails here. Omega(0) = -(V/T) gamma_dot P_xy(0)."""
    ly = 20.0 * 0.7                    # slab width 0.7
    box = (5.0, ly, 9.0)
    V, T, gd = box[0] * box[1] * box[2], 0.9, 3e-3
    ys, pxs, pys = [], [], []
    for k in (0, 3, 17, 19):           # slab centres
        ys.append((k + 0.5) * 0.7)
        pxs.append(k + 1.0)
        pys.append(2.0)
    ys.append(5 * 0.7)                 # exactly on the lower edge of slab 5
    pxs.append(-4.0)
    pys.append(0.5)
    ys.append(np.nextafter(ly, 0.0))   # just below L_y: the last slab
    pxs.append(10.0)
    pys.append(-1.0)
    n = len(ys)
    # z 1.5 apart: no pair comes closer than r_c
    r = np.concatenate([np.linspace(0.1, 4.9, n), np.array(ys), 1.5 * np.arange(n)])
    p = np.concatenate([np.array(pxs), np.array(pys), np.linspace(-1.0, 1.0, n)])
    vpxy0 = 12.5
    f = M.features(r, p, box, vpxy0, gd, T, V)
    assert f.shape == (64,)
    assert f[0] == vpxy0 / V
    assert f[1] == pytest.approx(-(V / T) * gd * (vpxy0 / V), rel=1e-15)
    mom = np.zeros(20)
    st = np.zeros(20)
    mom[0], st[0] = 1.0, 2.0
    mom[3], st[3] = 4.0, 8.0
    mom[17], st[17] = 18.0, 36.0
    mom[19], st[19] = 20.0 + 10.0, 40.0 - 10.0
    mom[5], st[5] = -4.0, -2.0
    assert np.array_equal(f[2:22], mom)
    assert np.array_equal(f[22:42], st)
    assert np.all(f[42:] == 0.0)  # no pair closer than r_c
