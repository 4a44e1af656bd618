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
    mom, st = slice(2, 33), slice(33, 64)
    assert np.abs(f0[mom]).max() > 0 and np.abs(f0[st]).max() > 0
    # p -> -p: momenta flip, kinetic stress and P_xy unchanged
    np.testing.assert_allclose(f[1][mom], -f0[mom], atol=1e-12)
    np.testing.assert_allclose(f[1][st], f0[st], atol=1e-12)
    # (x, px) -> (-x, -px): momenta and stress flip, as do P_xy and Omega
    np.testing.assert_allclose(f[2][mom], -f0[mom], atol=1e-12)
    np.testing.assert_allclose(f[2][st], -f0[st], atol=1e-12)
    np.testing.assert_allclose(f[2][:2], -f0[:2], rtol=1e-10)
    # (x, py, pz) -> (-x, -py, -pz): momenta unchanged, stress flips
    np.testing.assert_allclose(f[3][mom], f0[mom], atol=1e-12)
    np.testing.assert_allclose(f[3][st], -f0[st], atol=1e-12)
    # slab sums add up to the totals
    assert f0[mom].sum() == pytest.approx(p[:s.n].sum(), abs=1e-10)
    assert f0[st].sum() == pytest.approx(np.dot(p[:s.n], p[s.n:2 * s.n]), rel=1e-12)


def test_features_of_a_hand_placed_state():
    """Atoms placed by hand in known slabs (centres, lower edges, the top edge of the box) with
    momenta chosen per slab: every feature entry equals its value counted by hand, so a
    slab-index, offset or component error fails here. Omega(0) = -(V/T) gamma_dot P_xy(0)."""
    ly = 31.0 * 0.7                    # slab width 0.7
    box = (5.0, ly, 6.0)
    V, T, gd = box[0] * box[1] * box[2], 0.9, 3e-3
    ys, pxs, pys = [], [], []
    for k in (0, 3, 17, 30):           # slab centres
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
    r = np.concatenate([np.linspace(0.1, 4.9, n), np.array(ys), np.full(n, 3.0)])
    p = np.concatenate([np.array(pxs), np.array(pys), np.linspace(-1.0, 1.0, n)])
    vpxy0 = 12.5
    f = M.features(r, p, box, vpxy0, gd, T, V)
    assert f.shape == (64,)
    assert f[0] == vpxy0 / V
    assert f[1] == pytest.approx(-(V / T) * gd * (vpxy0 / V), rel=1e-15)
    mom = np.zeros(31)
    st = np.zeros(31)
    mom[0], st[0] = 1.0, 2.0
    mom[3], st[3] = 4.0, 8.0
    mom[17], st[17] = 18.0, 36.0
    mom[30], st[30] = 31.0 + 10.0, 62.0 - 10.0
    mom[5], st[5] = -4.0, -2.0
    assert np.array_equal(f[2:33], mom)
    assert np.array_equal(f[33:64], st)
