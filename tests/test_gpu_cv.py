"""Learned control variate on the GPU against the FP64 oracle (runs on an MI355X).

Inputs are seeded (ttcf_inputs, seeded network weights) or produced by the oracle; the
oracle never receives anything the GPU computed. Bars:
  * network forward pass and gradient: the oracle with the same bfloat16 rounding of every
    product operand (oracle/mlp.py, bf16=True); what remains is FP32 accumulation order and
    rare one-ulp bfloat16 rounding flips of intermediate activations, bounded by
    max |d| <= 2e-3 max |ref| (forward) and 1e-2 per parameter block (gradient);
  * features and targets of daughters with FP64 forces: equal to the oracle's up to the final
    FP32 rounding (two float32 ulps);
  * h series, mapping means, the mean term and the control-variate estimate: within 2e-3 of
    the scale of the oracle's values, the bfloat16 network being the only source of
    difference.
"""
import sys

import numpy as np
import pytest

import ttcf_inputs as I
from oracle import mlp as M

pytestmark = pytest.mark.gpu

TAU = 0.25
N_OUT = 30
GD = 1e-2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    from paper_2312_02990_amd import ttcf
    ttcf.lib()
    return ttcf


@pytest.fixture(scope="module")
def cfg(orc):
    """WCA N=256 at the paper's state point; 16 start states every 100 mother steps."""
    s = I.System(4)
    r, p = I.initial_state(s, 3)
    box = orc.make_box(s.n, s.box)
    st = orc.NHState(r.ravel().copy(), p.ravel().copy())
    orc.nh_run(box, st, 1000, 2.0, s.dt, orc.nh_q(s.nf, 2.0, TAU), s.nf)
    sr, sp = orc.mother_sample(box, st, 2000, 16, 100, s.temperature, s.dt,
                               orc.nh_q(s.nf, s.temperature, TAU), s.nf)
    return s, box, sr, sp


def seeded_net(n_out, seed=11):
    """He-initialised weights with non-zero biases, rounded to FP32 (what the GPU holds)."""
    net = M.init_weights(M_IN, M_HID, n_out, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    net.b1 += 0.1 * rng.standard_normal(net.b1.shape)
    net.b2 += 0.1 * rng.standard_normal(net.b2.shape)
    net.b3 += 0.1 * rng.standard_normal(net.b3.shape)
    w32 = net.flat().astype(np.float32)
    return w32, M.MLP.from_flat(w32.astype(np.float64), M_IN, M_HID, n_out)


M_IN, M_HID = 64, 256


def gsys(T, s, precision=0):
    return T.make_system(s.n, s.box, s.temperature, s.dt, precision=precision)


def oracle_features(orc, box, s, sr, sp, states, gd):
    """Features, B(0) and Omega(0) of the four mapped copies of each start state (rows
    state-major, mapping-minor), from the oracle's mapping and P_xy."""
    rows, b0, om = [], [], []
    for k in states:
        for m in range(4):
            rm, pm = orc.apply_mapping(box, m, sr[k], sp[k])
            vp = orc.vpxy(box, rm, pm)
            f = M.features(rm, pm, (s.box,) * 3, vp, gd, s.temperature, s.volume)
            rows.append(f)
            b0.append(f[0])
            om.append(f[1])
    return np.array(rows), np.array(b0), np.array(om)


def col_stats32(a):
    """Column mean and 1/std (ddof=1) as FP32, the form in which the network stores them."""
    a = np.asarray(a, np.float64)
    mu = a.mean(axis=0)
    sd = a.std(axis=0, ddof=1)
    return mu.astype(np.float32).astype(np.float64), \
        (1.0 / np.maximum(sd, 1e-12)).astype(np.float32).astype(np.float64)


def oracle_h(net, feats32, xmu, xinv, ymu, yinv, b0, om, dt):
    xs = (feats32 - xmu) * xinv
    pred, _ = M.forward(net, xs, bf16=True)
    return M.cv_h(pred / yinv + ymu, b0, om, dt)


@pytest.fixture(scope="module")
def ctx_mother(T, cfg):
    s, box, sr, sp = cfg
    ctx = T.Context()
    mid = ctx.ttcf_init_mother(gsys(T, s), sr[0], sp[0], n_equil=0)
    yield ctx, mid
    ctx.close()


# ----------------------------------------------------------------------------------------
# the network
# ----------------------------------------------------------------------------------------

@pytest.mark.parametrize("rows", [1, 63, 200])
def test_mlp_forward_matches_bf16_oracle(T, ctx_mother, rows):
    ctx, _ = ctx_mother
    say(f"mlp forward rows={rows}")
    w32, net = seeded_net(N_OUT)
    ctx.ttcf_cv_init(N_OUT, w32)
    rng = np.random.Generator(np.random.PCG64(20 + rows))
    x = rng.standard_normal((rows, M_IN)).astype(np.float32)
    y = ctx.ttcf_mlp_forward(x)
    ref, _ = M.forward(net, x.astype(np.float64), bf16=True)
    scale = np.abs(ref).max()
    err = np.abs(y - ref)
    assert err.max() <= 2e-3 * scale
    assert err.mean() <= 2e-4 * scale
    # and bfloat16 products stay close to the exact network
    exact, _ = M.forward(net, x.astype(np.float64))
    assert np.abs(y - exact).max() <= 5e-2 * scale


def test_mlp_gradient_matches_bf16_oracle(T, ctx_mother):
    ctx, _ = ctx_mother
    rows = 96
    say("mlp gradient")
    w32, net = seeded_net(N_OUT, seed=13)
    ctx.ttcf_cv_init(N_OUT, w32)
    rng = np.random.Generator(np.random.PCG64(31))
    x = rng.standard_normal((rows, M_IN)).astype(np.float32)
    t = rng.standard_normal((rows, N_OUT)).astype(np.float32)
    g = ctx.ttcf_mlp_gradient(x, t)
    y, cache = M.forward(net, x.astype(np.float64), bf16=True)
    ref = M.backward(net, cache, y, t.astype(np.float64), bf16=True)
    gm = M.MLP.from_flat(g.astype(np.float64), M_IN, M_HID, N_OUT)
    for name, a, b in zip(("W1", "b1", "W2", "b2", "W3", "b3"), gm.params(), ref.params()):
        scale = np.abs(b).max()
        assert np.abs(a - b).max() <= 1e-2 * scale, name


def test_weights_round_trip_and_bad_sizes(T, ctx_mother):
    ctx, _ = ctx_mother
    w32, _ = seeded_net(7, seed=5)
    ctx.ttcf_cv_init(7, w32)
    assert np.array_equal(ctx.ttcf_cv_export_weights(), w32)
    with pytest.raises(T.TTCFError):
        ctx.ttcf_cv_init(7, w32[:-1])
    with pytest.raises(T.TTCFError):
        ctx.ttcf_cv_response(5, GD)  # nothing trained, no mean term


# ----------------------------------------------------------------------------------------
# features, targets, training step, h and the estimate
# ----------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def trained(T, orc, cfg):
    """16 start states x 4 mappings at shear rate 1e-2, FP64 forces, N_OUT steps; the
    training set is these 64 daughters; one Adam step on all of them."""
    s, box, sr, sp = cfg
    say("cv pipeline: daughters")
    ctx = T.Context()
    mid = ctx.ttcf_init_mother(gsys(T, s), sr[0], sp[0], n_equil=0)
    ctx.ttcf_import_states(mid, sr, sp)
    first = ctx.ttcf_spawn_daughters(mid, 16, 0, GD, N_OUT)
    ctx.ttcf_step(N_OUT)
    w32, net = seeded_net(N_OUT, seed=17)
    ctx.ttcf_cv_init(N_OUT, w32)
    ctx.ttcf_cv_add_training(first, 64)
    x, t = ctx.ttcf_cv_export_training(0, 64)
    yield dict(ctx=ctx, mid=mid, first=first, w32=w32, net=net, x=x, t=t)
    ctx.close()


def test_features_and_targets_match_oracle(T, orc, cfg, trained):
    s, box, sr, sp = cfg
    x, t = trained["x"], trained["t"]
    fo, _, _ = oracle_features(orc, box, s, sr, sp, range(16), GD)
    # one FP32 rounding of FP64 values that agree to ~1e-12: at most 2 ulps apart
    ulp = np.spacing(np.abs(fo).astype(np.float32)).astype(np.float64)
    tiny = 1e-9 * np.abs(fo).max(axis=0)
    assert np.all(np.abs(x - fo) <= 2 * ulp + tiny)
    state_of = np.repeat(np.arange(16), 4)
    map_of = np.tile(np.arange(4), 16)
    vo, _ = orc.run_daughters(box, sr, sp, state_of, map_of, np.full(64, GD), s.dt, N_OUT,
                              nthreads=8)
    to = vo[:, 1:] / s.volume
    assert np.abs(t - to).max() <= 1e-6 * np.abs(to).max()


def test_one_adam_step_matches_oracle(T, orc, cfg, trained):
    s, box, sr, sp = cfg
    ctx, net, w32 = trained["ctx"], trained["net"], trained["w32"]
    fo, _, _ = oracle_features(orc, box, s, sr, sp, range(16), GD)
    state_of = np.repeat(np.arange(16), 4)
    map_of = np.tile(np.arange(4), 16)
    vo, _ = orc.run_daughters(box, sr, sp, state_of, map_of, np.full(64, GD), s.dt, N_OUT,
                              nthreads=8)
    fo32 = fo.astype(np.float32).astype(np.float64)
    to32 = (vo[:, 1:] / s.volume).astype(np.float32).astype(np.float64)
    xmu, xinv = col_stats32(fo32)
    ymu, yinv = col_stats32(to32)
    lr = 1e-3
    ctx.ttcf_cv_init(N_OUT, w32)
    ctx.ttcf_cv_add_training(trained["first"], 64)
    loss = ctx.ttcf_cv_train(1, 64, lr)
    w1 = ctx.ttcf_cv_export_weights().astype(np.float64)
    # oracle: standardise, bf16 forward/backward, Adam
    xs = (fo32 - xmu) * xinv
    ts = (to32 - ymu) * yinv
    y, cache = M.forward(net, xs, bf16=True)
    assert loss[0] == pytest.approx(M.mse_loss(y, ts), rel=2e-3)
    g = M.backward(net, cache, y, ts, bf16=True).flat()
    ref = net.flat().copy()
    refnet = M.MLP.from_flat(ref, M_IN, M_HID, N_OUT)
    M.Adam(lr=lr).step(refnet, M.MLP.from_flat(g, M_IN, M_HID, N_OUT))
    d_gpu = w1 - w32.astype(np.float64)
    d_ref = refnet.flat() - ref
    # the first Adam step moves every weight by lr g / (|g| + eps): where the gradient is
    # well resolved the two steps agree; nowhere does a step exceed lr
    assert np.abs(d_gpu).max() <= lr * (1 + 1e-5) + 1e-7
    big = np.abs(g) > 1e-2 * np.abs(g).max()
    assert big.sum() > 0.5 * g.size
    np.testing.assert_allclose(d_gpu[big], d_ref[big], rtol=1e-3, atol=2e-8)
    # an explicit identity order is the stored order
    ctx.ttcf_cv_init(N_OUT, w32)
    ctx.ttcf_cv_add_training(trained["first"], 64)
    ctx.ttcf_cv_train(1, 64, lr, order=np.arange(64, dtype=np.int32)[None, :])
    assert np.array_equal(ctx.ttcf_cv_export_weights().astype(np.float64), w1)


def test_cv_estimate_and_mean_term_match_oracle(T, orc, cfg):
    """Fixed seeded network with the training set's statistics: the h series of every
    daughter (through G_n - H_n), and a mean term over states the oracle reproduces (one
    replica of the mother, no kick, no decorrelation), against the oracle's arithmetic."""
    s, box, sr, sp = cfg
    say("cv estimate and mean term")
    n_between, n_mean = 25, 6
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(gsys(T, s), sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        first = ctx.ttcf_spawn_daughters(mid, 16, 0, GD, N_OUT)
        ctx.ttcf_step(N_OUT)
        w32, net = seeded_net(N_OUT, seed=19)
        ctx.ttcf_cv_init(N_OUT, w32)
        ctx.ttcf_cv_add_training(first, 64)
        ctx.ttcf_cv_train(0, 64, 1e-3)  # statistics only
        ctx.ttcf_cv_attach(first, 64)
        assert ctx.ttcf_accumulate() == 16
        tm, tse, _, _, _ = ctx.ttcf_response(N_OUT + 1, GD)
        cnt = ctx.ttcf_cv_mean_term(mid, 1, None, 0, 1, n_mean, n_between, GD)
        assert cnt == n_mean
        cm, cse, pm, pse, mu, mu_se, used = ctx.ttcf_cv_response(N_OUT + 1, GD)
        np.testing.assert_array_equal(pm, tm)  # same groups, same kernel
        np.testing.assert_array_equal(pse, tse)
        assert used == 16
        # the mother itself did not move
        r_m, p_m, _, steps = ctx.ttcf_export_mother(mid)
        assert np.array_equal(r_m, sr[0]) and np.array_equal(p_m, sp[0])
    # oracle: statistics of its own training set, h of the daughters
    fo, b0, om = oracle_features(orc, box, s, sr, sp, range(16), GD)
    state_of = np.repeat(np.arange(16), 4)
    map_of = np.tile(np.arange(4), 16)
    vo, _ = orc.run_daughters(box, sr, sp, state_of, map_of, np.full(64, GD), s.dt, N_OUT,
                              nthreads=8)
    fo32 = fo.astype(np.float32).astype(np.float64)
    xmu, xinv = col_stats32(fo32)
    ymu, yinv = col_stats32((vo[:, 1:] / s.volume).astype(np.float32).astype(np.float64))
    h = oracle_h(net, fo32, xmu, xinv, ymu, yinv, b0, om, s.dt)
    hn = h.reshape(16, 4, -1).mean(axis=1)
    # mean term: the oracle's own mother from the same start, the same sampling
    st = orc.NHState(sr[0].copy(), sp[0].copy())
    mr, mp = orc.mother_sample(box, st, 0, n_mean, n_between, s.temperature, s.dt,
                               orc.nh_q(s.nf, s.temperature, TAU), s.nf)
    fm, b0m, omm = oracle_features(orc, box, s, mr, mp, range(n_mean), GD)
    hm = oracle_h(net, fm.astype(np.float32).astype(np.float64), xmu, xinv, ymu, yinv, b0m, omm,
                  s.dt).reshape(n_mean, 4, -1).mean(axis=1)
    mu_ref = hm.mean(axis=0)
    hscale = np.abs(hn).max()
    assert hscale > 0.1 * np.abs(tm).max()  # the control variate is not negligible
    np.testing.assert_allclose(mu, mu_ref, atol=2e-3 * np.abs(hm).max())
    np.testing.assert_allclose(mu_se, hm.std(axis=0, ddof=1) / np.sqrt(n_mean),
                               atol=2e-3 * np.abs(hm).max())
    # G_n - H_n + mu_H from the GPU's G (the plain response) and the oracle's H
    np.testing.assert_allclose(cm - mu, tm - hn.mean(axis=0), atol=2e-3 * hscale)
    g_n = orc.ttcf_response(vo / s.volume, vo[:, 0], np.full(64, GD), s.temperature, s.dt).g
    resid = g_n - hn
    np.testing.assert_allclose(cse, resid.std(axis=0, ddof=1) / 4.0, atol=2e-3 * hscale)


def test_calibrated_cv_matches_oracle(T, orc, cfg):
    """Start states 0-7 calibrate beta(t) = Cov(G, H) / Var(H); states 8-15 form the
    estimate mean[G - beta H] + beta mu_H. Everything against the oracle's own daughters,
    network and mother."""
    s, box, sr, sp = cfg
    say("calibrated cv")
    n_between, n_mean = 25, 6
    with T.Context() as ctx:
        mid = ctx.ttcf_init_mother(gsys(T, s), sr[0], sp[0], n_equil=0)
        ctx.ttcf_import_states(mid, sr, sp)
        first = ctx.ttcf_spawn_daughters(mid, 16, 0, GD, N_OUT)
        ctx.ttcf_step(N_OUT)
        w32, net = seeded_net(N_OUT, seed=23)
        ctx.ttcf_cv_init(N_OUT, w32)
        ctx.ttcf_cv_add_training(first, 64)
        ctx.ttcf_cv_train(0, 64, 1e-3)
        ctx.ttcf_cv_attach(first, 32, T.TTCF_CV_CALIBRATE)
        ctx.ttcf_cv_attach(first + 32, 32, T.TTCF_CV_ESTIMATE)
        assert ctx.ttcf_accumulate() == 16
        beta = ctx.ttcf_cv_calibrate(N_OUT + 1, GD)
        ctx.ttcf_cv_mean_term(mid, 1, None, 0, 1, n_mean, n_between, GD)
        cm, cse, pm, pse, bmu, bmu_se, used = ctx.ttcf_cv_response(N_OUT + 1, GD)
    assert used == 8
    fo, b0, om = oracle_features(orc, box, s, sr, sp, range(16), GD)
    state_of = np.repeat(np.arange(16), 4)
    map_of = np.tile(np.arange(4), 16)
    vo, _ = orc.run_daughters(box, sr, sp, state_of, map_of, np.full(64, GD), s.dt, N_OUT,
                              nthreads=8)
    fo32 = fo.astype(np.float32).astype(np.float64)
    xmu, xinv = col_stats32(fo32)
    ymu, yinv = col_stats32((vo[:, 1:] / s.volume).astype(np.float32).astype(np.float64))
    hn = oracle_h(net, fo32, xmu, xinv, ymu, yinv, b0, om, s.dt).reshape(16, 4, -1).mean(axis=1)
    g_n = orc.ttcf_response(vo / s.volume, vo[:, 0], np.full(64, GD), s.temperature, s.dt).g
    gc, hc = g_n[:8], hn[:8]
    cov = ((gc - gc.mean(axis=0)) * (hc - hc.mean(axis=0))).sum(axis=0)
    var = ((hc - hc.mean(axis=0)) ** 2).sum(axis=0)
    beta_ref = np.where(var > 0, cov / np.where(var > 0, var, 1.0), 0.0)
    assert beta[0] == 0.0 and beta_ref[0] == 0.0
    np.testing.assert_allclose(beta[1:], beta_ref[1:], rtol=2e-2, atol=2e-2)
    st = orc.NHState(sr[0].copy(), sp[0].copy())
    mr, mp = orc.mother_sample(box, st, 0, n_mean, n_between, s.temperature, s.dt,
                               orc.nh_q(s.nf, s.temperature, TAU), s.nf)
    fm, b0m, omm = oracle_features(orc, box, s, mr, mp, range(n_mean), GD)
    mu_ref = oracle_h(net, fm.astype(np.float32).astype(np.float64), xmu, xinv, ymu, yinv, b0m,
                      omm, s.dt).reshape(n_mean, 4, -1).mean(axis=1).mean(axis=0)
    ge, he = g_n[8:], hn[8:]
    hscale = np.abs(he).max()
    close_plain = np.abs(pm - ge.mean(axis=0)).max() <= 1e-7 * np.abs(ge).max()
    assert close_plain
    np.testing.assert_allclose(bmu, beta_ref * mu_ref, atol=3e-2 * hscale)
    cv_ref = (ge - beta_ref * he).mean(axis=0) + beta_ref * mu_ref
    np.testing.assert_allclose(cm, cv_ref, atol=3e-2 * hscale)
    se_ref = (ge - beta_ref * he).std(axis=0, ddof=1) / np.sqrt(8)
    np.testing.assert_allclose(cse, se_ref, rtol=5e-2, atol=3e-2 * hscale)
