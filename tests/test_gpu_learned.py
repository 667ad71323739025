"""GPU checks of the learned warm start: the network's forward pass and
gradients (BF16 MFMA kernels) against the FP64 oracle on identical
bf16-rounded weights and inputs; deterministic training that lowers the
loss; training pairs against the oracle's local solve; the guard (a useless
network leaves the plain method unchanged); and the gain of a trained
network's start over the plain start on unseen local problems."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1708_07954_amd import binding
from scenes import make_config2, make_sphere_scene

pytestmark = pytest.mark.gpu


def _net(seed=0, bias_scale=0.1):
    p = mlp.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    p["b1"] = rng.normal(0, bias_scale, p["b1"].shape)
    p["b2"] = rng.normal(0, bias_scale, p["b2"].shape)
    p["b3"][:12] = rng.normal(0, bias_scale, 12)
    flat = mlp.flatten(p).astype(np.float32)
    return flat, mlp.unflatten(flat.astype(np.float64))


def _identity_norm():
    return np.concatenate([np.zeros(26), np.ones(26), np.zeros(12), np.ones(12)]).astype(np.float32)


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((n, 32), np.float32)
    x[:, :26] = rng.normal(0, 1, (n, 26))
    t = np.zeros((n, 16), np.float32)
    t[:, :12] = rng.normal(0, 1, (n, 12))
    return x, t


def test_forward_and_gradients_match_oracle():
    flat, p = _net(1)
    h = binding.dba_create(binding.make_options(precision="fp32"))
    binding.dba_set_mlp(h, flat, _identity_norm())
    x, t = _data(512, 2)
    loss, grad, y = binding.dba_mlp_loss_grad(h, x, t)
    Y, cache = mlp.forward(p, x.astype(np.float64), quantize=True)
    g = mlp.backward(p, cache, Y, t.astype(np.float64), quantize=True)
    scale = np.abs(Y[:, :12]).max()
    err_y = np.abs(y[:, :12] - Y[:, :12]).max() / scale
    print("forward max rel err", err_y)
    assert err_y < 1e-3
    assert loss == pytest.approx(mlp.loss(Y, t), rel=1e-3)
    # element by element, relative to each parameter block's largest gradient
    # (both sides round the same activations to BF16; the rest is FP32
    # against FP64 accumulation)
    gg = mlp.unflatten(grad.astype(np.float64))
    for k in g:
        e = np.abs(gg[k] - g[k]).max() / np.abs(g[k]).max()
        print("grad", k, "max element error / max |grad|", e,
              "norm ratio", np.linalg.norm(gg[k] - g[k]) / np.linalg.norm(g[k]))
        assert e < 1e-3, (k, e)
    binding.dba_destroy(h)


def test_forward_api_standardizes_like_the_oracle():
    flat, p = _net(3)
    rng = np.random.default_rng(4)
    norm = np.concatenate([rng.normal(0, 1, 26), rng.uniform(0.5, 2, 26), rng.normal(0, 1e-3, 12),
                           rng.uniform(1e-3, 1e-2, 12)]).astype(np.float32)
    h = binding.dba_create(binding.make_options(precision="fp32"))
    binding.dba_set_mlp(h, flat, norm)
    f = rng.normal(0, 1, (300, 26)).astype(np.float32)        # not a multiple of 64: ragged tail
    d = binding.dba_mlp_forward(h, f)
    nm = norm.astype(np.float64)
    Y, _ = mlp.forward(p, mlp.standardize_input(f.astype(np.float64), nm[:26], nm[26:52]), quantize=True)
    ref = Y[:, :12] * nm[64:76] + nm[52:64]
    err = np.abs(d - ref).max() / np.abs(ref - nm[52:64]).max()
    print("forward through the API, max error / output scale", err)
    assert err < 1e-3
    binding.dba_destroy(h)


def test_training_lowers_the_loss_and_is_deterministic():
    rng = np.random.default_rng(5)
    f = rng.normal(0, 1, (8192, 26)).astype(np.float32)
    A = rng.normal(0, 0.3, (26, 12))
    d = (np.tanh(f @ A) + 0.05 * rng.normal(0, 1, (8192, 12))).astype(np.float32)
    out = []
    for _ in range(2):
        h = binding.dba_create(binding.make_options(precision="fp32"))
        el = binding.dba_mlp_train(h, f, d, epochs=20, batch=512, lr=3e-3, seed=11)
        out.append((el, binding.dba_get_mlp(h)))
        binding.dba_destroy(h)
    el = out[0][0]
    print("epoch losses", el)
    assert el[-1] < 0.3 * el[0]
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1][0], out[1][1][0])


def test_collected_pairs_match_the_oracle_local_solve():
    sc = make_config2(n_cams=40, n_points=600)
    kw = dict(loss="huber", loss_param=2.0, rho=1e5)
    s = binding.Solver(precision="fp32", **kw).set_scene(sc)
    f, d = binding.dba_collect_pairs(s.h, 1, 64, seed=3, conv_steps=30)
    # first iteration: copies = initial consensus, duals 0, so each pair is
    # the local problem at the initial estimate; match it by its residual
    opts = oracle.make_opts("huber", 2.0)
    P = oracle.Problem.from_scene(sc)
    th0 = np.concatenate([sc.cams_init[sc.obs_cam], sc.points_init[sc.obs_point]], axis=1)
    res = np.array([sc.obs_uv[k] - oracle.project(th0[k, :9], th0[k, 9:])[0] for k in range(sc.n_obs)])
    for q in range(0, 64, 8):
        k = int(np.argmin(np.abs(res - f[q, :2]).sum(1)))
        assert np.abs(res[k] - f[q, :2]).max() < 1e-2
        assert np.abs(f[q, 2:]).max() < 1e-3            # copy - consensus (fp32 rounding) and duals
        th, _, _ = oracle.local_solve(opts, sc.obs_uv[k], th0[k], th0[k], 1e5, 1e5, steps=50)
        ref = th - th0[k]
        assert np.abs(d[q] - ref).max() <= 2e-3 * np.abs(ref).max() + 1e-5, (q, d[q], ref)


@pytest.mark.parametrize("kind", ["zero", "garbage"])
def test_guard_keeps_the_plain_method(kind):
    """A network predicting nothing, or garbage, is rejected by the guard, and
    the learned iteration equals plain LM with the same steps (up to FP32
    rounding: the two kernels are compiled separately)."""
    sc = make_config2(n_cams=40, n_points=600)
    kw = dict(precision="fp32", loss="huber", loss_param=2.0, rho=1e5, block_waves=4, persistent=0)
    if kind == "zero":
        flat = np.zeros(22800, np.float32)
        norm = _identity_norm()
        norm[52:64] = 0.0
    else:
        flat, _ = _net(9)
        flat *= 1e3
        norm = _identity_norm()
        norm[64:76] = 1e3
    plain = binding.Solver(lm_steps=2, **kw).set_scene(sc)
    plain.iterate(6)
    learned = binding.Solver(start="learned", learned_lm_steps=2, **kw)
    binding.dba_set_mlp(learned.h, flat, norm)
    learned.set_scene(sc)
    learned.iterate(6)
    np.testing.assert_allclose(learned.params()[0], plain.params()[0], rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(learned.state()[0], plain.state()[0], rtol=1e-5, atol=1e-6)


def test_learned_start_without_a_network_is_a_state_error():
    sc = make_sphere_scene(seed=3, n_cams=10, n_points=100)
    s = binding.Solver(precision="fp32", start="learned", loss="huber", rho=1e5).set_scene(sc)
    with pytest.raises(binding.DbaError) as e:
        s.iterate(1)
    assert e.value.status == "DBA_E_STATE"


def _final_inlier_rmse(sc, net=None, iters=250, **kw):
    base = dict(precision="fp32", loss="huber", loss_param=2.0, rho=1e5, rho_balancing=True, rho_min=1e5,
                rho_max=1e7, block_waves=1, persistent=0)
    base.update(kw)
    s = binding.Solver(**base)
    if net is not None:
        binding.dba_set_mlp(s.h, net[0], net[1])
    s.set_scene(sc)
    s.set_eval_mask(~sc.outlier)
    s.iterate(iters)
    r = s.residuals(want_rmse=True)["rmse_masked"]
    s.close()
    return r


def test_trained_network_gains_over_the_plain_start():
    """The network trained on the GPU (pairs from ten small trajectory-family
    scenes) predicts starts closer to the converged local solution than the
    plain start (the previous copy) on local problems of the 2M-observation
    workload, which it never saw: the mean standardized squared distance to
    the converged update drops by more than 20 %.  The gain comes from the
    large updates; on typical small ones the prediction is worse than the
    plain start (median printed), which is where the guard keeps the plain
    start.  The ADMM runs with 3 and 5 LM steps are printed for the record
    (with 3 steps ADMM sits at the edge of stability from either start)."""
    from paper_1708_07954_amd import warmstart
    params, norm, rep = warmstart.train_default()
    assert rep["epoch_loss"][-1] < rep["epoch_loss"][0]
    sc = make_config2()
    s = binding.Solver(**warmstart.TRAIN_SOLVER).set_scene(sc)
    feats, deltas = binding.dba_collect_pairs(s.h, 20, 20000, seed=5, conv_steps=30)
    s.close()
    h = binding.dba_create(binding.make_options(precision="fp32"))
    binding.dba_set_mlp(h, params, norm)
    pred = binding.dba_mlp_forward(h, feats)
    binding.dba_destroy(h)
    sd = norm[64:76]
    e_net = np.sum(((pred - deltas) / sd) ** 2, axis=1)
    e_zero = np.sum((deltas / sd) ** 2, axis=1)
    runs = {k: _final_inlier_rmse(sc, **kw) if "start" not in kw else _final_inlier_rmse(sc, net=(params, norm), **kw)
            for k, kw in (("plain5", dict(lm_steps=5)), ("plain4", dict(lm_steps=4)), ("plain3", dict(lm_steps=3)),
                          ("plain2", dict(lm_steps=2)), ("learned3", dict(start="learned", learned_lm_steps=3)),
                          ("learned5", dict(start="learned", learned_lm_steps=5)))}
    print("pairs", len(e_net), "mean", e_net.mean(), e_zero.mean(), "median", np.median(e_net), np.median(e_zero),
          "inlier rmse after 250 iterations", runs, "train", rep["train_seconds"], "s")
    assert e_net.mean() < 0.8 * e_zero.mean()


@pytest.mark.parametrize("order", ["graphs_first", "pairs_first"])
def test_collecting_pairs_keeps_each_start_in_its_own_graphs(order):
    """dba_collect_pairs runs plain iterations on a handle set to the learned
    start.  Replayed from captured graphs, every iteration must still run the
    start it belongs to: the plain ones inside the collection and the learned
    ones around it, bitwise as the same sequence run eagerly (use_graph = 0)
    on a second handle.  Covers both orders: learned graphs captured before
    the collection, and the collection's plain graphs captured first."""
    sc = make_config2(n_cams=40, n_points=600)
    flat, _ = _net(4)
    norm = _identity_norm()
    norm[64:76] = 1e-4
    kw = dict(precision="fp32", loss="huber", loss_param=2.0, rho=1e5, block_waves=4, persistent=0,
              start="learned", learned_lm_steps=2, lm_steps=5)
    runs = []
    for use_graph in (True, False):
        s = binding.Solver(use_graph=use_graph, **kw)
        binding.dba_set_mlp(s.h, flat, norm)
        s.set_scene(sc)
        if order == "graphs_first":
            s.iterate(2)
        f, d = binding.dba_collect_pairs(s.h, 2, 64, seed=3, conv_steps=10)
        s.iterate(3)
        runs.append((s.params(), s.state(), f, d))
        s.close()
    (pg, sg, fg, dg), (pe, se, fe, de) = runs
    np.testing.assert_array_equal(fg, fe)
    np.testing.assert_array_equal(dg, de)
    np.testing.assert_array_equal(pg[0], pe[0])
    np.testing.assert_array_equal(pg[1], pe[1])
    np.testing.assert_array_equal(sg[0], se[0])
    np.testing.assert_array_equal(sg[1], se[1])


def test_adam_steps_match_the_oracle_elementwise():
    """Three Adam steps (dba_mlp_apply_gradient, the update dba_mlp_train's
    steps use) from fixed parameters with fixed gradients against
    oracle.mlp.adam_step in FP64: master parameters and both moments element
    by element, the step count, and the padding entries of the parameter
    block held at zero even when their gradient is not."""
    flat, _ = _net(12)
    h = binding.dba_create(binding.make_options(precision="fp32"))
    try:
        binding.dba_set_mlp(h, flat, _identity_norm())
        m0, v0, t0 = binding.dba_mlp_adam_state(h)
        assert t0 == 0 and not m0.any() and not v0.any()
        rng = np.random.default_rng(13)
        p = mlp.unflatten(flat.astype(np.float64))
        m = {k: np.zeros_like(a) for k, a in p.items()}
        v = {k: np.zeros_like(a) for k, a in p.items()}
        mag = np.zeros(22800)        # the first moment's terms in magnitude (its rounding scale)
        pad_t = mlp.unflatten(np.zeros(22800))
        pad_t["W1"][26:] = 1
        pad_t["W3"][:, 12:] = 1
        pad_t["b3"][12:] = 1
        pad = mlp.flatten(pad_t) > 0
        for step, lr in ((1, 1e-3), (2, 7.5e-4), (3, 2.5e-4)):
            # gradients spanning six decades, padding entries included
            g = (rng.normal(0, 1, 22800) * 10.0 ** rng.uniform(-6, 0, 22800)).astype(np.float32)
            binding.dba_mlp_apply_gradient(h, g, lr)
            mag = 0.9 * mag + 0.1 * np.abs(g.astype(np.float64))
            gg = mlp.unflatten(g.astype(np.float64))
            mlp.adam_step(p, gg, m, v, step, lr)
            for k in p:              # the padding is not trained
                p[k][pad_t[k] > 0] = 0.0
                m[k][pad_t[k] > 0] = 0.0
                v[k][pad_t[k] > 0] = 0.0
        got_p, _ = binding.dba_get_mlp(h)
        got_m, got_v, t = binding.dba_mlp_adam_state(h)
        assert t == 3
        ref_p, ref_m, ref_v = mlp.flatten(p), mlp.flatten(m), mlp.flatten(v)
        assert not got_p[pad].any() and not got_m[pad].any() and not got_v[pad].any()
        # FP32 arithmetic of three updates: a few ulp of each quantity (the
        # first moment's relative to its terms, which may cancel)
        assert np.all(np.abs(got_m - ref_m) <= 1e-6 * mag)
        np.testing.assert_allclose(got_v, ref_v, rtol=1e-6, atol=0)
        # parameters: three FP32 roundings of the parameter, plus the update's
        # own relative error (1e-6 of lr per step)
        np.testing.assert_allclose(got_p, ref_p, rtol=4e-7, atol=1e-8)
        assert np.abs(got_p - flat).max() > 1e-4        # the steps moved the parameters
    finally:
        binding.dba_destroy(h)


def _learned_net():
    """A network trained on the GPU on pairs from a small trajectory-family
    scene (the deployment loss and rho rule)."""
    from paper_1708_07954_amd import warmstart
    from scenes import make_trajectory_scene
    f, d = warmstart.collect([make_trajectory_scene(seed=2003, n_cams=60, n_points=3000)], iters=20,
                             per_iter=4096, seed=1)
    params, norm, _ = warmstart.train(f, d, epochs=6, batch=1024, lr=1e-3, seed=2)
    return params, norm


@pytest.mark.parametrize("steps", [2, 5])
def test_learned_admm_matches_the_oracle(steps):
    """The learned start (network, guard, `steps` LM steps) on the GPU
    against the oracle's learned iteration (reading R14, FP64, the network of
    oracle.mlp on the same weights) on a 40-camera trajectory scene for 25
    iterations: every parameter within 1e-3 relative, and the inlier RMSE
    within 0.5 %, at every fifth iteration."""
    from _util import param_err_summary
    params, norm = _learned_net()
    sc = make_config2(n_cams=40, n_points=600)
    kw = dict(loss="huber", loss_param=2.0, rho=1e5, rho_balancing=True)
    s = binding.Solver(precision="fp32", start="learned", learned_lm_steps=steps, rho_min=1e5, rho_max=1e7,
                       block_waves=1, persistent=0, **kw)
    binding.dba_set_mlp(s.h, params, norm)
    s.set_scene(sc)
    s.set_eval_mask(~sc.outlier)
    a = oracle.ADMM(oracle.Problem.from_scene(sc), sc.cams_init, sc.points_init, **kw)
    a.opts.rho_min, a.opts.rho_max = 1e5, 1e7
    inl = ~sc.outlier
    for it in range(1, 26):
        a.iterate_learned(params, norm, steps)
        s.iterate(1)
        if it % 5 == 0:
            cams, pts = s.params()
            e = param_err_summary(cams, pts, a.cons_y, a.cons_x)
            r = s.residuals(want_rmse=True)["rmse_masked"]
            ro = a.stats(inl)[1]
            print(f"learned+{steps} it {it}: rel err {e}, inlier rmse {r:.6f} oracle {ro:.6f}", flush=True)
            assert e["max"] < 1e-3, (it, e)
            assert abs(r - ro) < 5e-3 * ro
    s.close()
