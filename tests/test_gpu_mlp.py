"""GPU learned binning: features, MLP forward/backward/Adam against the FP64
oracle, training on solver-logged iteration counts, and the queue order it
produces (results must not change; timings are reported)."""
import time

import numpy as np
import pytest

from oracle import features as OF
from oracle import mlp as OM
from synth import make_config, make_problem, mlp_init_weights, rngs_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B(gpu_lib):
    from paper_1402_7285_amd import binding
    return binding


def _plan(B, prob, **kw):
    P = B.Problem(prob.H, prob.S)
    extra = dict(out_ptr=prob.out_ptr, out_rows=prob.out_rows, tol=prob.tol)
    if prob.cluster_ptr is not None:
        extra.update(cluster_ptr=prob.cluster_ptr, cluster_atoms=prob.cluster_atoms)
    extra.update(kw)
    return P, B.Plan(P, prob.shifts, prob.rhs, **extra)


def test_features_match_oracle(B):
    for prob in (make_problem(lattice="fcc", L=4, bdim=9, hop=(0.0, 0.5), s_scale=0.03, K=4, nrhs=24,
                              radius=(1.0, 1.8), seed_key=(5, 6, 7)),
                 make_config(0)):
        P, plan = _plan(B, prob)
        g = plan.features().cpu().numpy().astype(np.float64)
        o = OF.all_features(prob)
        err = np.abs(g - o) / np.maximum(1.0, np.abs(o))
        assert err.max() < 1e-5, (prob.name, err.max(), np.unravel_index(err.argmax(), err.shape))


def _mlp_data(n=300, seed=3):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 16)).astype(np.float32)
    t = (np.tanh(X[:, 0]) + 0.3 * X[:, 2] * X[:, 3]).astype(np.float32)
    w = mlp_init_weights(rngs_for((7, 7, 7))["mlp_init"]).astype(np.float32)
    w[OM.NH * 16:OM.NH * 16 + OM.NH] = 0.05                      # nonzero b1 so ReLUs are mixed
    return X, t, w


def test_forward_and_gradient_match_oracle(B):
    import torch
    X, t, w = _mlp_data()
    Xd, td, wd = (torch.from_numpy(a).cuda() for a in (X, t, w))
    y = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
    B.scocg_mlp_forward(wd, Xd, y)
    yo, _ = OM.forward(w.astype(np.float64), X.astype(np.float64))
    assert np.abs(y.cpu().numpy() - yo).max() <= 1e-5 * max(1.0, np.abs(yo).max())
    work = torch.empty(B.scocg_mlp_work_floats(), dtype=torch.float32, device="cuda")
    grad = torch.empty(OM.NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    B.scocg_mlp_train_step(wd, None, None, Xd, td, None, 0.0, 1, loss, grad, work)
    Lo, go = OM.loss_and_grad(w.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    g = grad.cpu().numpy().astype(np.float64)
    assert abs(loss.item() - Lo) <= 1e-5 * Lo
    assert np.linalg.norm(g - go) <= 1e-5 * np.linalg.norm(go)
    assert np.abs(g - go).max() <= 1e-5 * np.abs(go).max()
    # determinism: the same step twice gives the same gradient bits
    grad2 = torch.empty_like(grad)
    B.scocg_mlp_train_step(wd, None, None, Xd, td, None, 0.0, 1, loss, grad2, work)
    assert torch.equal(grad, grad2)


def test_adam_steps_match_oracle(B):
    import torch
    X, t, w = _mlp_data(n=128)
    wd = torch.from_numpy(w.copy()).cuda()
    m = torch.zeros_like(wd)
    v = torch.zeros_like(wd)
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    work = torch.empty(B.scocg_mlp_work_floats(), dtype=torch.float32, device="cuda")
    wo, mo, vo = w.astype(np.float64), np.zeros(OM.NPARAM), np.zeros(OM.NPARAM)
    idx = torch.arange(0, 128, 2, dtype=torch.int32, device="cuda")
    for step in range(1, 4):
        B.scocg_mlp_train_step(wd, m, v, Xd, td, idx, 1e-3, step, None, None, work)
        _, go = OM.loss_and_grad(wo, X[::2].astype(np.float64), t[::2].astype(np.float64))
        wo, mo, vo = OM.adam_step(wo, mo, vo, go, 1e-3, step)
    assert np.abs(wd.cpu().numpy() - wo).max() < 2e-6


def test_learned_order_on_solver_logs(B):
    """Train on iteration counts the solver logs (scocg_mlp_train), let
    scocg_schedule order fresh RHS by their predicted cost, and check that
    order against the host sort of predicted iterations x block entries, and
    that every queue order leaves every result unchanged; report solve times
    of index order, by-size order, learned order and the order of the true
    costs."""
    import torch
    base = dict(lattice="fcc", L=5, bdim=9, hop=(0.0, 0.5), s_scale=0.03, K=16, eta=0.05, radius=(1.0, 2.2))
    train_p = make_problem(nrhs=192, seed_key=(21, 1, 1), **base)
    test_p = make_problem(nrhs=192, seed_key=(21, 2, 2), mats_key=(21, 1, 1), **base)
    P, plan = _plan(B, train_p, tol=1e-8)
    r = plan.solve()
    feats = plan.features().cpu().numpy()
    y = np.log(r["stats"][:, 0].astype(np.float64))
    rg = rngs_for((21, 1, 1))
    w0 = mlp_init_weights(rg["mlp_init"])
    model, best_val = B.scocg_mlp_train(feats, y, init_weights=w0, seed=21, epochs=150, batch=32, lr=3e-3)
    # the untrained network (same z-scoring) against the trained one, over all training samples
    untrained = model.copy()
    untrained[: w0.size] = w0
    mse0 = float(np.mean((B.scocg_mlp_predict(untrained, feats) - y) ** 2))
    mse1 = float(np.mean((B.scocg_mlp_predict(model, feats) - y) ** 2))
    print(f"[mlp] training MSE untrained {mse0:.3f} trained {mse1:.3f}, best validation {best_val:.3f}", flush=True)
    assert mse1 < 0.5 * mse0 and best_val < mse0
    Pt, plan_t = _plan(B, test_p, tol=1e-8)
    ref = plan_t.solve()
    ft = plan_t.features().cpu().numpy()
    pred = B.scocg_mlp_predict(model, ft).astype(np.float64)
    ent = ft[:, 0].astype(np.float64) * ft[:, 1].astype(np.float64)
    truth = ref["stats"][:, 0].astype(np.float64)
    corr = np.corrcoef(pred, np.log(truth))[0, 1]
    print(f"[mlp] correlation of predicted and true log iterations on fresh RHS: {corr:.3f}", flush=True)
    # the library's schedule is the stable decreasing sort of exp(pred) x entries
    order_l, cost_l = plan_t.schedule(model)
    np.testing.assert_allclose(cost_l, np.exp(pred) * ent, rtol=1e-5)
    assert np.all(np.diff(cost_l[order_l]) <= 0)
    assert np.array_equal(np.sort(order_l), np.arange(test_p.nrhs))
    order_s, cost_s = plan_t.schedule(None)
    assert np.array_equal(cost_s, ent.astype(np.float32))
    assert np.array_equal(order_s, np.argsort(-ent, kind="stable"))
    orders = {"index": None, "by_size": order_s, "learned": order_l,
              "true_cost": np.argsort(-(truth * ent), kind="stable").astype(np.int32)}
    times = {}
    Po, po = _plan(B, test_p, tol=1e-8, slots=24)
    for name, order in orders.items():
        po.set_order(order)
        bufs = po.alloc_outputs()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        po.run(bufs)
        torch.cuda.synchronize()
        times[name] = time.perf_counter() - t0
        out = bufs["out"].cpu().numpy()
        for j in range(test_p.nrhs):
            a, b_ = po.out_offsets[j] * test_p.nshift, po.out_offsets[j + 1] * test_p.nshift
            assert np.array_equal(out[a:b_].reshape(test_p.nshift, -1), ref["G"][j])
    print("[mlp] solve time by queue order (24 workgroups): "
          + ", ".join(f"{k} {v * 1e3:.1f} ms" for k, v in times.items()), flush=True)


def test_whole_training_run_and_prediction(B):
    """scocg_mlp_train / scocg_mlp_predict on host buffers: deterministic
    for a seed, learns the target, stores the feature standardisation, and
    predicts what the FP64 oracle network gives on the standardised input."""
    X, t, w = _mlp_data(n=600, seed=5)
    F = X * 3.0 + 1.0                                         # raw features: the model z-scores them
    kw = dict(epochs=120, batch=64, lr=3e-3, seed=11)
    model, vl = B.scocg_mlp_train(F, t, **kw)
    model2, vl2 = B.scocg_mlp_train(F, t, **kw)
    assert np.array_equal(model, model2) and vl == vl2
    NP = B.scocg_mlp_nparams()
    mu, sd = model[NP:NP + 16], model[NP + 16:]
    np.testing.assert_allclose(mu, F.astype(np.float64).mean(0), rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(sd, F.astype(np.float64).std(0), rtol=1e-5)
    y = B.scocg_mlp_predict(model, F)
    Z = (F.astype(np.float64) - mu) / sd
    yo, _ = OM.forward(model[:NP].astype(np.float64), Z)
    assert np.abs(y - yo).max() <= 1e-4 * max(1.0, np.abs(yo).max())
    corr = np.corrcoef(y, t)[0, 1]
    print(f"[mlp-train] validation MSE {vl:.4f} (target variance {np.var(t):.4f}), correlation {corr:.3f}",
          flush=True)
    assert vl < 0.5 * np.var(t) and corr > 0.8
    # given initial weights and a negligible step, the weights stay where they started
    m0, _ = B.scocg_mlp_train(F, t, init_weights=w, epochs=1, lr=1e-12, val_frac=0.0)
    assert np.abs(m0[:NP] - w).max() < 1e-6
