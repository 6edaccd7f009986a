"""Pins of the surrogate oracle against things other than itself: PyTorch's own
bfloat16 conversion, autograd and Adam, central finite differences, the
DeepSets symmetry, float32 summation in several orders (for the stated bound),
a hand-computed feature example, and the screened generation's reduction to
the plain one."""
import numpy as np
import pytest
import torch

import oracle
from oracle import surrogate as S
from paper_1903_10741_amd import workloads as W

H = 32      # narrow network for the derivative pins; the layout is the same at 256


def _model(seed, h=H, scale=1.0):
    p = S.unflatten(W.surrogate_init(seed, h), h)
    rng = np.random.default_rng(seed + 99)
    for k in ("b1", "b2"):                       # non-zero biases so every term is exercised
        p[k] = (rng.normal(size=p[k].shape) * 0.1 * scale).astype(np.float32)
    p["b3"] = np.array([0.3], np.float32)
    return p


def _case(seed=1, n=9, B=5):
    inst = W.random_instance(seed, n_jobs=n, n_stages=3, machines=[2, 3, 2], p_max=30)
    feats = S.job_features(inst)
    prio = W.random_population(seed, B, n)
    return inst, feats, prio


def test_bf16_matches_torch_round_to_nearest_even():
    rng = np.random.default_rng(0)
    x = (rng.normal(size=5000) * 10.0 ** rng.integers(-8, 8, size=5000)).astype(np.float32)
    u = x.view(np.uint32)
    ties = ((u & 0xFFFF0000) | 0x8000).view(np.float32)      # exact halfway cases
    near = ((u & 0xFFFF0000) | 0x7FFF).view(np.float32)
    for v in (x, ties, near, np.array([0.0, -0.0, 1.0, -3.5], np.float32)):
        want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float32).numpy()
        assert (S.bf16(v).view(np.uint32) == want.view(np.uint32)).all()


def test_exact_forward_matches_torch_network():
    inst, feats, prio = _case()
    p = _model(3)
    f = S.forward(p, feats, prio, exact=True)
    t = {k: torch.from_numpy(np.asarray(v, np.float64)) for k, v in p.items()}
    n = prio.shape[1]
    x = torch.cat([torch.from_numpy(prio.astype(np.float64) / n)[..., None],
                   torch.from_numpy(feats.astype(np.float64))[None].expand(prio.shape[0], -1, -1)],
                  dim=2)
    h1 = torch.relu(x @ t["W1"] + t["b1"])
    h2 = torch.relu(h1 @ t["W2"] + t["b2"])
    y = h2.mean(dim=1) @ t["w3"] + t["b3"]
    assert np.allclose(f["y"], y.numpy(), rtol=1e-12, atol=1e-12)


def test_exact_gradient_matches_autograd():
    inst, feats, prio = _case(2, n=7, B=4)
    p = _model(5)
    tgt = np.log(np.random.default_rng(1).integers(100, 10000, size=4))
    L, g, _ = S.loss_and_grad(p, feats, prio, tgt, exact=True)
    t = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True) for k, v in p.items()}
    n = prio.shape[1]
    x = torch.cat([torch.from_numpy(prio.astype(np.float64) / n)[..., None],
                   torch.from_numpy(feats.astype(np.float64))[None].expand(4, -1, -1)], dim=2)
    y = torch.relu(torch.relu(x @ t["W1"] + t["b1"]) @ t["W2"] + t["b2"]).mean(dim=1) @ t["w3"] + t["b3"]
    loss = ((y - torch.from_numpy(tgt)) ** 2).mean()
    loss.backward()
    assert abs(L - loss.item()) < 1e-12
    for k in p:
        assert np.allclose(g[k].reshape(-1), t[k].grad.numpy().reshape(-1), rtol=1e-10, atol=1e-12), k


def test_exact_gradient_matches_finite_differences():
    inst, feats, prio = _case(4, n=6, B=3)
    p = _model(7)
    tgt = np.array([5.0, 6.0, 7.5])
    _, g, _ = S.loss_and_grad(p, feats, prio, tgt, exact=True)
    rng = np.random.default_rng(3)
    for k in ("W1", "b1", "W2", "b2", "w3", "b3"):
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            def L_at(delta):
                q = {kk: vv.astype(np.float64).copy() for kk, vv in p.items()}
                q[k].reshape(-1)[idx] += delta
                return S.loss_and_grad(q, feats, prio, tgt, exact=True)[0]
            eps = 1e-6
            fd = (L_at(eps) - L_at(-eps)) / (2 * eps)
            assert abs(fd - g[k].reshape(-1)[idx]) < 1e-6 * (1 + abs(fd)), (k, idx)


def test_rounded_gradient_is_close_to_exact():
    """The bf16 roundings move the gradient by a bf16-sized relative amount, no more."""
    inst, feats, prio = _case(6, n=12, B=6)
    p = _model(8)
    tgt = np.full(6, 4.0)
    _, g, _ = S.loss_and_grad(p, feats, prio, tgt)
    _, ge, _ = S.loss_and_grad(p, feats, prio, tgt, exact=True)
    for k in g:
        rel = np.linalg.norm(g[k] - ge[k]) / max(np.linalg.norm(ge[k]), 1e-30)
        assert rel < 2 ** -5, (k, rel)


def test_adam_matches_torch_optimizer():
    rng = np.random.default_rng(11)
    theta = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(4)]
    t = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([t], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    th = theta.copy()
    for s, gr in enumerate(grads, start=1):
        t.grad = torch.from_numpy(gr.copy())
        opt.step()
        th, m, v = S.adam(th, m, v, gr, s, 3e-3)
        assert np.allclose(th, t.detach().numpy(), rtol=1e-12, atol=1e-15)
    # first step closed form: lr * g / (|g| + eps)
    th1, _, _ = S.adam(theta, np.zeros(50), np.zeros(50), grads[0], 1, 1e-3)
    assert np.allclose(theta - th1, 1e-3 * grads[0] / (np.abs(grads[0]) + 1e-8), rtol=1e-12)


def test_permutation_invariance():
    """Permuting jobs together with their genes and features leaves y unchanged."""
    inst, feats, prio = _case(9, n=10, B=4)
    p = _model(2)
    perm = np.random.default_rng(5).permutation(10)
    for exact in (True, False):
        y0 = S.forward(p, feats, prio, exact)["y"]
        y1 = S.forward(p, feats[perm], prio[:, perm], exact)["y"]
        assert np.allclose(y0, y1, rtol=1e-13, atol=1e-13)


def test_forward_bound_covers_float32_summation_orders():
    inst, feats, prio = _case(12, n=40, B=6)
    p = S.unflatten(W.surrogate_init(4), S.H)
    p["b2"] = np.random.default_rng(1).normal(size=S.H).astype(np.float32) * 0.05
    f = S.forward(p, feats, prio)
    bound = S.forward_bound(p, f)
    h1 = f["h1"].astype(np.float32)
    W2 = f["W2"].astype(np.float32)
    for order in (np.arange(S.H), np.arange(S.H)[::-1], np.random.default_rng(2).permutation(S.H)):
        acc = np.zeros(f["a2"].shape, np.float32)
        for k in order:                                  # one float32 rounding per addition
            acc = acc + h1[:, :, k:k + 1] * W2[k][None, None]
        a2 = acc + p["b2"]
        h2 = np.maximum(a2, np.float32(0))
        z = np.zeros(h2.shape[::2], np.float32)
        for r in range(h2.shape[1]):
            z = z + h2[:, r]
        z = z / np.float32(h2.shape[1])
        y = np.float32(p["b3"][0]) + np.zeros(z.shape[0], np.float32)
        for k in order:
            y = y + z[:, k] * p["w3"][k]
        err = np.abs(y.astype(np.float64) - f["y"])
        assert (err <= bound).all(), (err.max(), bound.min())
    assert (bound < 1e-3 * np.abs(f["y"]) + 1e-3).all()


def test_job_features_by_hand():
    """Two stages, machines (2, 1); jobs: P = [[4,6],[5]] and [[3,9],[2]]; due 20, 7."""
    proc = np.array([[[4, 6], [5, 1]], [[3, 9], [2, 1]]], np.int32)
    inst = W.initial_instance(proc, np.ones_like(proc), np.zeros(2), np.array([20, 7]),
                              np.array([2, 1]), 5, 10)
    f = S.job_features(inst)
    # tot = (4 + 5, 3 + 2) = (9, 5); slack = (20 - 9, 7 - 5) = (11, 2); rel = 0; scale 9
    want = np.array([[9, 11, 0], [5, 2, 0]], np.float32) / np.float32(9)
    assert (f == want).all()
    # a later event: job 0 frozen through stage 0, ready 12 at RS 10
    inst.rs, inst.first_stage, inst.ready = 10, np.array([1, 0], np.int32), np.array([12, 0], np.int32)
    f = S.job_features(inst)
    # job 0: tot 5, slack 20 - 12 - 5 = 3, rel 2; job 1: tot 5, slack 7 - 10 - 5 = -8, rel 0; scale 5
    assert (f == np.array([[5, 3, 2], [5, -8, 0]], np.float32) / np.float32(5)).all()


def test_screen_ties_go_to_lowest_variant():
    s = np.array([[1.0, 2.0, 3.0], [1.0, 1.5, 3.0], [0.5, 1.5, 3.0]])
    assert list(S.screen(s)) == [2, 1, 0]


def test_screened_generation_with_one_variant_is_plain():
    inst = W.random_instance(21, n_jobs=11, n_stages=3, machines=2)
    ga = W.GaParams(2, 2, 4, mig_interval=2, mig_k=1)
    p = S.unflatten(W.surrogate_init(1), S.H)
    st = oracle.ga_init(inst, ga, 3, 1, 0)
    for gen in (1, 2):
        plain = oracle.ga_generation(inst, ga, 3, 1, 0, gen, st)
        scr, cands, scores, choice = S.screened_generation(inst, ga, 3, 1, 0, gen, st, p, variants=1)
        assert (choice == 0).all()
        for k in plain:
            assert (plain[k] == scr[k]).all()
        st = plain
    # with four variants, variant 0 is the plain generation's child
    _, cands, scores, choice = S.screened_generation(inst, ga, 3, 1, 0, 3, st, p, variants=4)
    assert (cands[0] == oracle.ga_breed(inst, ga, 3, 1, 0, 3, 0, st)).all()
    assert cands.shape == (4, ga.pop, 11) and scores.shape == (4, ga.pop)
    assert (scores[choice, np.arange(ga.pop)] == scores.min(axis=0)).all()


def _f32_sum(terms, axis, order):
    """Sum along `axis` in float32, one rounding per addition, in index order `order`."""
    t = np.moveaxis(np.asarray(terms, np.float32), axis, 0)
    acc = np.zeros(t.shape[1:], np.float32)
    for i in order:
        acc = acc + t[i]
    return acc


def test_forward_bound_covers_row_order():
    inst, feats, prio = _case(13, n=30, B=5)
    p = S.unflatten(W.surrogate_init(6), S.H)
    p["b2"] = np.random.default_rng(3).normal(size=S.H).astype(np.float32) * 0.05
    f = S.forward(p, feats, prio)
    bound = S.forward_bound(p, f, "row")
    h2 = np.maximum(f["a2"], 0).astype(np.float32)          # a2 rounded once to float32
    for rev in (False, True):
        o_ord = np.arange(S.H)[::-1] if rev else np.arange(S.H)
        k_ord = np.arange(30)[::-1] if rev else np.arange(30)
        r = _f32_sum(h2 * p["w3"][None, None], 2, o_ord)      # per-row dot with w3
        y = np.float32(p["b3"][0]) + _f32_sum(r, 1, k_ord) / np.float32(30)
        assert (np.abs(y.astype(np.float64) - f["y"]) <= bound).all()


def test_grad_bound_covers_float32_table_evaluation():
    """Evaluate the gradient the way the kernels do (aggregated (job, rank) table,
    bf16 layer-2 gradient operand, float32 sums) and check every entry against
    the oracle's float64 gradient within grad_bound."""
    rng = np.random.default_rng(17)
    n, B = 9, 64
    inst = W.random_instance(17, n_jobs=n, n_stages=3, machines=2, p_max=30)
    feats = S.job_features(inst)
    prio = W.random_population(17, B, n)
    p = S.unflatten(W.surrogate_init(9), S.H)
    p["b1"] = rng.normal(size=S.H).astype(np.float32) * 0.1
    p["b2"] = rng.normal(size=S.H).astype(np.float32) * 0.05
    tgt = rng.uniform(11.0, 13.0, size=B)
    L, g, f = S.loss_and_grad(p, feats, prio, tgt)
    bnd = S.grad_bound(p, f)
    # float32 evaluation in table form
    f32 = np.float32
    Q = n * n
    kk, vv = np.divmod(np.arange(Q), n)
    rank = (vv + 1).astype(f32) / f32(n)
    a1 = (((p["b1"][None] + feats[kk, 0:1] * p["W1"][1][None]) + feats[kk, 1:2] * p["W1"][2][None])
          + feats[kk, 2:3] * p["W1"][3][None]) + rank[:, None] * p["W1"][0][None]
    h1 = S.bf16(np.maximum(a1, f32(0)))
    W2b = S.bf16(p["W2"])
    a2 = _f32_sum(h1[:, :, None] * W2b[None], 1, range(S.H)) + p["b2"][None]
    h2 = np.maximum(a2, f32(0))
    qi = np.arange(n)[None, :] * n + (prio - 1)
    z = _f32_sum(h2[qi], 1, range(n)) / f32(n)                       # [B, H]
    y = f32(p["b3"][0]) + _f32_sum(z * p["w3"][None], 1, range(S.H))
    t32 = tgt.astype(f32)
    dy = f32(2) * (y - t32) / f32(B)
    D = np.zeros(Q, f32)
    for b in range(B):
        for k in range(n):
            D[qi[b, k]] = D[qi[b, k]] + dy[b]
    G = np.where(a2 > 0, (D[:, None] * p["w3"][None]) / f32(n), f32(0)).astype(f32)
    Gb = S.bf16(G)
    gpu = {"b3": np.array([_f32_sum(dy, 0, range(B))]),
           "w3": _f32_sum(dy[:, None] * z, 0, range(B)),
           "b2": _f32_sum(G, 0, range(Q)),
           "W2": _f32_sum(h1[:, :, None] * Gb[:, None, :], 0, range(Q))}
    dH1 = _f32_sum(Gb[:, None, :] * W2b[None], 2, range(S.H))
    dA1 = np.where(a1 > 0, dH1, f32(0))
    x = np.concatenate([rank[:, None], feats[kk]], axis=1).astype(f32)
    gpu["b1"] = _f32_sum(dA1, 0, range(Q))
    gpu["W1"] = _f32_sum(x[:, :, None] * dA1[:, None, :], 0, range(Q))
    for k in g:
        err = np.abs(gpu[k].astype(np.float64).reshape(g[k].shape) - g[k])
        assert (err <= bnd[k] + 1e-30).all(), (k, float((err - bnd[k]).max()))
        rel = np.linalg.norm(err) / max(np.linalg.norm(g[k]), 1e-30)
        assert rel < 2 ** -6, (k, rel)          # the bound is tight enough to mean something


def test_targets_are_per_group_zscores_of_ln_obj():
    from scipy import stats
    rng = np.random.default_rng(4)
    obj = rng.integers(1000, 900000, size=1000)
    t = S.targets(obj, 250)
    for g in range(4):
        seg = slice(250 * g, 250 * (g + 1))
        assert np.allclose(t[seg], stats.zscore(np.log(obj[seg].astype(np.float64))), atol=1e-12)
        assert np.array_equal(np.argsort(t[seg], kind="stable"), np.argsort(obj[seg], kind="stable"))
    assert (S.targets(np.full(5, 77), 5) == 0).all()
    short = S.targets(obj[:10], 4)                      # last group of 2
    assert np.allclose(short[8:], [-1.0, 1.0]) or np.allclose(short[8:], [1.0, -1.0])
