"""CPU oracle of the learned offspring pre-screen (DeepSets surrogate). TEST INFRASTRUCTURE ONLY.

The surrogate is an addition to the paper's method (it has no counterpart in
the paper): a small permutation-invariant network predicts ln(objective) of
a chromosome from its genes, and a screened GA generation breeds several
candidate children per cell, keeps the one the network scores lowest and
decodes only that one exactly (Section 4.3's decoder stays the judge of
every fitness). This module states what the GPU kernels compute, plainly:

  per-job features (integers first, then one rounding each to float32):
    tot_j   = sum over unfrozen stages s of min over machines of P_jsm
    slack_j = D_j - max(ready_j, RS) - tot_j
    rel_j   = max(ready_j - RS, 0)
    scale   = max(1, max_j tot_j);  f_j = fl32(x) / fl32(scale) for x in (tot, slack, rel)
    rank    = fl32(gene value) / fl32(n)            (gene values are 1..n)
  layer 1 (float32, this order, no fused multiply-add):
    c_j  = ((b1 + f0 * W1[1]) + f1 * W1[2]) + f2 * W1[3]
    a1   = c_j + rank * W1[0];   h1 = bf16(max(a1, 0))
  layer 2:   a2 = h1 . bf16(W2) + b2     (bf16 operands, exact products, summed)
             h2 = max(a2, 0)
  pool/out:  z = mean over the chromosome's jobs of h2;  y = z . w3 + b3
  target:    t = ln obj standardised within the chromosome's population
  loss:      L = mean over the batch of (y - t)^2

The forward keeps float32 exactly where the kernels do (features, layer 1,
the bf16 roundings) and sums layer 2, the pool and the output in float64;
`forward_bound` states how far float32 summation may move y. The backward
rounds the layer-2 output gradient to bf16 where it is a matrix-core operand,
as the kernels do. Parameters are float32 arrays; the flat layout is
[W1 (4 x H), b1 (H), W2 (H x H, row = input unit), b2 (H), w3 (H), b3 (1)].

Everything here is numpy; nothing is shared with or imported from the GPU
library.
"""
from __future__ import annotations

import numpy as np

H = 256
U32 = 2.0 ** -24          # unit roundoff of float32


def n_params(h: int = H) -> int:
    return 4 * h + h + h * h + h + h + 1


def unflatten(theta, h: int = H) -> dict:
    t = np.asarray(theta, dtype=np.float32).reshape(-1)
    assert t.size == n_params(h)
    o = 0
    out = {}
    for name, shape in (("W1", (4, h)), ("b1", (h,)), ("W2", (h, h)), ("b2", (h,)), ("w3", (h,)),
                        ("b3", (1,))):
        k = int(np.prod(shape))
        out[name] = t[o:o + k].reshape(shape).copy()
        o += k
    return out


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], np.float32).reshape(-1)
                           for k in ("W1", "b1", "W2", "b2", "w3", "b3")])


def bf16(x) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even); the
    result is returned as float32 holding the bfloat16 value."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    assert np.isfinite(a).all()
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).reshape(a.shape)


def job_features(inst) -> np.ndarray:
    """float32 [n_active, 3]: (tot, slack, rel) / scale of every active job, gene order."""
    g = int(inst.n_stages)
    om = int(inst.o_max)
    n_m = np.asarray(inst.n_machines)
    proc = np.asarray(inst.proc).reshape(-1, g, om)
    rs = int(inst.rs)
    act = np.asarray(inst.active).reshape(-1)
    tot = np.zeros(len(act), np.int64)
    slack = np.zeros(len(act), np.int64)
    rel = np.zeros(len(act), np.int64)
    for k, j in enumerate(act):
        f = int(np.asarray(inst.first_stage)[j])
        tot[k] = sum(int(proc[j, s, :n_m[s]].min()) for s in range(f, g))
        ready = int(np.asarray(inst.ready)[j])
        slack[k] = int(np.asarray(inst.due)[j]) - max(ready, rs) - tot[k]
        rel[k] = max(ready - rs, 0)
    scale = np.float32(max(1, int(tot.max()) if len(act) else 1))
    out = np.stack([tot, slack, rel], axis=1).astype(np.float32) / scale
    return out.astype(np.float32)


def rank_feature(prio, n: int) -> np.ndarray:
    return np.asarray(prio, dtype=np.float32) / np.float32(n)


def layer1(p: dict, feats, rank, exact: bool = False):
    """a1 [..., n, H] (float32 in the stated order; float64 when exact)."""
    if exact:
        W1 = p["W1"].astype(np.float64)
        c = p["b1"].astype(np.float64) + feats.astype(np.float64) @ W1[1:]
        return c[None] + rank.astype(np.float64)[..., None] * W1[0]
    W1 = p["W1"]
    c = p["b1"][None] + feats[:, 0:1] * W1[1][None]
    c = c + feats[:, 1:2] * W1[2][None]
    c = c + feats[:, 2:3] * W1[3][None]
    return c[None] + rank[..., None] * W1[0][None, None]


def forward(p: dict, feats, prio, exact: bool = False) -> dict:
    """y [B] and the intermediates for chromosomes prio [B, n] (int, gene values 1..n).

    exact=True drops every rounding (a plain float64 network) for the
    derivative and library pins."""
    prio = np.atleast_2d(np.asarray(prio))
    n = prio.shape[1]
    rank = prio.astype(np.float64) / n if exact else rank_feature(prio, n)
    a1 = layer1(p, feats, rank, exact)
    if exact:
        h1 = np.maximum(a1, 0.0)
        W2 = p["W2"].astype(np.float64)
    else:
        h1 = bf16(np.maximum(a1, np.float32(0))).astype(np.float64)
        W2 = bf16(p["W2"]).astype(np.float64)
    a2 = h1 @ W2 + p["b2"].astype(np.float64)
    h2 = np.maximum(a2, 0.0)
    z = h2.mean(axis=1)
    y = z @ p["w3"].astype(np.float64) + float(p["b3"][0])
    return {"prio": prio, "rank": rank, "a1": a1, "h1": h1, "a2": a2, "h2": h2, "z": z, "y": y,
            "W2": W2}


def _gamma(m):
    """gamma_m = m u / (1 - m u): |fl(sum of m+1 terms) - sum| <= gamma_m sum |terms|
    for any order of float32 additions (one rounding each)."""
    return m * U32 / (1 - m * U32)


def _a2_bound(p: dict, f: dict) -> np.ndarray:
    """|a2_float32 - a2| for layer 2 summed in float32 (exact bf16 products, bias added)."""
    h = f["h1"].shape[-1]
    abs_terms = np.abs(f["h1"]) @ np.abs(f["W2"]) + np.abs(p["b2"].astype(np.float64))
    return _gamma(h + 1) * abs_terms


def forward_bound(p: dict, f: dict, order: str = "pool") -> np.ndarray:
    """A bound on |y_float32 - y| per chromosome, layer 1 and the bf16 roundings
    being identical on both sides and every sum taken in float32 in any order.

    order "pool": z = (sum over jobs of h2) / n, then y = b3 + z . w3.
    order "row":  r_k = h2_k . w3 per job, then y = b3 + (sum over jobs of r_k) / n.
    Each product and the division by n add one rounding (u |value|)."""
    h = f["h1"].shape[-1]
    n = f["h1"].shape[1]
    e_a2 = _a2_bound(p, f)                               # ReLU is 1-Lipschitz
    w3 = np.abs(p["w3"].astype(np.float64))
    b3 = abs(float(p["b3"][0]))
    if order == "pool":
        zs = np.abs(f["h2"]).sum(axis=1)                 # sum over jobs, per unit
        e_z = (e_a2.sum(axis=1) + _gamma(n) * zs) / n + U32 * zs / n
        terms = np.abs(f["z"]) * w3
        return e_z @ w3 + (_gamma(h + 1) + U32) * (terms.sum(axis=1) + b3)
    if order == "row":
        rows = np.abs(f["h2"]) * w3                      # [B, n, h]
        e_r = e_a2 @ w3 + (_gamma(h) + U32) * rows.sum(axis=2)
        rs = np.abs(f["h2"] @ p["w3"].astype(np.float64))
        ssum = rs.sum(axis=1)
        e_s = e_r.sum(axis=1) + _gamma(n) * (ssum + e_r.sum(axis=1))
        return e_s / n + U32 * (ssum + e_s) / n + U32 * (ssum / n + b3 + e_s / n) * 2
    raise ValueError(order)


def loss_and_grad(p: dict, feats, prio, target, exact: bool = False):
    """L = mean (y - target)^2 over the batch and its gradient (dict like p, float64).

    The gradient is that of the network as evaluated by `forward` (with
    exact=False the bf16 roundings of h1 and W2 are part of the function and
    pass the gradient straight through), taken in float64 with nothing
    rounded. The kernels round the layer-2 output gradient to bf16 where it
    is a matrix-core operand; `grad_bound` states how far that and their
    float32 sums may move each entry."""
    f = forward(p, feats, prio, exact)
    y = f["y"]
    t = np.asarray(target, dtype=np.float64)
    B, n = f["h1"].shape[0], f["h1"].shape[1]
    L = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / B
    g = {}
    g["w3"] = dy @ f["z"]
    g["b3"] = np.array([dy.sum()])
    gz = dy[:, None] * p["w3"].astype(np.float64)[None] / n          # dL/dh2 of every row
    dA2 = np.where(f["a2"] > 0, gz[:, None, :], 0.0)
    g["b2"] = dA2.sum(axis=(0, 1))
    g["W2"] = np.einsum("bkh,bko->ho", f["h1"], dA2)
    dH1 = dA2 @ f["W2"].T
    dA1 = np.where(f["a1"] > 0, dH1, 0.0)
    g["b1"] = dA1.sum(axis=(0, 1))
    x = np.concatenate([f["rank"].astype(np.float64)[..., None],
                        np.broadcast_to(feats.astype(np.float64)[None], (B, n, 3))], axis=2)
    g["W1"] = np.einsum("bkf,bkh->fh", x, dA1)
    f.update({"dy": dy, "dA2": dA2, "dA1": dA1, "x": x, "target": t})
    return L, g, f


def grad_bound(p: dict, f: dict) -> dict:
    """Elementwise bounds on |g_gpu - g| for the kernels' evaluation of the
    gradient of `loss_and_grad` (f is its third result):

      y in float32, pool order (forward_bound); t = fl32(ln obj);
      dy_b = 2 (y_b - t_b) / B;  D_q = sum of dy_b over the chromosomes b
      whose gene for job k has value v, q = (k, v);  the layer-2 output
      gradient of table row q is G_q = mask(a2_q > 0) * fl(D_q * w3 / n),
      rounded to bf16 (unit roundoff 2^-8) as a matrix-core operand;
      dW2 = sum_q h1_q^T bf16(G_q), dH1_q = bf16(G_q) bf16(W2)^T,
      dA1 = mask(a1 > 0) * dH1, db1/dW1/db2/dw3/db3 the matching sums,
      every sum in float32 in any order.

    A layer-2 mask entry whose a2 lies within its float32 error of zero may
    differ between the two sides; such entries contribute their whole value
    to the bound. Layer 1 is bit-identical on both sides, so its mask is too."""
    ub = 2.0 ** -8
    B, n, h = f["h1"].shape
    w3 = p["w3"].astype(np.float64)
    aw3 = np.abs(w3)
    e_y = forward_bound(p, f, "pool")
    t = f["target"]
    dy = f["dy"]
    e_dy = 2.0 * (e_y + U32 * np.abs(t)) / B + 2 * U32 * np.abs(dy)
    out = {}
    out["b3"] = np.array([e_dy.sum() + _gamma(B) * np.abs(dy).sum()])
    zs = np.abs(f["h2"]).sum(axis=1)
    e_z = (_a2_bound(p, f).sum(axis=1) + _gamma(n) * zs) / n + U32 * zs / n
    out["w3"] = (e_dy @ np.abs(f["z"]) + np.abs(dy) @ e_z
                 + (_gamma(B) + U32) * (np.abs(dy) @ np.abs(f["z"])))
    # the table rows (k, v) the batch touches, with D_q and its bound
    q = np.arange(n)[None, :] * n + (np.asarray(f["prio"], np.int64) - 1)   # [B, n]
    D = np.zeros(n * n)
    Dabs = np.zeros(n * n)
    eD = np.zeros(n * n)
    np.add.at(D, q.reshape(-1), np.repeat(dy, n))
    np.add.at(Dabs, q.reshape(-1), np.repeat(np.abs(dy), n))
    np.add.at(eD, q.reshape(-1), np.repeat(e_dy, n))
    eD += _gamma(B) * Dabs
    used = Dabs > 0
    # per touched row: h1, a2, a2 bound, G and its bound (with uncertain masks)
    first = np.full(n * n, -1)
    rows_b, rows_k = np.nonzero(np.ones((B, n), bool))
    first[q[rows_b, rows_k]] = rows_b * n + rows_k
    idx = first[used]
    h1 = f["h1"].reshape(B * n, h)[idx]
    a2 = f["a2"].reshape(B * n, h)[idx]
    a1 = f["a1"].reshape(B * n, h)[idx]
    x = f["x"].reshape(B * n, 4)[idx]
    e_a2 = _a2_bound(p, f).reshape(B * n, h)[idx]
    Dq, eDq = D[used][:, None], eD[used][:, None]
    G = np.where(a2 > 0, Dq * w3[None] / n, 0.0)
    Gmax = (np.abs(Dq) + eDq) * aw3[None] / n
    unsure = np.abs(a2) <= e_a2
    e_G = np.where(unsure, Gmax + np.abs(G), (eDq * aw3[None] / n) + 2 * U32 * np.abs(G))
    Gabs = np.abs(G) + e_G
    e_Gb = e_G + ub * Gabs                                         # after the bf16 rounding
    Q = len(idx)
    out["b2"] = e_G.sum(axis=0) + _gamma(Q) * Gabs.sum(axis=0)
    out["W2"] = np.abs(h1).T @ e_Gb + _gamma(Q) * (np.abs(h1).T @ (Gabs + e_Gb))
    W2 = f["W2"]
    e_dH1 = e_Gb @ np.abs(W2).T + _gamma(h) * ((Gabs + e_Gb) @ np.abs(W2).T)
    m1 = (a1 > 0).astype(np.float64)
    dH1abs = (Gabs + e_Gb) @ np.abs(W2).T
    out["b1"] = (m1 * e_dH1).sum(axis=0) + _gamma(Q) * (m1 * dH1abs).sum(axis=0)
    out["W1"] = np.abs(x).T @ (m1 * e_dH1) + (_gamma(Q) + U32) * (np.abs(x).T @ (m1 * dH1abs))
    return out


def targets(obj, group: int) -> np.ndarray:
    """Training targets, float64: ln obj standardised within each group of `group`
    consecutive entries (mean and population standard deviation; 0 where the
    deviation is 0)."""
    lo = np.log(np.asarray(obj, np.float64))
    out = np.zeros_like(lo)
    for g0 in range(0, len(lo), group):
        x = lo[g0:g0 + group]
        sd = x.std()
        out[g0:g0 + group] = (x - x.mean()) / sd if sd > 0 else 0.0
    return out


def adam(theta, m, v, grad, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), float64. Returns (theta, m, v)."""
    th = np.asarray(theta, np.float64)
    gr = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * gr
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * gr * gr
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return th - lr * mh / (np.sqrt(vh) + eps), m, v


def screen(scores) -> np.ndarray:
    """Per cell, the candidate with the lowest score; ties go to the lowest variant.
    scores [V, pop] -> int [pop]."""
    s = np.asarray(scores)
    return np.argmin(s, axis=0)


def screened_generation(inst, ga, seed, shop, event, gen, state, p: dict, variants: int = 4,
                        n_threads: int = 1):
    """One screened generation: `variants` candidate children per cell (the
    breeding of variant v draws from block v), scored by the network, the
    lowest-scored kept per cell and decoded exactly, then replacement and
    migration as in a plain generation. Returns (new state, candidates
    [V, pop, n], scores [V, pop], choice [pop])."""
    import oracle
    cands = np.stack([oracle.ga_breed(inst, ga, seed, shop, event, gen, v, state)
                      for v in range(variants)])
    feats = job_features(inst)
    scores = np.stack([forward(p, feats, c)["y"] for c in cands])
    choice = screen(scores)
    pop = cands.shape[1]
    children = cands[choice, np.arange(pop)]
    new = oracle.ga_finish(inst, ga, gen, children, state, n_threads=n_threads)
    return new, cands, scores, choice
