"""Learned corrections of the optimal 4th-kind weights (orchestration of the C ABI).

beta[p, l] = beta_opt(k) + MLP(features[p, l])  for stacked problem p, smoothing level l,
trained to minimise the residual reduction of two V-cycle iterations,
    loss = mean_p ||r_2,p|| / ||r_0,p||,
with the library's hand-written adjoint (amg_train_loss_grad), its MLP
forward / backward / Adam kernels and its weight composition and fallback
(amg_learned_beta, amg_learned_beta_grad).  A predicted weight row whose polynomial
leaves Pi_k (|p| >= 1 somewhere on (0, 1], eq. polspace) falls back to the
tabulated weights; the caller can also keep the tabulated weights when the
network does not lower the loss (the plain optimal-beta smoother is both the
fallback and the yardstick of the network's benefit).

Everything numerical runs in the library's kernels; this module only
allocates device tensors and sequences the calls.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from . import _binding as B


@dataclass
class TrainResult:
    params: "object"               # float32 device tensor [5126]
    losses: list = field(default_factory=list)
    plain_loss: float = 0.0           # loss of the tabulated weights on the (first) training set
    invalid_rows: int = 0             # rows of the last step that fell back to the table
    plain_loss_per_set: list = field(default_factory=list)
    final_loss_per_set: list = field(default_factory=list)


def predict_beta(h, params, feats, degree, nbatch):
    """beta [nbatch, nlevels, degree] float64 with fallback to the table for rows outside Pi_k,
    the MLP cache (for backward) and the validity mask [nbatch * (nlevels - 1)]."""
    import torch
    rows = feats.shape[0]
    y = torch.empty((rows, 6), dtype=torch.float32, device="cuda")
    cache = torch.empty((rows, 128), dtype=torch.float32, device="cuda")
    B.mlp_fwd(params, feats, y, cache)
    beta, valid = B.amg_learned_beta(h, degree, y, nbatch)
    return beta, cache, valid


def plain_beta(h, degree, nbatch):
    """The tabulated optimal weights on every (problem, level) row, layout of predict_beta."""
    beta, _ = B.amg_learned_beta(h, degree, None, nbatch)
    return beta


def evaluate(h, beta, b, degree, nbatch):
    import torch
    g = torch.empty_like(beta)
    loss, ratios = B.amg_train_loss_grad(h, degree, beta, b, g, nbatch)
    return loss, ratios


def count_fallbacks(valid):
    """Number of rows that fell back to the table (host-side count of the device mask)."""
    return valid.cpu().tolist().count(0)


def train(h, b, sigmas, degree=6, steps=100, lr=1e-3, init_params=None, log=None):
    """Train the network on the stacked problems of handle h (right-hand side b, one sigma per
    problem).  h, b and sigmas may also be lists of the same length (training sets of different
    operators or sizes): each Adam step then takes the gradient of one set, in turn."""
    import torch
    many = isinstance(h, (list, tuple))
    hs, bs, sgs = (list(h), list(b), list(sigmas)) if many else ([h], [b], [sigmas])
    n = B.mlp_num_params()
    params = torch.as_tensor(init_params, dtype=torch.float32).to("cuda").contiguous()
    assert params.numel() == n
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    gp = torch.empty_like(params)
    sets = []
    for hh, bb, sg in zip(hs, bs, sgs):
        nb = len(sg)
        feats = B.amg_level_features(hh, degree, sg)
        base = plain_beta(hh, degree, nb)
        st = {"h": hh, "b": bb, "nb": nb, "feats": feats, "gbeta": torch.empty_like(base),
              "gy": torch.empty((feats.shape[0], 6), dtype=torch.float32, device="cuda"),
              "work": torch.empty(2 * feats.shape[0] * 64, dtype=torch.float32, device="cuda")}
        st["plain"], _ = evaluate(hh, base, bb, degree, nb)
        sets.append(st)
    res = TrainResult(params=params)
    res.plain_loss = sets[0]["plain"]
    res.plain_loss_per_set = [st["plain"] for st in sets]
    valid = None
    for step in range(1, steps + 1):
        st = sets[(step - 1) % len(sets)]
        beta, cache, valid = predict_beta(st["h"], params, st["feats"], degree, st["nb"])
        loss, _ = B.amg_train_loss_grad(st["h"], degree, beta, st["b"], st["gbeta"], st["nb"])
        res.losses.append(loss)
        # d loss / d y = d loss / d beta on the kept rows of the smoothing levels, zero elsewhere
        B.amg_learned_beta_grad(st["h"], degree, st["gbeta"], valid, st["gy"])
        B.mlp_bwd(params, st["feats"], cache, st["gy"], gp, st["work"])
        B.mlp_adam(params, gp, m, v, step, lr)
        if log is not None and (step == 1 or step % 10 == 0):
            log(f"step {step} loss {loss:.6f} (plain {st['plain']:.6f}) fallback rows {count_fallbacks(valid)}")
    if valid is not None:
        res.invalid_rows = count_fallbacks(valid)
    res.final_loss_per_set = []
    for st in sets:
        beta, _, _ = predict_beta(st["h"], params, st["feats"], degree, st["nb"])
        res.final_loss_per_set.append(evaluate(st["h"], beta, st["b"], degree, st["nb"])[0])
    return res


def learned_level_betas(h, params, degree, sigma):
    """Per-level weights of a single-problem handle from the trained network (fallback applied)."""
    feats = B.amg_level_features(h, degree, [sigma])
    beta, _, _ = predict_beta(h, params, feats, degree, 1)
    L = B.amg_num_levels(h)
    tab = beta.cpu().tolist()[0]
    return [tab[l] for l in range(L - 1)]


def apply_level_betas(h, degree, level_betas):
    for l, bl in enumerate(level_betas):
        B.amg_set_beta(h, degree, l, bl)


def with_level_betas(table, level_betas):
    """A copy of the single-problem weight table [1, nlevels, degree] (device) whose smoothing
    rows are replaced by level_betas (host lists), e.g. to evaluate them with evaluate()."""
    import torch
    rows = table.cpu().tolist()[0]
    for l, bl in enumerate(level_betas):
        rows[l] = list(bl)
    return torch.tensor([rows], dtype=torch.float64, device="cuda")
