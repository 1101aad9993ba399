"""Learned corrections of the optimal 4th-kind weights (orchestration of the C ABI).

beta[p, l] = beta_opt(k) + MLP(features[p, l])  for stacked problem p, smoothing level l,
trained to minimise the residual reduction of two V-cycle iterations,
    loss = mean_p ||r_2,p|| / ||r_0,p||,
with the library's hand-written adjoint (amg_train_loss_grad) and its MLP
forward / backward / Adam kernels.  A predicted weight row whose polynomial
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
    plain_loss: float = 0.0
    invalid_rows: int = 0


def _tables(torch, h, degree, nbatch):
    L = B.amg_num_levels(h)
    base = torch.tensor(B.amg_default_beta(degree), dtype=torch.float64, device="cuda")
    return L, base.repeat(nbatch * L).reshape(nbatch, L, degree).contiguous()


def predict_beta(h, params, feats, degree, nbatch):
    """beta [nbatch, nlevels, degree] float64 with fallback to the table for rows outside Pi_k,
    the MLP cache (for backward) and the validity mask [nbatch * (nlevels - 1)]."""
    import torch
    L, base = _tables(torch, h, degree, nbatch)
    NL = L - 1
    rows = feats.shape[0]
    y = torch.empty((rows, 6), dtype=torch.float32, device="cuda")
    cache = torch.empty((rows, 128), dtype=torch.float32, device="cuda")
    B.mlp_fwd(params, feats, y, cache)
    beta = base.clone()
    delta = y[:, :degree].to(torch.float64).reshape(nbatch, NL, degree)
    beta[:, :NL, :] += delta
    valid = B.amg_beta_valid(beta[:, :NL, :].contiguous().reshape(-1), degree)
    vmask = valid.reshape(nbatch, NL, 1).to(torch.bool)
    beta[:, :NL, :] = torch.where(vmask, beta[:, :NL, :], base[:, :NL, :])
    return beta.contiguous(), cache, valid


def evaluate(h, beta, b, degree, nbatch):
    import torch
    g = torch.empty_like(beta)
    loss, ratios = B.amg_train_loss_grad(h, degree, beta, b, g, nbatch)
    return loss, ratios


def train(h, b, sigmas, degree=6, steps=100, lr=1e-3, init_params=None, log=None):
    """Train the network on the stacked problems of handle h (right-hand side b, one sigma per problem)."""
    import torch
    nbatch = len(sigmas)
    L, base = _tables(torch, h, degree, nbatch)
    NL = L - 1
    feats = B.amg_level_features(h, degree, sigmas)
    n = B.mlp_num_params()
    params = torch.as_tensor(init_params, dtype=torch.float32).to("cuda").contiguous()
    assert params.numel() == n
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    gp = torch.empty_like(params)
    work = torch.empty(2 * feats.shape[0] * 64, dtype=torch.float32, device="cuda")
    gbeta = torch.empty_like(base)
    res = TrainResult(params=params)
    res.plain_loss, _ = evaluate(h, base, b, degree, nbatch)
    for step in range(1, steps + 1):
        beta, cache, valid = predict_beta(h, params, feats, degree, nbatch)
        loss, _ = B.amg_train_loss_grad(h, degree, beta, b, gbeta, nbatch)
        res.losses.append(loss)
        # d loss / d y = d loss / d beta on the smoothing levels (zero where the row fell back)
        gy = torch.zeros((feats.shape[0], 6), dtype=torch.float32, device="cuda")
        gy[:, :degree] = (gbeta[:, :NL, :].reshape(-1, degree) * valid.reshape(-1, 1).to(torch.float64)).to(
            torch.float32)
        B.mlp_bwd(params, feats, cache, gy, gp, work)
        B.mlp_adam(params, gp, m, v, step, lr)
        res.invalid_rows = int((valid == 0).sum().item())
        if log is not None and (step == 1 or step % 10 == 0):
            log(f"step {step} loss {loss:.6f} (plain {res.plain_loss:.6f}) invalid rows {res.invalid_rows}")
    return res


def learned_level_betas(h, params, degree, sigma):
    """Per-level weights of a single-problem handle from the trained network (fallback applied)."""
    import torch
    feats = B.amg_level_features(h, degree, [sigma])
    beta, _, _ = predict_beta(h, params, feats, degree, 1)
    L = B.amg_num_levels(h)
    return [beta[0, l].tolist() for l in range(L - 1)]


def apply_level_betas(h, degree, level_betas):
    for l, bl in enumerate(level_betas):
        B.amg_set_beta(h, degree, l, bl)
