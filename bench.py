"""Benchmark: AMG-PCG on the 27-point trilinear-FE Laplacian at 320^3 (one MI355X).

Workload (the largest configuration, 32.8M rows, 879M stored entries): A x = b
with b uniform(-1, 1) from a seed, solved to ||r|| <= 1e-8 ||b|| from x = 0 by
CG preconditioned with the V-cycle of the 2x2x2 box-aggregation hierarchy
(320^3 -> 10^3, six levels, dense coarsest solve), smoothed by the optimal
4th-kind polynomial of degree 4, all in FP64, on a hierarchy already resident
in HBM (setup excluded, reported separately).  A step is one such solve.

value        = bytes one solve must move in the storage layouts the kernels use
               (summed from the per-kernel models below over the launches of one
               solve) / the solve's wall time, GB/s;
roofline     = the fine-level fused recurrence step (k_fused<double,0,true,true,1,true>):
               the bytes it must move per launch / its average duration, timed
               here with events on the launch stream (degree-5 minus degree-4
               and degree-7 minus degree-6 smoother applications from x = 0,
               each one such step); beside it
               the per-step figure of the CSR byte model (12 nnz + 60 n), and
               the measured ceiling of this GPU (the library's plain read and
               copy kernels);
cpu_baseline = the FP64 CPU oracle applying the same smoother (degree 4, from
               x = 0) to the fine level once, on one host thread, in GB/s of
               the same byte model; its result is compared with the GPU's;
variants     = time to 1e-8 of the other three variants of this workload (FP32
               hierarchy inside FP64 CG, learned weights, optimal 1st kind),
               of the remaining smoother kinds, optionally (--variants ...,zeros)
               of the same operator with its stored zero entries eliminated (a
               21-point pattern: the same iterates, bitwise), and the
               FP32-against-FP64 comparison on the 256^3 variable-coefficient
               diffusion problem (with its fine
               level's fused step); beside them the learned-weights
               configuration (32 stacked 64^3 diffusion problems, degree 6):
               training and held-out solves, plain against learned.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Smoother HBM GB/s (% peak); AMG-PCG time to 1e-8 residual, learned/FP32 vs plain"
PEAK_HBM = 8000.0  # GB/s, MI355X HBM3E
KIND_NAMES = {0: "l1jacobi", 1: "cheb4", 2: "optcheb4", 3: "optcheb1"}
FUSED_PROLONG_MAX_ROWS = 1 << 20  # box levels up to this size carry the prolongation in the smoother
STREAM_MIN_BLOCKS = 12288  # levels above this many 256-row blocks take the streaming kernels
WIDE_MIN_STEPS = 24  # streaming offset-aligned levels with this many stored steps per row take wide batches


# ---------------------------------------------------------------------------
# Byte models: the bytes each kernel must move in the layout it reads (values of w bytes,
# int32 indices, gathered vectors counted once).  M is the matrix's bytes in its layout:
# offset-aligned slices w per stored entry plus a 4-byte offset per 64, packed slices w + 4.
# ---------------------------------------------------------------------------
def matrix_bytes(amg, h, level, w):
    padded, _, aligned = amg.amg_level_layout(h, level)
    return padded * w + 4 * (padded // 64) if aligned else padded * (w + 4)


def level_table(amg, h, w):
    """[(n, M, lanes, R)] for every level of handle h, with values of w bytes; R is the bytes of the
    restriction product's slices (0 when the level restricts its residual instead)."""
    out = []
    L = amg.amg_num_levels(h)
    for l in range(L):
        n, _ = amg.amg_level_info(h, l)
        R = 0
        if l < L - 1:
            form, stored = amg.amg_level_transfer(h, l)
            if form == amg.AMG_TRANSFER_PRODUCT:
                R = stored * w + 4 * (stored // 64)
        out.append((n, matrix_bytes(amg, h, l, w), amg.amg_level_layout(h, l)[1], R))
    return out


def fused_bytes(n, M, w, store, xupd=True):
    # reads minv, the gathered direction, r (and x); writes r and the new direction (store), x (xupd)
    return M + (3 + (2 if store else 0) + (2 if xupd else 0)) * w * n


def loop_bytes(n, M, w, steps, pending):
    """The fused steps after an application's first kernel: x is brought up to date on every other
    step and on the last one (a step that finds no update pending leaves x alone)."""
    tot = 0
    for s in range(steps):
        last = s == steps - 1
        defer = not last and not pending
        tot += fused_bytes(n, M, w, not last, not defer)
        pending = defer
    return tot


def smooth_bytes(n, M, w, kind, k, from_zero, nc=0, prol=0):
    """One smoother application of degree k; prol: 0 none, 1 carried by the first two kernels."""
    if kind == 0:
        if from_zero:
            return 3 * w * n + (k - 1) * (M + 4 * w * n)
        return k * (M + 4 * w * n) + (2 * w * n if k % 2 else 0)
    if from_zero:
        if k == 1:
            return 3 * w * n
        tot = M + (5 if k > 2 else 3) * w * n  # steps 1 and 2 merged (reads minv, b; writes x, r, g)
        return tot + loop_bytes(n, M, w, k - 2, False)
    tot = M + 5 * w * n  # first step on x: reads b, x, minv; writes r, g (its x update is deferred)
    if prol:
        tot += 8 * n + 2 * w * nc  # aggregate index and coarse value, in the first two kernels
    if k == 1:
        return tot + 3 * w * n
    return tot + loop_bytes(n, M, w, k - 1, True)


def vcycle_bytes(levels, w, kind, k, nbatch=1):
    tot = 0
    for l, (n, M, lanes, R) in enumerate(levels[:-1]):
        nc = levels[l + 1][0]
        tot += smooth_bytes(n, M, w, kind, k, True)
        if R:  # b_c = P^T b - R x: R, b and x once, the children, b_c
            tot += R + 2 * w * n + 32 * nc + w * nc
        elif n > FUSED_PROLONG_MAX_ROWS:  # residual, then restriction over 8 children
            tot += M + 3 * w * n + w * n + 32 * nc + w * nc
        else:
            tot += M + 2 * w * n + 32 * nc + w * nc
        fused = kind != 0 and lanes == 1 and n <= FUSED_PROLONG_MAX_ROWS
        if not fused:
            tot += 2 * w * n + 4 * n + w * nc
        tot += smooth_bytes(n, M, w, kind, k, False, nc, 1 if fused else 0)
    nL = levels[-1][0] // nbatch
    nb = (nL + 63) // 64
    # coarsest: the packed lower 64 x 64 tiles of the inverse once, the tile partials written and read
    tot += nbatch * (nb * (nb + 1) // 2 * 64 * 64 * 8 + 2 * nb * nb * 64 * 8) + 2 * w * levels[-1][0]
    return tot


def solve_bytes(levels, M0_64, w, kind, k, iters, flexible, u_path=False):
    """One PCG solve from x = 0: b checks and copies, then per iteration the CG product with the
    direction update and the previous iteration's x += alpha p (not in the first), the r update,
    one V-cycle (FP32: with the casts) and its dot products; the last x += alpha p after the loop.
    u_path: the r update also writes u = M^-1 r (reading M^-1), which the V-cycle's merged first
    two steps read in place of the gathered M^-1 and r (large 27-point FP64 fine levels).
    Hierarchies with a degree of at least 2 and more than one level take the dot products of z
    inside the V-cycle's last kernel, which then reads r (and r_old) but not z again."""
    n = levels[0][0]
    wz = w  # the CG kernels read the hierarchy's own output
    vc = vcycle_bytes(levels, w, kind, k) + (12 * n if w == 4 else 0)
    dots = (8 + wz) * n + (8 * n if flexible else 0)
    if kind != 0 and k >= 2 and len(levels) > 1:
        dots -= wz * n
    per_it = (M0_64 + (24 + wz + 16) * n) + (24 + (8 if flexible else 0)) * n + vc + dots
    if u_path:
        per_it += 24 * n
    return 48 * n - 16 * n + iters * per_it + 24 * n


def csr_model_step(nnz, n):
    """The per-step figure of the CSR model: 12 bytes per stored entry plus 60 per row."""
    return 12 * nnz + 60 * n


def cpu_description():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


# ---------------------------------------------------------------------------
# helpers on the GPU
# ---------------------------------------------------------------------------
def progress(msg):
    """One line on stderr per finished part of the run (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def event_time(stream, fn, reps):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        out = fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, out


def fused_step_time(amg, h, kind, bd, xs, stream, reps=10, apply=None):
    """Average duration (ms) of the fine level's stored fused step that updates x, from smoother
    applications on level 0 from x = 0 timed with events on the launch stream.  x is updated on
    every other step, so degree 5 minus degree 4 and degree 7 minus degree 6 each add one such
    step (k_fused<...> in a kernel trace; the steps between them, which leave x alone, are
    k_fused_keep_x).  apply: the smoother entry (smoother_apply, or smoother_apply_f32 with
    float32 vectors on an FP32 hierarchy)."""
    apply = apply or amg.smoother_apply

    def time_apply(k):
        for _ in range(2):
            apply(h, 0, kind, k, bd, xs, True)
        t, _ = event_time(stream, lambda: apply(h, 0, kind, k, bd, xs, True), reps)
        return t

    t4, t5, t6, t7 = (time_apply(k) for k in (4, 5, 6, 7))
    return ((t5 - t4) + (t7 - t6)) / 2.0


def true_relres(amg, h, bd, x):
    """||b - A x|| / ||b|| with the library's level-0 product (a check, not part of the path)."""
    import torch
    y = torch.empty_like(x)
    amg.amg_spmv(h, 0, x, y)
    torch.cuda.synchronize()
    return float(torch.linalg.norm(bd - y) / torch.linalg.norm(bd))


def rel_to(x, ref):
    """||x - ref|| / ||ref||: a variant's solution against the FP64 headline solve's."""
    import torch
    return float(torch.linalg.norm(x - ref) / torch.linalg.norm(ref))


def ceiling(amg, stream):
    """Plain read and copy of this GPU through the library's bandwidth kernels (16-byte
    nontemporal accesses): a 4 GiB read, a 2 GiB -> 2 GiB copy."""
    import torch
    x = torch.ones(1 << 29, dtype=torch.float64, device="cuda")
    part = torch.empty(amg.AMG_HBM_PARTIALS, dtype=torch.float64, device="cuda")
    amg.amg_hbm_read(x, part)
    t_read, _ = event_time(stream, lambda: amg.amg_hbm_read(x, part), 10)
    half = x.numel() // 2
    src, dst = x[:half], x[half:]
    amg.amg_hbm_copy(src, dst)
    t_copy, _ = event_time(stream, lambda: amg.amg_hbm_copy(src, dst), 10)
    torch.cuda.synchronize()
    out = {"read_GBps": round(x.numel() * 8 / (t_read * 1e-3) / 1e9, 1),
           "copy_GBps": round(2 * half * 8 / (t_copy * 1e-3) / 1e9, 1),
           "kernels": "amg_hbm_read (4 GiB), amg_hbm_copy (2 GiB to 2 GiB)"}
    del x, part
    return out


# ---------------------------------------------------------------------------
# learned weights on the 27-point family
# ---------------------------------------------------------------------------
def train_learned(args, amg, W):
    """Train the 8-64-64-6 network (FP32, the library's adjoint and network kernels) on the
    27-point family (stacks of 40^3 and 80^3 problems) and on stacked 64^3 diffusion problems,
    Adam steps alternating between the three sets; report the loss of the plain and the
    learned weights on each set and on held-out problems (a 160^3 27-point problem and 32
    further diffusion problems)."""
    import torch

    from paper_2407_09848_amd import learned
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    deg = args.degree
    t0 = time.perf_counter()

    def stack(mats, seed, prec=amg.AMG_FP32):
        big = W.stack_block_diagonal(mats)
        h = amg.amg_setup(dev(big.row_ptr), dev(big.col), dev(big.val), big.grid[0], big.grid[1],
                          big.grid[2] // len(mats), len(mats), 4096, prec)
        return h, dev(W.rhs_uniform(big.n, seed))

    sets = []
    q40 = stack([W.q1_27pt(40)] * 8, W.SEED_RHS + 50)
    q80 = stack([W.q1_27pt(80)] * 2, W.SEED_RHS + 51)
    sig = W.config4_sigmas(32)
    diff = [W.fv_diffusion(np.exp(sig[p] * W.gaussian_random_field((64,) * 3, 8.0, W.SEED_GRF + p)))
            for p in range(32)]
    dh = stack(diff, W.SEED_RHS + 4)
    sets = [(q40, [0.0] * 8), (q80, [0.0] * 2), (dh, list(sig))]
    setup_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = learned.train([s[0][0] for s in sets], [s[0][1] for s in sets], [s[1] for s in sets], degree=deg,
                        steps=args.train_steps, lr=3e-3, init_params=W.mlp_init(W.SEED_MLP))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    out = {"degree": deg, "train_steps": args.train_steps, "setup_s": round(setup_s, 2),
           "train_s": round(train_s, 2), "invalid_rows_last_step": res.invalid_rows,
           "train_sets": {name: {"loss_plain": round(p, 6), "loss_learned": round(f, 6)}
                          for name, p, f in zip(("q1_27pt_8x40^3", "q1_27pt_2x80^3", "diffusion_32x64^3"),
                                                res.plain_loss_per_set, res.final_loss_per_set)}}
    for (h, _), _s in sets:
        amg.amg_destroy(h)
    # held out: a 160^3 27-point problem, 32 further diffusion problems
    held = {}
    h160, b160 = stack([W.q1_27pt(160)], W.SEED_RHS + 52, amg.AMG_FP64)
    held["q1_27pt_160^3"] = heldout_loss(amg, learned, h160, b160, res.params, deg, [0.0])
    amg.amg_destroy(h160)
    diff2 = [W.fv_diffusion(np.exp(sig[p] * W.gaussian_random_field((64,) * 3, 8.0, W.SEED_GRF + 500 + p)))
             for p in range(32)]
    hd2, bd2 = stack(diff2, W.SEED_RHS + 40)
    held["diffusion_32x64^3"] = heldout_loss(amg, learned, hd2, bd2, res.params, deg, list(sig))
    amg.amg_destroy(hd2)
    out["heldout"] = held
    return res.params, out


def heldout_loss(amg, learned, h, b, params, deg, sigmas):
    f = amg.amg_level_features(h, deg, sigmas)
    beta, _, valid = learned.predict_beta(h, params, f, deg, len(sigmas))
    lp, _ = learned.evaluate(h, learned.plain_beta(h, deg, len(sigmas)), b, deg, len(sigmas))
    ll, _ = learned.evaluate(h, beta, b, deg, len(sigmas))
    return {"loss_plain": round(lp, 6), "loss_learned": round(ll, 6), "fallback_rows": learned.count_fallbacks(valid)}


def learned_variant(args, amg, W, h, bd, x, stream, params, x_ref):
    """Apply the trained network per level to this hierarchy; the learned weights are kept
    when they lower the two-cycle residual ratio of this right-hand side (else the plain
    weights: the fallback); time the solve."""
    import torch

    from paper_2407_09848_amd import learned
    deg = args.degree
    lb = learned.learned_level_betas(h, params, deg, 0.0)
    plain = learned.plain_beta(h, deg, 1)
    r_learned, _ = learned.evaluate(h, learned.with_level_betas(plain, lb), bd, deg, 1)
    r_plain, _ = learned.evaluate(h, plain, bd, deg, 1)
    use = r_learned < r_plain
    if use:
        learned.apply_level_betas(h, deg, lb)
    amg.pcg_solve(h, args.kind, deg, bd, x, True, 1e-8, 1000)
    torch.cuda.synchronize()
    tm, (rc, itv, _, _) = event_time(stream, lambda: amg.pcg_solve(h, args.kind, deg, bd, x, True, 1e-8, 1000), 2)
    rr = true_relres(amg, h, bd, x)
    amg.amg_reset_beta(h)
    return {"ms": round(tm, 3), "iters": itv, "true_relres": rr, "vs_fp64_headline_solution": rel_to(x, x_ref),
            "weights": "learned" if use else "plain (fallback)",
            "two_cycle_ratio_plain": round(r_plain, 6), "two_cycle_ratio_learned": round(r_learned, 6),
            "level_betas": [[round(v, 6) for v in row] for row in lb]}


def c4_variant(args, amg, W, stream):
    """The learned-weights configuration at its own size and degree: 32 stacked 64^3 diffusion
    problems (sigma 0.5, 1, 2 in turn), optimal 4th kind of degree 6 on an FP32 hierarchy, the
    network trained through the adjoint of two V-cycles (Adam); then three held-out problems
    (one per sigma, FP64 hierarchy) solved to 1e-8 with the plain and the learned weights (the
    learned ones kept when they lower the problem's two-cycle ratio)."""
    import torch

    from paper_2407_09848_amd import learned
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    deg, P_ = 6, 32
    sig = W.config4_sigmas(P_)
    t0 = time.perf_counter()
    mats = [W.fv_diffusion(np.exp(sig[p] * W.gaussian_random_field((64,) * 3, 8.0, W.SEED_GRF + p)))
            for p in range(P_)]
    big = W.stack_block_diagonal(mats)
    h = amg.amg_setup(dev(big.row_ptr), dev(big.col), dev(big.val), big.grid[0], big.grid[1], big.grid[2] // P_,
                      P_, 4096, amg.AMG_FP32)
    b = dev(W.rhs_uniform(big.n, W.SEED_RHS + 4))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = learned.train(h, b, list(sig), degree=deg, steps=args.c4_steps, lr=3e-3, init_params=W.mlp_init(W.SEED_MLP))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    out = {"workload": "fv_diffusion_7pt_32x64^3_sigma_0.5_1_2", "degree": deg, "rows": int(big.n),
           "levels": amg.amg_num_levels(h), "setup_s": round(setup_s, 2),
           "train": {"steps": args.c4_steps, "s": round(train_s, 2),
                     "ms_per_step": round(train_s / max(args.c4_steps, 1) * 1e3, 2),
                     "loss_plain": round(res.plain_loss, 6), "loss_learned": round(res.final_loss_per_set[0], 6),
                     "invalid_rows_last_step": res.invalid_rows}}
    amg.amg_destroy(h)
    del mats, big
    held = {}
    for i, s in enumerate((0.5, 1.0, 2.0)):
        A = W.fv_diffusion(np.exp(s * W.gaussian_random_field((64,) * 3, 8.0, W.SEED_GRF + 900 + i)))
        bh = dev(W.rhs_uniform(A.n, W.SEED_RHS + 60 + i))
        hh = amg.amg_setup(dev(A.row_ptr), dev(A.col), dev(A.val), *A.grid, 1, 4096, amg.AMG_FP64)
        lb = learned.learned_level_betas(hh, res.params, deg, s)
        plain = learned.plain_beta(hh, deg, 1)
        r_l, _ = learned.evaluate(hh, learned.with_level_betas(plain, lb), bh, deg, 1)
        r_p, _ = learned.evaluate(hh, plain, bh, deg, 1)
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")

        def timed():
            amg.pcg_solve(hh, 2, deg, bh, x, True, 1e-8, 1000)
            torch.cuda.synchronize()
            tm, (_, itv, _, _) = event_time(stream, lambda: amg.pcg_solve(hh, 2, deg, bh, x, True, 1e-8, 1000), 5)
            return tm, itv

        t_p, it_p = timed()
        use = r_l < r_p
        if use:
            learned.apply_level_betas(hh, deg, lb)
        t_l, it_l = timed()
        amg.amg_reset_beta(hh)
        held[f"sigma_{s}"] = {"two_cycle_ratio_plain": round(r_p, 6), "two_cycle_ratio_learned": round(r_l, 6),
                              "weights": "learned" if use else "plain (fallback)",
                              "plain_ms": round(t_p, 3), "plain_iters": it_p, "learned_ms": round(t_l, 3),
                              "learned_iters": it_l, "learned_vs_plain": round(t_l / t_p, 3)}
        amg.amg_destroy(hh)
    out["heldout_solves"] = held
    return out


def c3_variant(amg, W, stream):
    """The 256^3 variable-coefficient diffusion problem (sigma = 1): FP64 and FP32 hierarchy,
    optimal 4th kind, k = 4, time to 1e-8 and the difference of the two solutions, and the
    FP64 fine level's fused step."""
    import torch
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    t0 = time.perf_counter()
    A, b, _ = W.config_problem(3)
    asm = time.perf_counter() - t0
    rp, cl, vl, bd = dev(A.row_ptr), dev(A.col), dev(A.val), dev(b)
    out = {"workload": "fv_diffusion_7pt_256^3_sigma1", "n": A.n, "nnz": A.nnz, "assembly_s": round(asm, 2)}
    xs = {}
    for prec, name in ((amg.AMG_FP64, "fp64"), (amg.AMG_FP32, "fp32")):
        t0 = time.perf_counter()
        h = amg.amg_setup(rp, cl, vl, *A.grid, 1, 4096, prec)
        torch.cuda.synchronize()
        st = time.perf_counter() - t0
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        flex = prec == amg.AMG_FP32
        amg.pcg_solve(h, 2, 4, bd, x, True, 1e-8, 1000, flex)
        tm, (rc, it, _, _) = event_time(stream, lambda: amg.pcg_solve(h, 2, 4, bd, x, True, 1e-8, 1000, flex), 3)
        out[name] = {"ms": round(tm, 3), "iters": it, "setup_s": round(st, 3),
                     "true_relres": true_relres(amg, h, bd, x)}
        if prec == amg.AMG_FP64:
            # the fine level's x-updating fused step on this 7-point level (the same kernel as the
            # headline's, 7 stored entries per row)
            n0 = amg.amg_level_info(h, 0)[0]
            M0 = matrix_bytes(amg, h, 0, 8)
            xw = torch.zeros(n0, dtype=torch.float64, device="cuda")
            t_step = fused_step_time(amg, h, 2, bd, xw, stream)
            step_bytes = fused_bytes(n0, M0, 8, True, True)
            achieved = step_bytes / (t_step * 1e-3) / 1e9
            out["fused_step"] = {"avg_launch_us": round(t_step * 1e3, 2), "bytes_per_launch": int(step_bytes),
                                 "GBps": round(achieved, 1), "frac_of_peak": round(achieved / PEAK_HBM, 4)}
            del xw
        xs[name] = x
        amg.amg_destroy(h)
    out["fp32_vs_fp64_time"] = round(out["fp32"]["ms"] / out["fp64"]["ms"], 3)
    out["fp32_vs_fp64_solution_relerr"] = float(torch.linalg.norm(xs["fp32"] - xs["fp64"]) /
                                                torch.linalg.norm(xs["fp64"]))
    return out


def cpu_baseline(args, A, b, x_gpu, gpu_apply_ms, apply_bytes):
    """The oracle's smoother application (optimal 4th kind, degree args.degree, from x = 0) on the
    fine level, one host thread; the l1 diagonal is computed beforehand and not timed."""
    from threadpoolctl import threadpool_limits

    from oracle import polynomials as P
    from oracle import smoothers as S
    model, ncpu = cpu_description()
    with threadpool_limits(limits=1):
        As = A.to_scipy()
        t0 = time.perf_counter()
        Minv = S.l1_diagonal(As)
        l1_s = time.perf_counter() - t0
        beta = P.optimal_beta(args.degree)[0] if args.kind == 2 else None
        a = P.a_star(args.degree) if args.kind == 3 else None
        t0 = time.perf_counter()
        xo = S.smooth(As, Minv, b, None, args.kind, args.degree, beta, a)
        cpu_s = time.perf_counter() - t0
    err = float(np.max(np.abs(x_gpu - xo)) / np.max(np.abs(xo)))
    return {"value": round(apply_bytes / cpu_s / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"one FP64 oracle application of the {KIND_NAMES[args.kind]} smoother of degree "
                      f"{args.degree} from x = 0 on the {A.grid[0]}^3 fine level ({A.n} rows; {cpu_s:.1f} s, "
                      f"scipy/numpy on one thread), GB/s of the same byte model as the GPU application",
            "apply_s": round(cpu_s, 3), "l1_diagonal_s_untimed": round(l1_s, 2), "host_cpu_model": model,
            "host_cpu_count": ncpu, "gpu_same_apply_ms": round(gpu_apply_ms, 3),
            "gpu_vs_oracle_max_abs_err_rel": err}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="q1_27pt", choices=("q1_27pt", "poisson_7pt", "fv_diffusion"),
                    help="the matrix: the 27-point Q1 Laplacian (the headline), the 7-point Poisson problem or "
                         "the variable-coefficient diffusion problem (sigma = 1)")
    ap.add_argument("--size", type=int, default=320)
    ap.add_argument("--kind", type=int, default=2)
    ap.add_argument("--degree", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--variants", default="fp32,learned,kinds,c3,c4",
                    help="comma-separated subset of the variants to time: fp32 (the FP32 hierarchy), learned "
                         "(the trained network's weights), kinds (the other smoother kinds), zeros (the 27-point "
                         "operator with its stored zero entries eliminated; not in the default run, whose kernel "
                         "trace would mix its fine level with the headline's), c3 (FP32 against FP64 on the 256^3 "
                         "diffusion problem), c4 (the network trained on 32 x 64^3 diffusion problems at degree "
                         "6, held-out solves); empty for none")
    ap.add_argument("--train-steps", type=int, default=150)
    ap.add_argument("--c4-steps", type=int, default=100,
                    help="Adam steps of the c4 variant (32 x 64^3 diffusion problems, degree 6)")
    ap.add_argument("--counter-sample", action="store_true",
                    help="setup, three smoother applications of degree 6 on the fine level and one 1 GiB copy "
                         "through the library's copy kernel, then exit (the program the HBM byte counters are "
                         "read on)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2407_09848_amd as amg
    import workloads as W

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    t0 = time.perf_counter()
    A, b, _ = W.config_problem({"q1_27pt": 5, "poisson_7pt": 2, "fv_diffusion": 3}[args.workload], size=args.size)
    assembly_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    rp, cl, vl, bd = dev(A.row_ptr), dev(A.col), dev(A.val), dev(b)
    torch.cuda.synchronize()
    upload_s = time.perf_counter() - t0
    free_before = torch.cuda.mem_get_info()[0]
    t0 = time.perf_counter()
    h = amg.amg_setup(rp, cl, vl, *A.grid, 1, 4096, amg.AMG_FP64)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    # device memory the handle holds (hierarchy, level-0 CSR copy, workspace), from the driver
    hierarchy_bytes = free_before - torch.cuda.mem_get_info()[0]
    n0, nnz0 = amg.amg_level_info(h, 0)
    x = torch.zeros(n0, dtype=torch.float64, device="cuda")

    if args.counter_sample:
        xs = torch.zeros(n0, dtype=torch.float64, device="cuda")
        for _ in range(3):
            amg.smoother_apply(h, 0, args.kind, 6, bd, xs, True)
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        amg.amg_hbm_copy(src, dst)
        torch.cuda.synchronize()
        amg.amg_destroy(h)
        print(json.dumps({"counter_sample": True, "n": n0, "copy_bytes_each_way": src.numel() * 8}), flush=True)
        return

    def solve(handle, kind, k, flexible=False):
        return amg.pcg_solve(handle, kind, k, bd, x, True, 1e-8, 1000, flexible)

    for _ in range(args.warmup):
        solve(h, args.kind, args.degree)
    torch.cuda.synchronize()
    ms, (rc, it, rel, _) = event_time(stream, lambda: solve(h, args.kind, args.degree), args.steps)
    # once more, untimed, for the residual history and the solution
    _, _, _, hist = amg.pcg_solve(h, args.kind, args.degree, bd, x, True, 1e-8, 1000, False, True)
    solve_info = {"iters": len(hist) - 1, "relres_history": [float(f"{v:.4e}") for v in hist],
                  "true_relres": true_relres(amg, h, bd, x)}
    x_head = x.clone()
    L = amg.amg_num_levels(h)
    lv64 = level_table(amg, h, 8)
    M0 = lv64[0][1]
    padded, lanes, aligned = amg.amg_level_layout(h, 0)
    streams = ((n0 + 255) // 256 + 7) // 8 * 8 > STREAM_MIN_BLOCKS
    # wide slices (at least 24 stored steps per row on average) take the wide-batch variant
    wide = streams and aligned and lanes == 1 and padded >= WIDE_MIN_STEPS * n0
    u_path = wide and args.kind != 0 and args.degree >= 2
    value = solve_bytes(lv64, M0, 8, args.kind, args.degree, it, False, u_path) / (ms * 1e-3) / 1e9

    progress(f"headline solves: {ms:.1f} ms, {it} iterations")
    # ---- the fine level's fused step ----
    xs = torch.zeros(n0, dtype=torch.float64, device="cuda")
    t_step = fused_step_time(amg, h, args.kind, bd, xs, stream)
    step_bytes = fused_bytes(n0, M0, 8, True, True)
    achieved = step_bytes / (t_step * 1e-3) / 1e9
    csr_bytes = csr_model_step(nnz0, n0)
    progress(f"fused step: {t_step * 1e3:.1f} us")
    ceil = ceiling(amg, stream)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM, 4), "traffic": None,
                "kernel": f"k_fused<double,0,true,{str(streams).lower()},1,{str(wide).lower()}> (fine level, "
                          f"{args.workload} {args.size}^3)",
                "bytes_per_launch": int(step_bytes), "avg_launch_us": round(t_step * 1e3, 2),
                "layout": {"stored_entries": int(padded), "lanes_per_row": lanes, "offset_aligned": aligned,
                           "bytes_per_launch": "8 per stored entry + 4 per 64 + 56 per row"},
                "csr_model": {"bytes_per_launch": int(csr_bytes), "formula": "12 nnz + 60 n",
                              "GBps": round(csr_bytes / (t_step * 1e-3) / 1e9, 1),
                              "note": "counts column indices and row pointers the offset-aligned layout "
                                      "does not read"},
                "ceiling": ceil, "frac_of_read_ceiling": round(achieved / ceil["read_GBps"], 4)}
    traffic = measured_traffic(args.size) if args.workload == "q1_27pt" else None
    if traffic is not None:
        roofline["traffic"] = traffic

    progress("ceiling and roofline done")
    # ---- variants ----
    chosen = {v for v in args.variants.split(",") if v}
    variants = {f"fp64_{KIND_NAMES[args.kind]}_k{args.degree}": {"ms": round(ms, 3), "iters": it}}
    base = ms

    def time_solve(handle, kind, k, flexible=False, reps=2):
        solve(handle, kind, k, flexible)
        torch.cuda.synchronize()
        tm, (rcv, itv, _, _) = event_time(stream, lambda: solve(handle, kind, k, flexible), reps)
        return tm, itv

    other_kinds = (3,) if args.kind != 3 else (2,)
    if "kinds" in chosen:
        other_kinds = tuple(kd for kd in (3, 1, 0) if kd != args.kind)
    for kind in other_kinds:
        tm, itv = time_solve(h, kind, args.degree)
        variants[f"fp64_{KIND_NAMES[kind]}_k{args.degree}"] = {"ms": round(tm, 3), "iters": itv,
                                                              "true_relres": true_relres(amg, h, bd, x),
                                                              "vs_fp64_headline_solution": rel_to(x, x_head)}
    progress("other smoother kinds done")
    if "fp32" in chosen:
        t0 = time.perf_counter()
        h32 = amg.amg_setup(rp, cl, vl, *A.grid, 1, 4096, amg.AMG_FP32)
        torch.cuda.synchronize()
        s32 = time.perf_counter() - t0
        tm, itv = time_solve(h32, args.kind, args.degree, flexible=True)
        variants[f"fp32_{KIND_NAMES[args.kind]}_k{args.degree}"] = {
            "ms": round(tm, 3), "iters": itv, "setup_s": round(s32, 3), "outer": "FP64 flexible CG",
            "true_relres": true_relres(amg, h, bd, x), "vs_fp64_headline_solution": rel_to(x, x_head)}
        # the FP32 hierarchy's fine-level fused step (k_fused<float,...>), timed as the headline's
        b32 = bd.float()
        x32 = torch.zeros(n0, dtype=torch.float32, device="cuda")
        t32 = fused_step_time(amg, h32, args.kind, b32, x32, stream, apply=amg.smoother_apply_f32)
        step32 = fused_bytes(n0, matrix_bytes(amg, h32, 0, 4), 4, True, True)
        variants[f"fp32_{KIND_NAMES[args.kind]}_k{args.degree}"]["fused_step"] = {
            "avg_launch_us": round(t32 * 1e3, 2), "bytes_per_launch": int(step32),
            "GBps": round(step32 / (t32 * 1e-3) / 1e9, 1), "frac_of_peak": round(step32 / (t32 * 1e-3) / 1e9 / PEAK_HBM, 4)}
        del b32, x32
        amg.amg_destroy(h32)
        progress("fp32 hierarchy done")
    if "zeros" in chosen and args.workload == "q1_27pt":
        # the same operator without its stored zero face entries (21-point pattern), as a caller
        # gets it by eliminating stored zeros: same hierarchy below the fine level, same iterates
        t0 = time.perf_counter()
        Bz = W.q1_27pt(args.size, store_zeros=False)
        asm_z = time.perf_counter() - t0
        rpz, clz, vlz = dev(Bz.row_ptr), dev(Bz.col), dev(Bz.val)
        hz = amg.amg_setup(rpz, clz, vlz, *Bz.grid, 1, 4096, amg.AMG_FP64)
        torch.cuda.synchronize()
        tm, itv = time_solve(hz, args.kind, args.degree)
        variants[f"fp64_{KIND_NAMES[args.kind]}_k{args.degree}_zeros_eliminated"] = {
            "ms": round(tm, 3), "iters": itv, "nnz": int(Bz.nnz), "assembly_s": round(asm_z, 2),
            "fine_level_stored_entries": int(amg.amg_level_layout(hz, 0)[0]),
            "solution_bitwise_equal": bool(torch.equal(x, x_head))}
        amg.amg_destroy(hz)
        del rpz, clz, vlz, Bz
        torch.cuda.empty_cache()
        progress("zeros eliminated done")
    learned_info = None
    if "learned" in chosen and args.kind == 2:
        params, learned_info = train_learned(args, amg, W)
        variants[f"learned_{KIND_NAMES[args.kind]}_k{args.degree}"] = learned_variant(args, amg, W, h, bd, x,
                                                                                    stream, params, x_head)
        progress("learned weights done")
    for v in variants.values():
        v["vs_plain_fp64"] = round(v["ms"] / base, 3)
    c3 = c3_variant(amg, W, stream) if "c3" in chosen else None
    if c3 is not None:
        progress("diffusion 256^3 done")
    c4 = c4_variant(args, amg, W, stream) if "c4" in chosen else None
    if c4 is not None:
        progress("learned 32 x 64^3 done")

    # ---- CPU baseline: the oracle's smoother application on the same fine level ----
    cpu = None
    if not args.no_cpu:
        xs.zero_()
        amg.smoother_apply(h, 0, args.kind, args.degree, bd, xs, True)
        t_apply, _ = event_time(stream, lambda: amg.smoother_apply(h, 0, args.kind, args.degree, bd, xs, True), 5)
        apply_bytes = smooth_bytes(n0, M0, 8, args.kind, args.degree, True)
        x_gpu = xs.cpu().numpy()
        amg.amg_destroy(h)
        h = None
        del rp, cl, vl
        torch.cuda.empty_cache()
        cpu = cpu_baseline(args, A, b, x_gpu, t_apply, apply_bytes)
    if h is not None:
        amg.amg_destroy(h)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}_{args.size}^3_amg_pcg_to_1e-8",
                   "smoother": KIND_NAMES[args.kind], "degree": args.degree, "n": int(n0), "nnz": int(nnz0),
                   "levels": [int(l[0]) for l in lv64], "iters": it, "assembly_s": round(assembly_s, 2), "upload_s": round(upload_s, 3),
                   "setup_s": round(setup_s, 3), "hierarchy_device_GB": round(hierarchy_bytes / 1e9, 2)},
        "value_frac_of_read_ceiling": round(value / ceil["read_GBps"], 4),
        "roofline": roofline, "cpu_baseline": cpu, "solve": solve_info, "variants": variants,
        "learned": learned_info, "diffusion_256": c3, "learned_32x64": c4,
    }
    print(json.dumps(out), flush=True)


def measured_traffic(size):
    """HBM bytes per launch of the fine-level fused step from the committed rocprofv3 counter
    summary of this workload, or None when there is none or the kernel source has changed since
    the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"fused_step_q1_{size}.md")
    if not os.path.exists(path):
        return None
    try:
        src = open(os.path.join(ROOT, "paper_2407_09848_amd", "csrc", "kernels_sparse.hip")).read()
        a = src.index("\n", src.index("// BEGIN fused-step")) + 1
        digest = hashlib.sha256(src[a:src.index("// END fused-step")].encode()).hexdigest()[:16]
        prof = open(path).read()
        if re.search(r"sha256 prefix: (\w+)", prof).group(1) != digest:
            return None
        return int(re.search(r"traffic_bytes_per_launch: (\d+)", prof).group(1))
    except (OSError, ValueError, AttributeError):
        return None


if __name__ == "__main__":
    main()
