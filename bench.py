"""Benchmark: AMG-PCG on the 3D 7-point Poisson problem at 128^3 (one MI355X).

A step is one complete solve A x = b to ||r|| <= 1e-8 ||b|| from x = 0 with
the V-cycle preconditioner (box-aggregation hierarchy 128^3 -> 16^3, dense
coarsest solve) smoothed by the optimal 4th-kind polynomial of degree 4, on
a hierarchy already resident in HBM (setup excluded, reported separately).

value       = algorithmic HBM bytes of the whole solve / its wall time (GB/s),
              bytes summed from the per-kernel models below over the launches
              one solve makes;
roofline    = the fused recurrence-step kernel on the fine level, its
              algorithmic bytes per launch / its average duration, timed here
              with events on the launch stream (difference of degree-6 and
              degree-2 smoother applications = 4 fused steps);
cpu_baseline= the FP64 CPU oracle solving the same system once (host cores);
variants    = time to 1e-8 of the other smoother kinds, of the FP32 hierarchy
              inside FP64 CG, and (when a trained network is available) of the
              learned beta, against the plain FP64 optimal 4th kind.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Smoother HBM GB/s (% peak); AMG-PCG time to 1e-8 residual, learned/FP32 vs plain"
PEAK_HBM = 8000.0  # GB/s, MI355X HBM3E


# ---- algorithmic byte models (float64 values, int32 indices) ----
def b_fused(nnz, n, store=True, w=8):
    # A (w + 4 per entry), gathered direction once, minv, r in, x read+write; + r out, g out
    return (w + 4) * nnz + (w * 7 if store else w * 5) * n


def b_first_zero(n, store, mode, w=8):
    return w * (2 + 1 + (1 if store else 0) + (1 if (store and mode == 1) else 0)) * n


def b_first_res(nnz, n, w=8):
    return (w + 4) * nnz + 5 * w * n


def b_restrict(nnz, n, w=8):
    return (w + 4) * nnz + 2 * w * n + 4 * n + w * n // 8


def b_prolong(n, w=8):
    return 2 * w * n + 4 * n + w * n // 8


def vcycle_bytes(levels, ncp, nbatch, kind, k, w=8):
    """Algorithmic bytes of one V-cycle (pre from zero, restrict, coarse, prolong, post)."""
    tot = 0
    mode = 1 if kind == 3 else 0
    for (n, nnz) in levels[:-1]:
        # pre-smoothing from zero
        tot += b_first_zero(n, k > 1, mode, w) + max(k - 2, 0) * b_fused(nnz, n, True, w) + \
            (b_fused(nnz, n, False, w) if k > 1 else 0)
        tot += b_restrict(nnz, n, w) + b_prolong(n, w)
        # post-smoothing from x
        tot += b_first_res(nnz, n, w) + max(k - 2, 0) * b_fused(nnz, n, True, w) + \
            (b_fused(nnz, n, False, w) if k > 1 else 2 * w * n + w * n)
    nL = levels[-1][0]
    nb = ncp // 64
    # coarsest: the lower 64x64 blocks of the symmetric inverse once, the block partials written and read
    tot += nbatch * (nb * (nb + 1) // 2) * 64 * 64 * 8 + 2 * nbatch * nb * nb * 64 * 8 + 2 * w * nL
    return tot


def pcg_bytes(levels, ncp, nbatch, kind, k, iters, w=8):
    n, nnz = levels[0]
    # SpMV with the fused direction update (gathers z and p_old, writes p and q), x/r update with (r, r),
    # the V-cycle, and (r, z)
    per_it = (12 * nnz + 32 * n) + 48 * n + vcycle_bytes(levels, ncp, nbatch, kind, k, w) + 16 * n
    if w == 4:
        per_it += 12 * n  # casts r -> f32, z -> f64
    # x = 0, r = b, the first V-cycle, (r, z), p_old = 0
    setup = 8 * n + 16 * n + vcycle_bytes(levels, ncp, nbatch, kind, k, w) + 16 * n + 8 * n
    return setup + iters * per_it


def measured_traffic(size):
    """HBM bytes per launch of the fine-level fused step from the committed rocprofv3 counter
    summary, or None when that summary does not cover this workload or the kernel source
    has changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"fused_step_poisson{size}.md")
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


def stacked_diffusion(W, nprob, size, seed0):
    import numpy as np
    sig = W.config4_sigmas(nprob)
    mats = [W.fv_diffusion(np.exp(sig[p] * W.gaussian_random_field((size, size, size), 8.0, seed0 + p)))
            for p in range(nprob)]
    return W.stack_block_diagonal(mats), sig


def learned_variant(args, amg, W, h, bd, x, stream, variants):
    """Train the 8-64-64-6 network on 32 stacked 64^3 diffusion problems (the learned-weights
    workload, FP32, the library's adjoint and network kernels), report its loss against the plain
    optimal weights at degree 6 and at the bench degree, then apply the bench-degree network to
    this system (kept only if it lowers the two-cycle residual ratio here) and time the solve."""
    import numpy as np
    import torch

    from paper_2407_09848_amd import learned
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = {}
    t0 = time.perf_counter()
    big, sig = stacked_diffusion(W, 32, 64, W.SEED_GRF)
    held, _ = stacked_diffusion(W, 32, 64, W.SEED_GRF + 500)
    b4 = dev(W.rhs_uniform(big.n, W.SEED_RHS + 4))
    b4h = dev(W.rhs_uniform(held.n, W.SEED_RHS + 40))
    hs = [amg.amg_setup(dev(M.row_ptr), dev(M.col), dev(M.val), M.grid[0], M.grid[1], M.grid[2] // 32, 32,
                        4096, amg.AMG_FP32) for M in (big, held)]
    out["setup_s"] = round(time.perf_counter() - t0, 2)
    nets = {}
    for deg in sorted({6, args.degree}):
        t0 = time.perf_counter()
        res = learned.train(hs[0], b4, sig, degree=deg, steps=args.train_steps, lr=3e-3,
                            init_params=W.mlp_init(W.SEED_MLP))
        torch.cuda.synchronize()
        tt = time.perf_counter() - t0
        f = amg.amg_level_features(hs[0], deg, sig)
        beta, _, valid = learned.predict_beta(hs[0], res.params, f, deg, 32)
        lt, _ = learned.evaluate(hs[0], beta, b4, deg, 32)
        fh = amg.amg_level_features(hs[1], deg, sig)
        bh, _, _ = learned.predict_beta(hs[1], res.params, fh, deg, 32)
        L = amg.amg_num_levels(hs[1])
        plain = dev(np.tile(np.array(amg.amg_default_beta(deg)), (32, L, 1)).ravel())
        lh, _ = learned.evaluate(hs[1], bh, b4h, deg, 32)
        lp, _ = learned.evaluate(hs[1], plain, b4h, deg, 32)
        out[f"degree{deg}"] = {"train_steps": args.train_steps, "train_s": round(tt, 2),
                               "train_loss_plain": round(res.plain_loss, 6), "train_loss_learned": round(lt, 6),
                               "heldout_loss_plain": round(lp, 6), "heldout_loss_learned": round(lh, 6),
                               "invalid_rows": int((valid == 0).sum().item())}
        nets[deg] = res.params
    for hh in hs:
        amg.amg_destroy(hh)
    # apply to this system at the bench degree, kept only if it lowers the two-cycle residual ratio here
    deg = args.degree
    lb = learned.learned_level_betas(h, nets[deg], deg, 0.0)
    L = amg.amg_num_levels(h)
    tab_l = np.array(amg.amg_default_beta(deg) * L).reshape(L, deg)
    tab_l[:L - 1] = np.array(lb)
    plain = dev(np.tile(np.array(amg.amg_default_beta(deg)), (L, 1)).ravel())
    r_learned, _ = learned.evaluate(h, dev(tab_l.ravel()), bd, deg, 1)
    r_plain, _ = learned.evaluate(h, plain, bd, deg, 1)
    use = r_learned < r_plain
    if use:
        learned.apply_level_betas(h, deg, lb)
    amg.pcg_solve(h, args.kind, deg, bd, x, True, 1e-8, 1000)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(3):
        rc, itv, relv, _ = amg.pcg_solve(h, args.kind, deg, bd, x, True, 1e-8, 1000)
    e1.record(stream)
    torch.cuda.synchronize()
    amg.amg_reset_beta(h)
    tm = e0.elapsed_time(e1) / 3
    base = variants.get(f"fp64_optcheb4_k{deg}", {}).get("ms")
    variants[f"learned_optcheb4_k{deg}"] = {"ms": round(tm, 3), "iters": itv,
                                           "vs_plain_fp64": round(tm / base, 3) if base else None,
                                           "weights": "learned" if use else "plain (fallback)"}
    out["this_system"] = {"two_cycle_ratio_plain": round(r_plain, 6), "two_cycle_ratio_learned": round(r_learned, 6),
                          "weights_used": "learned" if use else "plain (fallback)", "level_betas": lb}
    out["heldout_solves"] = heldout_solves(args, amg, W, nets[deg], deg, stream)
    return out


def heldout_solves(args, amg, W, params, deg, stream):
    """Time to 1e-8 on held-out problems of the training family (one 64^3 diffusion problem per
    sigma, FP64 hierarchy, standard PCG), plain optimal weights against the learned ones (kept only
    where they lower the two-cycle residual ratio of the problem's right-hand side)."""
    import numpy as np
    import torch

    from paper_2407_09848_amd import learned
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    res = {}
    for idx, sigma in enumerate((0.5, 1.0, 2.0)):
        M = W.fv_diffusion(np.exp(sigma * W.gaussian_random_field((64, 64, 64), 8.0, W.SEED_GRF + 900 + idx)))
        b = dev(W.rhs_uniform(M.n, W.SEED_RHS + 90 + idx))
        hp = amg.amg_setup(dev(M.row_ptr), dev(M.col), dev(M.val), *M.grid, 1, 4096, amg.AMG_FP64)
        x = torch.zeros(M.n, dtype=torch.float64, device="cuda")
        L = amg.amg_num_levels(hp)
        lb = learned.learned_level_betas(hp, params, deg, sigma)
        tab = np.array(amg.amg_default_beta(deg) * L).reshape(L, deg)
        tab[:L - 1] = np.array(lb)
        r_l, _ = learned.evaluate(hp, dev(tab.ravel()), b, deg, 1)
        r_p, _ = learned.evaluate(hp, dev(np.tile(np.array(amg.amg_default_beta(deg)), (L, 1)).ravel()), b, deg, 1)
        entry = {"two_cycle_ratio_plain": round(r_p, 6), "two_cycle_ratio_learned": round(r_l, 6)}
        for name, use in (("plain", False), ("learned", r_l < r_p)):
            amg.amg_reset_beta(hp)
            if use:
                learned.apply_level_betas(hp, deg, lb)
            amg.pcg_solve(hp, args.kind, deg, b, x, True, 1e-8, 1000)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(3):
                rc, itv, _, _ = amg.pcg_solve(hp, args.kind, deg, b, x, True, 1e-8, 1000)
            e1.record(stream)
            torch.cuda.synchronize()
            entry[name] = {"ms": round(e0.elapsed_time(e1) / 3, 3), "iters": itv}
            if name == "learned":
                entry[name]["weights"] = "learned" if use else "plain (fallback)"
        entry["learned_vs_plain"] = round(entry["learned"]["ms"] / entry["plain"]["ms"], 3)
        amg.amg_destroy(hp)
        res[f"sigma{sigma}"] = entry
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--kind", type=int, default=2)
    ap.add_argument("--degree", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--variants", default="kinds,fp32,paper",
                    help="comma-separated subset of the variants to time: kinds (the other smoother kinds), "
                         "fp32 (the FP32 hierarchy), paper (smoothed prolongators on box, matching and VBM "
                         "aggregates)")
    ap.add_argument("--no-learned", action="store_true", help="skip training the learned-weight network")
    ap.add_argument("--train-steps", type=int, default=100)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2407_09848_amd as amg
    import workloads as W

    torch.cuda.set_device(0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    A, b, _ = W.config_problem(2, size=args.size)
    rp, cl, vl, bd = dev(A.row_ptr), dev(A.col), dev(A.val), dev(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = amg.amg_setup(rp, cl, vl, *A.grid, 1, 4096, amg.AMG_FP64)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    L = amg.amg_num_levels(h)
    levels = [amg.amg_level_info(h, l) for l in range(L)]
    nL = levels[-1][0]
    ncp = (nL + 63) // 64 * 64
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")

    def solve(handle, kind, k, flexible=False):
        return amg.pcg_solve(handle, kind, k, bd, x, True, 1e-8, 1000, flexible)

    for _ in range(args.warmup):
        solve(h, args.kind, args.degree)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    iters = []
    for _ in range(args.steps):
        rc, it, rel, _ = solve(h, args.kind, args.degree)
        iters.append(it)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    it = iters[-1]
    # the solve once more, untimed, for its residual history and solution
    _, _, _, hist = amg.pcg_solve(h, args.kind, args.degree, bd, x, True, 1e-8, 1000, False, True)
    x_gpu = x.cpu().numpy()
    solve_info = {"iters": len(hist) - 1, "relres_history": [float(f"{v:.4e}") for v in hist],
                  "true_relres": float(np.linalg.norm(b - A.to_scipy() @ x_gpu) / np.linalg.norm(b))}
    solve_bytes = pcg_bytes(levels, ncp, 1, args.kind, args.degree, it)
    value = solve_bytes / (ms * 1e-3) / 1e9

    # ---- fused recurrence step on the fine level: events around smoother applications ----
    n0, nnz0 = levels[0]
    xs = torch.zeros(n0, dtype=torch.float64, device="cuda")
    reps = 50

    def time_apply(k):
        for _ in range(3):
            amg.smoother_apply(h, 0, args.kind, k, bd, xs, True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            amg.smoother_apply(h, 0, args.kind, k, bd, xs, True)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t6, t2 = time_apply(6), time_apply(2)
    t_fused_ms = (t6 - t2) / 4.0
    fused_bytes = b_fused(nnz0, n0, True)
    achieved = fused_bytes / (t_fused_ms * 1e-3) / 1e9
    # the bytes the kernel must move in the layout it uses: offset-aligned slices read no column
    # indices (8 bytes per stored entry plus a 4-byte offset per 64), packed ones 12
    padded, lanes, aligned = amg.amg_level_layout(h, 0)
    format_bytes = (8 * padded + 4 * (padded // 64) if aligned else 12 * padded) + 56 * n0
    achieved_fmt = format_bytes / (t_fused_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM, 4), "traffic": measured_traffic(args.size),
                "kernel": f"k_fused<double,0,true> (fine level, {args.size}^3)",
                "bytes_per_launch": fused_bytes, "avg_launch_us": round(t_fused_ms * 1e3, 2),
                "layout": {"stored_entries": int(padded), "lanes_per_row": lanes, "offset_aligned": aligned,
                           "format_bytes_per_launch": int(format_bytes),
                           "achieved_format": round(achieved_fmt, 1),
                           "frac_format": round(achieved_fmt / PEAK_HBM, 4)}}

    # ---- plain device copy of 1 GiB: measured copy bandwidth, and the reference
    #      dispatch that calibrates the HBM byte counters of a profiling run ----
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    roofline["copy_GBps"] = round(copy_gbs, 1)
    del dst
    src2 = torch.ones(1 << 28, dtype=torch.float64, device="cuda")  # 2 GiB read by a reduction
    src2.sum()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(10):
        src2.sum()
    e1.record(stream)
    torch.cuda.synchronize()
    roofline["read_GBps"] = round(src2.numel() * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del src, src2

    # ---- variants: other kinds, FP32 hierarchy ----
    variants = {}
    chosen = set(args.variants.split(","))
    if not args.no_variants:
        def time_solve(handle, kind, k, reps=3, flexible=False):
            solve(handle, kind, k, flexible)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                rc, itv, relv, _ = solve(handle, kind, k, flexible)
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps, itv
        names = {0: "l1jacobi", 1: "cheb4", 2: "optcheb4", 3: "optcheb1"}
        for kind in ((0, 1, 2, 3) if "kinds" in chosen else (args.kind,)):
            tm, itv = time_solve(h, kind, args.degree)
            variants[f"fp64_{names[kind]}_k{args.degree}"] = {"ms": round(tm, 3), "iters": itv}
        if "fp32" in chosen:
            h32 = amg.amg_setup(rp, cl, vl, *A.grid, 1, 4096, amg.AMG_FP32)
            tm, itv = time_solve(h32, args.kind, args.degree)
            xr = x.cpu().numpy()
            variants[f"fp32_{names[args.kind]}_k{args.degree}"] = {
                "ms": round(tm, 3), "iters": itv,
                "true_relres": float(np.linalg.norm(b - A.to_scipy() @ xr) / np.linalg.norm(b))}
            amg.amg_destroy(h32)
        # the paper's own preconditioner ingredients (Section 4): smoothed prolongator,
        # 30 l1-Jacobi sweeps on the coarsest level, flexible CG
        # (on the box aggregates, on compatible-matching aggregates of up to 8 rows and on the
        # classical smoothed-aggregation (VBM) aggregates with strength threshold 0.08), and the
        # smoothed prolongator with the dense Cholesky coarsest solve of the plain configuration
        paper = (("box", amg.AMG_AGG_BOX, 30), ("matching", amg.AMG_AGG_MATCHING, 30),
                 ("vbm", amg.AMG_AGG_VBM, 30), ("box", amg.AMG_AGG_BOX, 0))
        for tag, agg, sweeps in (paper if "paper" in chosen else ()):
            name = f"{tag}_smoothed_p_" + (f"sweeps{sweeps}_fcg" if sweeps else "cholesky_fcg")
            t0 = time.perf_counter()
            try:
                hsa = amg.amg_setup(rp, cl, vl, *A.grid, 1, 4096, amg.AMG_FP64, 2, True, sweeps, agg)
            except amg.AmgError as e:
                hsa = None
                variants[name] = {"error": str(e)}
            if hsa is None:
                continue
            torch.cuda.synchronize()
            sa_setup = time.perf_counter() - t0
            for kind in (args.kind, 3):
                tm, itv = time_solve(hsa, kind, args.degree, flexible=True)
                variants[f"fp64_{names[kind]}_k{args.degree}_{name}"] = {
                    "ms": round(tm, 3), "iters": itv, "setup_s": round(sa_setup, 3),
                    "levels": [amg.amg_level_info(hsa, l) for l in range(amg.amg_num_levels(hsa))]}
            amg.amg_destroy(hsa)
        base = variants[f"fp64_{names[args.kind]}_k{args.degree}"]["ms"]
        for v in variants.values():
            if "ms" in v:
                v["vs_plain_fp64"] = round(v["ms"] / base, 3)
    # ---- learned weights: trained on the stacked diffusion problems, applied to this system ----
    learned_info = None
    if not args.no_variants and not args.no_learned:
        learned_info = learned_variant(args, amg, W, h, bd, x, stream, variants)
    amg.amg_destroy(h)

    # ---- CPU baseline: the oracle solving the same system once ----
    cpu = None
    if not args.no_cpu:
        from threadpoolctl import threadpool_limits

        from oracle import amg as OA
        with threadpool_limits(limits=1):
            As = A.to_scipy()
            H = OA.build_hierarchy(As, A.grid)
            t0 = time.perf_counter()
            res, _ = OA.amg_pcg(As, b, A.grid, args.kind, args.degree, H=H)
            cpu_s = time.perf_counter() - t0
        cpu_bytes = pcg_bytes(levels, ncp, 1, args.kind, args.degree, res.iters)
        cpu = {"value": round(cpu_bytes / cpu_s / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"one full FP64 oracle AMG-PCG solve of the same {args.size}^3 system "
                         f"({res.iters} iterations, {cpu_s:.1f} s, scipy/numpy single thread)",
               "solve_s": round(cpu_s, 2), "iters": res.iters}
        solve_info["error_vs_oracle"] = float(np.linalg.norm(x_gpu - res.x) / np.linalg.norm(res.x))
        solve_info["iters_oracle"] = res.iters

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"poisson3d_7pt_{args.size}^3_amg_pcg_to_1e-8",
                   "smoother": {0: "l1jacobi", 1: "cheb4", 2: "optcheb4", 3: "optcheb1"}[args.kind],
                   "degree": args.degree, "n": int(n0), "nnz": int(nnz0), "levels": [int(l[0]) for l in levels],
                   "iters": it, "setup_s": round(setup_s, 3)},
        "roofline": roofline, "cpu_baseline": cpu, "solve": solve_info, "variants": variants,
        "learned": learned_info,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
