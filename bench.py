"""Benchmark of the eigCG hot path on one MI355X.

Workload (one step = one quark mass): 16^3 x 32 Wilson lattice, synthetic
SU(3) links exp(i 0.5 H) (seed 1), FP64, single-RHS launches:
  phase 1: Incremental eigCG(10, 100) on 24 Gaussian right-hand sides (the bank
           grows to 240 vectors);
  phase 2: init-CG deflated by the 240 vectors on 100 more right-hand sides;
every solve to FP64 true relative residual <= 1e-10.  Steps cycle over three
masses approaching the critical one.  `value` = right-hand sides solved per
second over the timed steps (phase 1 and 2 together, bank building amortised
as in the paper's phase accounting).  Extra fields give plain FP64 CG on a
sample of the same right-hand sides (the speed-up baseline), the stencil's
achieved bandwidth against the HBM roofline (dominant kernel) and the CPU
oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

LATTICE = (16, 16, 16, 32)
EPS, SEED = 0.5, 1
MASSES = (-0.55, -0.58, -0.60)
NEV, M, NBANK = 10, 100, 240
N_EIG, N_DEFL = 24, 100
TOL = 1e-10
HBM_LATTICE, HBM_SEED = (24, 24, 24, 48), 3
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def site_bytes_stencil(two_row_links: bool, elem=16):
    # spinor in + links as stored + spinor out, each read/written once per site
    links = 4 * (6 if two_row_links else 9) * elem
    return 12 * elem + links + 12 * elem


# Stencil passes of every SAMPLE_EVERY-th CG iteration of the timed steps are
# timed with events (each timed pass costs a few microseconds of dispatch gap,
# so sampling every iteration or every 4th would slow the measured workload);
# the 24^3x48 CG sample, outside the timed steps, times every HBM_SAMPLE_EVERY-th.
SAMPLE_EVERY = 32
HBM_SAMPLE_EVERY = 4
STENCIL_SOURCES = ("paper_0707_0131_amd/csrc/stencil_impl.h",
                   "paper_0707_0131_amd/csrc/dslash_f64.hip", "paper_0707_0131_amd/csrc/wilson.h",
                   "paper_0707_0131_amd/csrc/common.h")
TRAFFIC_SUMMARY = "profiles/k_wilson_pair_cgr_f64_16x16x16x32.md"
TRAFFIC_SUMMARY_HBM = "profiles/k_wilson_pair_cgr_f64_24x24x24x48.md"
HBM_CG_MASS = -0.58
HBM_CG_ITERS = 240  # FP64 CG iterations sampled on the 24^3x48 lattice


RESTART_RULE = {"fixed": 0, "dynamic": 1}
restart_rule = 0  # init-CG restart threshold of the timed steps (--restart-rule)
sample_every = SAMPLE_EVERY  # event-timed CG iterations of the timed steps (--sample-every)
use_graphs = 0  # timed steps replay captured CG segments (--graphs)
DEFL_BATCH = 4  # phase-2 init-CG right-hand sides solved together in lockstep
defl_batch = DEFL_BATCH  # (--defl-batch; plain CG runs the same batches)


def run_step(B, torch, g, mass, bt, xt, n_eig=N_EIG):
    p = B.eigcg_default_params(dims=LATTICE, mass=mass, nev=NEV, m=M, max_bank=NBANK,
                               max_iter=40000, check_every=16, sample_every=sample_every,
                               use_graphs=use_graphs, max_batch=defl_batch,
                               restart_rule=restart_rule)
    ctx = B.eigcg_create(p, g)
    try:
        xt.zero_()
        t0 = time.perf_counter()
        samples = None
        if defl_batch == 1:
            rc1, st1 = B.eigcg_solve(ctx, bt[:n_eig], xt[:n_eig], TOL, B.EIGCG_MODE_EIGCG)
        else:  # Incremental eigCG stays sequential: one right-hand side per call
            st1 = []
            for i in range(n_eig):
                _, st = B.eigcg_solve(ctx, bt[i:i + 1], xt[i:i + 1], TOL, B.EIGCG_MODE_EIGCG)
                st1 += st
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if defl_batch > 1:  # the single-column launches of phase 1 for the roofline
            samples = B.eigcg_kernel_samples(ctx, reset=True)["f64"]
            t1 = time.perf_counter()
        rc2, st2 = B.eigcg_solve(ctx, bt[n_eig:], xt[n_eig:], TOL, B.EIGCG_MODE_INITCG)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        vals, _ = B.eigcg_bank_info(ctx)
        if samples is None:
            samples = B.eigcg_kernel_samples(ctx)["f64"]
        samples["stencil_variant"] = B.eigcg_layout_info(ctx)["variant64"]
    finally:
        B.eigcg_destroy(ctx)
    bad = [s for s in st1 + st2 if s["status"] != 0 or s["true_rel_res"] > TOL]
    return {
        "mass": mass,
        "phase1_restarts": sum(s["restarts"] for s in st1),
        "phase2_restarts": sum(s["outer_steps"] for s in st2),
        "phase1_s": t1 - t0,
        "phase2_s": t2 - t1,
        "phase1_iters": [s["iters"] for s in st1],
        "phase2_iters": [s["iters"] for s in st2],
        "phase2_first_leg_iters": [s["first_leg_iters"] for s in st2],
        "phase2_restart_tau": sorted({s["restart_tau"] for s in st2}),
        "max_true_rel_res": max(s["true_rel_res"] for s in st1 + st2),
        "failed": len(bad),
        "bank_lambda_min": float(vals[0]) if len(vals) else None,
        "bank_size": int(len(vals)),
        "samples": samples,
    }


def plain_cg(B, torch, g, mass, bt, xt, n):
    p = B.eigcg_default_params(dims=LATTICE, mass=mass, max_iter=40000, check_every=32,
                               max_batch=defl_batch)
    ctx = B.eigcg_create(p, g)
    try:
        xt[:n].zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = B.eigcg_solve(ctx, bt[:n], xt[:n], TOL, B.EIGCG_MODE_CG)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        B.eigcg_destroy(ctx)
    return dt, [s["iters"] for s in st], max(s["true_rel_res"] for s in st)


def lambda_max_est(B, torch, g, mass, dims=None, iters=60, seed=4242):
    """Largest eigenvalue of A = M^H M by power iteration through the library's
    FP64 operator (Rayleigh quotient of the last iterate; a lower bound that
    converges from below)."""
    from synthetic import gaussian_rhs
    dims = dims or LATTICE
    p = B.eigcg_default_params(dims=dims, mass=mass, max_bank=0)
    ctx = B.eigcg_create(p, g)
    try:
        v = torch.from_numpy(gaussian_rhs(dims, seed)).to("cuda:0")[None]
        w = torch.empty_like(v)
        lam = 0.0
        for _ in range(iters):
            v /= torch.linalg.vector_norm(v)
            B.eigcg_apply(ctx, B.EIGCG_OP_A, v, w)
            lam = float(torch.vdot(v.reshape(-1), w.reshape(-1)).real)
            v, w = w, v
    finally:
        B.eigcg_destroy(ctx)
    return lam


CRIT_MASS = -0.61


def critical_leg(B, torch, g, bt, xt, n_eig=N_EIG, n_defl=24, n_plain=2):
    """The deflated workload closer to the critical mass (Section 5.4's claim
    that deflation removes the critical slowdown): plain FP64 CG on n_plain
    right-hand sides, then Incremental eigCG(10,100) on n_eig and init-CG on
    n_defl at m_q = CRIT_MASS, with kappa = lambda_max / lambda_min from power
    iteration and the bank's lowest Ritz value."""
    log(f"critical-mass leg (mass {CRIT_MASS})")
    dt, its, res = plain_cg(B, torch, g, CRIT_MASS, bt[n_eig:], xt[n_eig:], n_plain)
    r = run_step(B, torch, g, CRIT_MASS, bt[:n_eig + n_defl], xt[:n_eig + n_defl], n_eig)
    lam_max = lambda_max_est(B, torch, g, CRIT_MASS)
    out = {"mass": CRIT_MASS, "plain_cg_iters": its, "plain_cg_s_per_rhs": dt / n_plain,
           "plain_max_true_rel_res": res, "lambda_max": lam_max,
           "bank_lambda_min": r["bank_lambda_min"],
           "kappa": lam_max / r["bank_lambda_min"] if r["bank_lambda_min"] else None,
           "phase1_iters": r["phase1_iters"],
           "phase2_mean_iters": sum(r["phase2_iters"]) / len(r["phase2_iters"]),
           "phase2_s_per_rhs": r["phase2_s"] / n_defl,
           "phase2_speedup": (dt / n_plain) / (r["phase2_s"] / n_defl),
           "max_true_rel_res": r["max_true_rel_res"], "failed": r["failed"]}
    log(f"critical mass {CRIT_MASS}: kappa {out['kappa']:.2e}, plain CG {its} iterations, "
        f"init-CG {out['phase2_mean_iters']:.0f} iterations, phase 2 "
        f"{out['phase2_speedup']:.1f}x plain CG")
    return out


SCHUR_MASS = -0.58


def schur_leg(B, torch, g, bt, n_plain=4, n_eig=N_EIG, n_defl=N_DEFL):
    """Odd-even (Schur complement) preconditioning on the bench lattice: M x = b
    for the same right-hand sides through the full normal equations
    (M^H M x = M^H b) and through the even-site system (Mhat^H Mhat x_e =
    Mhat^H bhat, then x_o), plain FP64 CG both ways, then the deflated
    workload (Incremental eigCG on n_eig, init-CG on n_defl) on the even-site
    system.  Every timing includes the maps between the two systems."""
    log(f"odd-even leg (mass {SCHUR_MASS})")
    mass = SCHUR_MASS
    nh = bt[0].numel() // 12 // 2
    full = B.eigcg_create(B.eigcg_default_params(dims=LATTICE, mass=mass, max_iter=40000,
                                                 check_every=32), g)
    out = {"mass": mass}
    try:
        b = bt[:n_plain]
        xf = torch.zeros_like(b)
        mb = torch.empty_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.eigcg_apply(full, B.EIGCG_OP_MDAG, b, mb)
        rc, st = B.eigcg_solve(full, mb, xf, TOL, B.EIGCG_MODE_CG)
        torch.cuda.synchronize()
        dt_full = time.perf_counter() - t0
        out["plain_full_cg"] = {"s_per_rhs": dt_full / n_plain, "iters": [s["iters"] for s in st]}
        sch = B.eigcg_create(B.eigcg_default_params(dims=LATTICE, mass=mass, max_iter=40000,
                                                    check_every=32, schur=1), g)
        try:
            rhs = torch.empty((n_plain, nh, 4, 3), dtype=torch.complex128, device="cuda:0")
            xe = torch.zeros_like(rhs)
            xs = torch.empty_like(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.eigcg_schur_rhs(sch, b, rhs)
            rc, st = B.eigcg_solve(sch, rhs, xe, TOL, B.EIGCG_MODE_CG)
            B.eigcg_schur_reconstruct(sch, b, xe, xs)
            torch.cuda.synchronize()
            dt_s = time.perf_counter() - t0
        finally:
            B.eigcg_destroy(sch)
        # both solutions of M x = b: residual with the full operator, and their difference
        mx = torch.empty_like(b)
        B.eigcg_apply(full, B.EIGCG_OP_M, xs, mx)
        res_m = max(float(torch.linalg.vector_norm(mx[i] - b[i]) / torch.linalg.vector_norm(b[i]))
                    for i in range(n_plain))
        dx = max(float(torch.linalg.vector_norm(xs[i] - xf[i]) / torch.linalg.vector_norm(xf[i]))
                 for i in range(n_plain))
        out["plain_schur_cg"] = {"s_per_rhs": dt_s / n_plain, "iters": [s["iters"] for s in st],
                                 "max_true_rel_res": max(s["true_rel_res"] for s in st),
                                 "max_M_rel_res": res_m, "max_rel_diff_vs_full": dx}
        out["plain_speedup"] = dt_full / dt_s
        del mx, mb, xf, xs, rhs, xe
    finally:
        B.eigcg_destroy(full)
    # deflated workload on the even-site system
    sch = B.eigcg_create(B.eigcg_default_params(dims=LATTICE, mass=mass, nev=NEV, m=M,
                                                max_bank=NBANK, max_iter=40000, check_every=16,
                                                schur=1), g)
    try:
        n = n_eig + n_defl
        rhs = torch.empty((n, nh, 4, 3), dtype=torch.complex128, device="cuda:0")
        xe = torch.zeros_like(rhs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.eigcg_schur_rhs(sch, bt[:n], rhs)
        rc1, st1 = B.eigcg_solve(sch, rhs[:n_eig], xe[:n_eig], TOL, B.EIGCG_MODE_EIGCG)
        rc2, st2 = B.eigcg_solve(sch, rhs[n_eig:], xe[n_eig:], TOL, B.EIGCG_MODE_INITCG)
        xs = torch.empty_like(bt[:1])
        for i in range(n):  # reconstruction of every solution, one at a time (memory)
            B.eigcg_schur_reconstruct(sch, bt[i:i + 1], xe[i:i + 1], xs)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        vals, _ = B.eigcg_bank_info(sch)
    finally:
        B.eigcg_destroy(sch)
    allst = st1 + st2
    out["deflated_schur"] = {
        "rhs_per_s": n / dt,
        "wall_s": dt,
        "phase1_iters": [s["iters"] for s in st1],
        "phase2_mean_iters": sum(s["iters"] for s in st2) / max(1, len(st2)),
        "bank": int(len(vals)),
        "max_true_rel_res": max(s["true_rel_res"] for s in allst),
        "failed": sum(1 for s in allst if s["status"] != 0 or s["true_rel_res"] > TOL),
    }
    out["deflated_schur_speedup_vs_plain_full_cg"] = (n / dt) * out["plain_full_cg"]["s_per_rhs"]
    log(f"odd-even: plain full {out['plain_full_cg']['s_per_rhs']:.3f} s/RHS, plain Schur "
        f"{out['plain_schur_cg']['s_per_rhs']:.3f} s/RHS, deflated Schur {n / dt:.1f} RHS/s")
    return out


def auto_leg(B, torch, g, bt, xt, mass=-0.58):
    """The whole right-hand-side sequence of one step in EIGCG_MODE_AUTO: the
    library runs Incremental eigCG while its measured gain outweighs its
    overhead, then init-CG (against the step's fixed 24 + 100 plan)."""
    log(f"automatic eigCG/init-CG switch (mass {mass})")
    p = B.eigcg_default_params(dims=LATTICE, mass=mass, nev=NEV, m=M, max_bank=NBANK,
                               max_iter=40000, check_every=16)
    ctx = B.eigcg_create(p, g)
    try:
        xt.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = B.eigcg_solve(ctx, bt, xt, TOL, B.EIGCG_MODE_AUTO)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bank = len(B.eigcg_bank_info(ctx)[0])
    finally:
        B.eigcg_destroy(ctx)
    keig = sum(1 for s in st if s["mode_used"] == B.EIGCG_MODE_EIGCG)
    out = {"mass": mass, "rhs": len(st), "eigcg_rhs": keig, "bank": bank,
           "rhs_per_s": len(st) / dt, "wall_s": dt,
           "max_true_rel_res": max(s["true_rel_res"] for s in st),
           "failed": sum(1 for s in st if s["status"] != 0 or s["true_rel_res"] > TOL)}
    log(f"automatic switch: {keig} eigCG right-hand sides (bank {bank}), {len(st) / dt:.1f} RHS/s")
    return out


BICG_SOLVERS = ((False, False), (False, True), (True, True), (True, False))


def bicgstab_leg(B, torch, g, bt, xt, mass=-0.58, n_eig=N_EIG, n_rhs=4, max_iter=20000,
                 solvers=BICG_SOLVERS):
    """Section 1's use of the bank for a nonsymmetric solver: after 24
    Incremental eigCG solves, the next right-hand sides are solved for M x = b
    by BiCGSTAB on M and on gamma5 M, with and without the bank's
    least-squares guess, beside init-CG on A x = M^H b with the same bank."""
    log(f"deflated BiCGSTAB (mass {mass})")
    p = B.eigcg_default_params(dims=LATTICE, mass=mass, nev=NEV, m=M, max_bank=NBANK,
                               max_iter=40000, check_every=16)
    ctx = B.eigcg_create(p, g)
    out = {"mass": mass, "rhs": n_rhs, "max_iter": max_iter, "runs": []}
    try:
        xt.zero_()
        B.eigcg_solve(ctx, bt[:n_eig], xt[:n_eig], TOL, B.EIGCG_MODE_EIGCG)
        out["bank"] = len(B.eigcg_bank_info(ctx)[0])
        b = bt[n_eig:n_eig + n_rhs]
        x = xt[n_eig:n_eig + n_rhs]
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = B.eigcg_solve(ctx, b, x, TOL, B.EIGCG_MODE_INITCG)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["runs"].append({
            "solver": "init-CG on A x = M^H b (reference)", "s_per_rhs": dt / n_rhs,
            "mean_iters": sum(s["iters"] for s in st) / n_rhs,
            "mean_matvecs": 2.0 * sum(s["iters"] for s in st) / n_rhs,
            "max_true_rel_res": max(s["true_rel_res"] for s in st),
            "failed": sum(1 for s in st if s["status"] != 0)})
        for gamma5, deflate in solvers:
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = B.eigcg_solve_bicgstab(ctx, b, x, TOL, gamma5=gamma5, deflate=deflate,
                                           max_iter=max_iter)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            name = ("BiCGSTAB on gamma5 M" if gamma5 else "BiCGSTAB on M") + \
                (", deflated" if deflate else "")
            run = {"solver": name, "s_per_rhs": dt / n_rhs,
                   "mean_iters": sum(s["iters"] for s in st) / n_rhs,
                   "mean_matvecs": 2.0 * sum(s["iters"] for s in st) / n_rhs,
                   "mean_guess_rel_res": sum(s["guess_rel_res"] for s in st) / n_rhs,
                   "max_true_rel_res": max(s["true_rel_res"] for s in st),
                   "failed": sum(1 for s in st if s["status"] != 0)}
            out["runs"].append(run)
            log(f"{name}: {run['s_per_rhs']:.3f} s/RHS, {run['mean_iters']:.0f} iterations, "
                f"failed {run['failed']}")
    finally:
        B.eigcg_destroy(ctx)
    return out


def spectral_leg(B, torch, g, bt, xt, mass=-0.58, n_rhs=4):
    """Section 2.1's alternative to init-CG and Section 4's example: after one
    eigCG(10, 100) solve (10 Ritz vectors) and after 24 Incremental eigCG
    solves (240), the next right-hand sides are solved by plain CG, by init-CG
    with the bank, and by CG with the same bank as a spectral preconditioner
    (P^{-1} = I + U_R (sigma Theta^{-1} - I) U_R^H, two passes over the bank
    per iteration; the bank is copied into a preconditioned context), FP64,
    tol 1e-10."""
    log(f"spectral preconditioning (mass {mass})")
    out = {"mass": mass, "rhs": n_rhs, "banks": []}
    b = bt[N_EIG:N_EIG + n_rhs]
    x = xt[N_EIG:N_EIG + n_rhs]
    shape = tuple(bt.shape[1:])

    def timed(ctx, mode):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = B.eigcg_solve(ctx, b, x, TOL, mode)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return {"s_per_rhs": dt / n_rhs, "mean_iters": sum(s["iters"] for s in st) / n_rhs,
                "max_true_rel_res": max(s["true_rel_res"] for s in st),
                "failed": sum(1 for s in st if s["status"] != 0 or s["true_rel_res"] > TOL)}

    kw = dict(dims=LATTICE, mass=mass, nev=NEV, m=M, max_bank=NBANK, max_iter=40000,
              check_every=16, restart_tol=-1.0)
    for n_bank_rhs in (1, N_EIG):
        ctx = B.eigcg_create(B.eigcg_default_params(**kw), g)
        spec = None
        try:
            xt[:n_bank_rhs].zero_()
            B.eigcg_solve(ctx, bt[:n_bank_rhs], xt[:n_bank_rhs], TOL, B.EIGCG_MODE_EIGCG)
            l = len(B.eigcg_bank_info(ctx)[0])
            entry = {"bank_rhs": n_bank_rhs, "bank": l, "runs": []}
            runs = [("init-CG (no restart)", ctx, B.EIGCG_MODE_INITCG)]
            if n_bank_rhs == 1:
                runs.insert(0, ("plain CG", ctx, B.EIGCG_MODE_CG))
            vecs = torch.empty((l,) + shape, dtype=torch.complex128, device="cuda:0")
            B.eigcg_bank_vectors(ctx, 0, l, vecs)
            h = B.eigcg_bank_matrix(ctx, l)
            spec = B.eigcg_create(B.eigcg_default_params(precond=1, **kw), g)
            B.eigcg_bank_restore(spec, vecs, h)
            del vecs
            runs.append(("spectral preconditioned CG", spec, B.EIGCG_MODE_CG))
            for name, c, mode in runs:
                run = timed(c, mode)
                run["solver"] = name
                entry["runs"].append(run)
                log(f"bank of {l}: {name}: {run['s_per_rhs']:.3f} s/RHS, "
                    f"{run['mean_iters']:.0f} iterations, failed {run['failed']}")
            out["banks"].append(entry)
        finally:
            B.eigcg_destroy(ctx)
            if spec is not None:
                B.eigcg_destroy(spec)
        torch.cuda.empty_cache()
    return out


FP64_MFMA_PEAK_TF = 78.6
FP32_MFMA_PEAK_TF = 157.3


def gemm_roofline(B, torch, reps=10):
    """The window and deflation contractions alone, at the bench lattice's
    vector length (n = 12 V complex entries), through eigcg_debug_gemm:
    V (QZ) of the eigCG restart (m = 100 -> 2 nev = 20, FP64), the init-CG
    deflation U^H r and U c with a 240-vector FP64 bank (one column), and the
    batched FP32 forms for 12 columns.  Each shape: mean time of reps calls,
    algorithmic bytes (every input column read once, every output written
    once) and complex flops (8 n K N)."""
    V = LATTICE[0] * LATTICE[1] * LATTICE[2] * LATTICE[3]
    n = 12 * V
    shapes = [("restart V(QZ)", 0, 0, M, 2 * NEV), ("deflation U c", 0, 0, NBANK, 1),
              ("deflation U^H r", 0, 1, NBANK, 1), ("batched U C fp32", 1, 0, NBANK, 12),
              ("batched U^H R fp32", 1, 1, NBANK, 12)]
    kmax = max(k for _, _, _, k, _ in shapes)
    out = []
    for name, prec, kind, K, N in shapes:
        dt = torch.complex128 if prec == 0 else torch.complex64
        eb = 16 if prec == 0 else 8
        a = torch.randn((K, n), dtype=dt, device="cuda:0")
        r = torch.randn((N, n), dtype=dt, device="cuda:0") if kind == 1 else None
        o = torch.empty((N, n) if kind == 0 else (N, K), dtype=torch.complex128 if kind == 1 else dt,
                        device="cuda:0")
        sm = torch.randn((N, K), dtype=torch.complex128, device="cuda:0")  # S column-major K x N
        scratch = torch.empty(2 * 1024 * K * 24, dtype=torch.float64, device="cuda:0")

        def call():
            rc = B.LIB.eigcg_debug_gemm(prec, kind, n, K, N, B._ptr(a),
                                        B._ptr(r) if r is not None else None, B._ptr(sm),
                                        B._ptr(o), B._ptr(scratch), scratch.numel())
            if rc != 0:
                raise RuntimeError(f"eigcg_debug_gemm {name}: {rc}")
        call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        nbytes = (K + N) * n * eb
        flops = 8.0 * n * K * N
        peak = FP64_MFMA_PEAK_TF if prec == 0 else FP32_MFMA_PEAK_TF
        out.append({"shape": name, "prec": "f64" if prec == 0 else "f32", "K": K, "N": N, "n": n,
                    "ms": ms, "GBs": nbytes / ms / 1e6, "hbm_frac": nbytes / ms / 1e6 / HBM_PEAK_GBS,
                    "TFLOPs": flops / ms / 1e9, "mfma_frac": flops / ms / 1e9 / peak,
                    "algorithmic_bytes": nbytes, "flops": flops,
                    "arith_intensity": flops / nbytes})
        log(f"{name}: {ms:.3f} ms, {nbytes / ms / 1e6:.0f} GB/s, {flops / ms / 1e9:.1f} TFLOP/s")
        del a, r, o, sm, scratch
        torch.cuda.empty_cache()
    return out


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in STENCIL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(summary=TRAFFIC_SUMMARY, variant=None):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when the stencil sources changed since it was taken or
    the sampled launches ran another stencil variant than the counted ones."""
    import re
    path = os.path.join(ROOT, summary)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_sha256_16:\s*([0-9a-f]{16})", txt)
    t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not t or m.group(1) != source_hash():
        return None
    v = re.search(r"stencil_variant:\s*(\d+)", txt)
    if variant is not None and (not v or int(v.group(1)) != int(variant)):
        return None
    return float(t.group(1))


def cg_pass_samples(B, torch, g, dims, mass, n_iter, variant=0):
    """FP64 CG (one Gaussian right-hand side, seed 1000) for n_iter iterations
    on the given links; the two stencil passes of every HBM_SAMPLE_EVERY-th
    iteration are timed by their own dispatch start/stop events on the
    solver's stream.  Returns the sampled mean durations and the variant."""
    from synthetic import gaussian_rhs
    b = torch.from_numpy(gaussian_rhs(dims, 1000)[None].copy()).to("cuda:0")
    x = torch.zeros_like(b)
    p = B.eigcg_default_params(dims=dims, mass=mass, max_bank=0, max_iter=n_iter, check_every=16,
                               sample_every=HBM_SAMPLE_EVERY, stencil_variant=variant)
    ctx = B.eigcg_create(p, g)
    try:
        B.eigcg_solve(ctx, b, x, TOL, B.EIGCG_MODE_CG)  # stops at n_iter (ENOTCONV)
        s = B.eigcg_kernel_samples(ctx)["f64"]
        s["stencil_variant"] = B.eigcg_layout_info(ctx)["variant64"]
    finally:
        B.eigcg_destroy(ctx)
    return s


def stencil_roofline(B, torch, dims, seed, reps, variant=0, g=None):
    if g is None:
        from synthetic import gauge_field
        U = gauge_field(dims, EPS, seed)
        g = torch.from_numpy(U).to("cuda:0")
        del U
    p = B.eigcg_default_params(dims=dims, mass=-0.5, max_bank=0, stencil_variant=variant)
    ctx = B.eigcg_create(p, g)
    try:
        info = B.eigcg_layout_info(ctx)
        ms_m = B.eigcg_time_kernel(ctx, 0, reps)
        ms_copy = B.eigcg_time_kernel(ctx, 1, reps)
        ms_it = B.eigcg_time_kernel(ctx, 2, max(1, reps // 4))
    finally:
        B.eigcg_destroy(ctx)
    V = info["sites"]
    bytes_m = V * site_bytes_stencil(info["links64_two_rows"])
    bytes_copy = 2 * 16 * 12 * info["plane_stride"]  # one padded FP64 field read + written
    return {
        "sites": V,
        "two_row_links": info["links64_two_rows"],
        "stencil_variant": info["variant64"],
        "variant_ms": info["tune_ms64"],
        "stencil_M_ms": ms_m,
        "stencil_M_GBs": bytes_m / ms_m / 1e6,
        "copy_ms": ms_copy,
        "copy_GBs": bytes_copy / ms_copy / 1e6,
        "cg_iteration_ms": ms_it,
        "bytes_per_launch_M": bytes_m,
    }


BATCH_MASS = -0.58
BATCH_SIZES = (1, 4, 8, 12)
SERVE_FIELDS = (((8, 8, 8, 8), 2), ((16, 16, 16, 32), SEED), ((24, 24, 24, 48), HBM_SEED))
SERVE_MASS = -0.58
SERVE_MAX_ITER = 20000  # per request (inner iterations over all refinement steps)


def batching_leg(B, torch, g, bt, nrhs=12):
    """Plain CG on nrhs right-hand sides in blocks of k columns per stencil
    launch: FP32 inner iteration with FP64 reliable updates every 50
    iterations (and FP64 for k = 1 and 4, for comparison), tol 1e-10."""
    out = []
    for prec in (2, 1, 0):
        for k in BATCH_SIZES:
            if (prec == 0 and k > 4) or (prec == 2 and k == 8):
                continue
            p = B.eigcg_default_params(dims=LATTICE, mass=BATCH_MASS, precision=prec, max_batch=k,
                                       reliable_every=50, max_iter=40000, check_every=32,
                                       max_bank=0, use_graphs=1)
            ctx = B.eigcg_create(p, g)
            try:
                x = torch.zeros_like(bt[:nrhs])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc, st = B.eigcg_solve(ctx, bt[:nrhs], x, TOL, B.EIGCG_MODE_CG)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                info = B.eigcg_layout_info(ctx)
            finally:
                B.eigcg_destroy(ctx)
            r = {"precision": ("fp16-storage+fp64-refinement", "fp32+fp64-reliable")[prec % 2]
                 if prec else "fp64", "k": k,
                 "rhs_per_s": nrhs / dt, "mean_iters": sum(s["iters"] for s in st) / nrhs,
                 "max_true_rel_res": max(s["true_rel_res"] for s in st),
                 "failed": sum(1 for s in st if s["status"] != 0 or s["true_rel_res"] > TOL),
                 "stencil_variant": info["variant32" if prec else "variant64"]}
            if prec == 2:
                r["mean_outer_steps"] = sum(q["outer_steps"] for q in st) / nrhs
            log(f"batching {r['precision']} k={k}: {r['rhs_per_s']:.1f} RHS/s, "
                f"mean iters {r['mean_iters']:.0f}, max res {r['max_true_rel_res']:.1e}")
            out.append(r)
    return out


def serving_leg(B, torch, n_bank_rhs, n_requests, seed=7):
    """Continuous batching over three resident gauge fields (8^4, 16^3x32,
    24^3x48): each field's FP32 bank is grown by mixed-precision eigCG on
    n_bank_rhs right-hand sides (not timed), then a seeded Poisson stream of
    n_requests deflated mixed-precision solves (tol 1e-10) is submitted to the
    server at a saturating rate (throughput, p50/p99 under queueing) and again
    at half the measured capacity (p50/p99 latency); latency = submit to
    completion."""
    import numpy as np
    from synthetic import gauge_field, gaussian_rhs
    rng = np.random.default_rng(seed)
    fields = []
    for dims, fseed in SERVE_FIELDS:
        U = gauge_field(dims, EPS, fseed)
        g = torch.from_numpy(U).to("cuda:0")
        del U
        shape = (dims[3], dims[2], dims[1], dims[0], 4, 3)
        # the bank is grown by FP64 Incremental eigCG (phase 1 of the paper),
        # then held in FP32 by the mixed-precision serving context
        t0 = time.perf_counter()
        p64 = B.eigcg_default_params(dims=dims, mass=SERVE_MASS, nev=NEV, m=M, max_bank=NBANK,
                                     max_iter=SERVE_MAX_ITER, check_every=16)
        ctx64 = B.eigcg_create(p64, g)
        try:
            for i in range(n_bank_rhs):  # one at a time: each RHS is deflated by the bank so far
                b = torch.from_numpy(gaussian_rhs(dims, 7000 + i)).to("cuda:0")[None]
                B.eigcg_solve(ctx64, b, torch.zeros_like(b), TOL, B.EIGCG_MODE_EIGCG)
            l64 = len(B.eigcg_bank_info(ctx64)[0])
            vecs = torch.empty((l64,) + shape, dtype=torch.complex128, device="cuda:0")
            B.eigcg_bank_vectors(ctx64, 0, l64, vecs)
        finally:
            B.eigcg_destroy(ctx64)
        p = B.eigcg_default_params(dims=dims, mass=SERVE_MASS, precision=1, max_batch=12, nev=NEV,
                                   m=M, max_bank=NBANK, reliable_every=50, max_iter=SERVE_MAX_ITER,
                                   check_every=16, use_graphs=1)
        ctx = B.eigcg_create(p, g)
        B.eigcg_bank_load(ctx, vecs)
        del vecs
        torch.cuda.synchronize()
        vals = B.eigcg_bank_info(ctx)[0]
        l = len(vals)
        log(f"serving field {dims}: bank {l} vectors (lowest {vals[0] if l else 0:.3e}) "
            f"in {time.perf_counter() - t0:.1f}s")
        fields.append({"dims": dims, "g": g, "ctx": ctx, "shape": shape, "bank": l})
    # one isolated deflated request per field through the server first
    iso = {}
    srv = B.eigcg_server_create(0)
    try:
        fids = [B.eigcg_server_add(srv, F["ctx"]) for F in fields]
        for k, F in enumerate(fields):
            b = torch.from_numpy(gaussian_rhs(F["dims"], 8000 + k)).to("cuda:0")[None]
            tk = B.eigcg_submit(srv, fids[k], b, torch.zeros_like(b), TOL)
            B.eigcg_server_drain(srv)
            rc, st = B.eigcg_poll(srv, tk)
            iso[k] = st["seconds"]
            log(f"serving isolated request on {F['dims']}: rc {rc} {st['seconds'] * 1e3:.0f} ms, "
                f"iters {st['iters']}, outer {st['outer_steps']}, res {st['true_rel_res']:.1e}")
    finally:
        B.eigcg_server_destroy(srv)
    # requests: field chosen uniformly, right-hand sides pre-generated on the device
    which = rng.integers(0, len(fields), n_requests)
    reqs = []
    for i, f in enumerate(which):
        F = fields[f]
        b = torch.from_numpy(gaussian_rhs(F["dims"], 9000 + i)).to("cuda:0")[None]
        reqs.append((int(f), b, torch.zeros_like(b)))
    torch.cuda.synchronize()
    def stream(idx, mean_gap, label):
        """Submit requests idx with exponential gaps; returns (wall, results)."""
        gaps = rng.exponential(mean_gap, len(idx))
        srv = B.eigcg_server_create(0)
        try:
            fids = [B.eigcg_server_add(srv, F["ctx"]) for F in fields]
            tickets = []
            t0 = time.perf_counter()
            t_next = t_log = t0
            for n, i in enumerate(idx):
                f, b, x = reqs[i]
                t_next += gaps[n]
                while time.perf_counter() < t_next:
                    time.sleep(min(1e-3, max(0.0, t_next - time.perf_counter())))
                tickets.append(B.eigcg_submit(srv, fids[f], b, x, TOL))
                if time.perf_counter() - t_log > 5.0:
                    t_log = time.perf_counter()
                    ndone = sum(1 for t in tickets if B.eigcg_poll(srv, t)[0] != B.EIGCG_EBUSY)
                    log(f"serving ({label}): {len(tickets)} submitted, {ndone} done")
            while True:  # drain with progress lines
                ndone = sum(1 for t in tickets if B.eigcg_poll(srv, t)[0] != B.EIGCG_EBUSY)
                if ndone == len(tickets):
                    break
                if time.perf_counter() - t_log > 5.0:
                    t_log = time.perf_counter()
                    log(f"serving ({label}): all {len(tickets)} submitted, {ndone} done")
                time.sleep(2e-3)
            t1 = time.perf_counter()
            return t1 - t0, [B.eigcg_poll(srv, t) for t in tickets]
        finally:
            B.eigcg_server_destroy(srv)

    # saturating load (throughput): mean gap = 1/4 of the mean isolated latency
    mean_iso = float(np.mean([iso[int(f)] for f in which]))
    all_idx = list(range(n_requests))
    wall, res = stream(all_idx, mean_iso / 4.0, "saturated")
    t0, t1 = 0.0, wall
    # latency at 50 %, 80 % and 95 % of the measured capacity: every other
    # request of the same mix again, Poisson arrivals at that rate
    loads = []
    half_idx = all_idx[::2]
    for frac in (0.5, 0.8, 0.95):
        rate = frac * n_requests / wall
        wall_l, res_l = stream(half_idx, 1.0 / rate, f"{int(frac * 100)}% load")
        lat_l = np.array([st["seconds"] for _, st in res_l])
        loads.append({"load": frac, "requests": len(half_idx), "offered_rhs_per_s": rate,
                      "rhs_per_s": len(half_idx) / wall_l,
                      "p50_s": float(np.percentile(lat_l, 50)),
                      "p99_s": float(np.percentile(lat_l, 99)),
                      "failed": int(sum(1 for rc, st in res_l
                                        if rc != 0 or st["true_rel_res"] > TOL))})
        log(f"serving at {int(frac * 100)}% of capacity: p50 {loads[-1]['p50_s'] * 1e3:.0f} ms "
            f"p99 {loads[-1]['p99_s'] * 1e3:.0f} ms")
    light = loads[0]
    lat = np.array([st["seconds"] for _, st in res])
    ok = [rc == 0 and st["true_rel_res"] <= TOL for rc, st in res]
    per_field = []
    for k, F in enumerate(fields):
        sel = which == k
        if sel.any():
            per_field.append({"dims": list(F["dims"]), "bank": F["bank"], "requests": int(sel.sum()),
                              "p50_s": float(np.percentile(lat[sel], 50)),
                              "p99_s": float(np.percentile(lat[sel], 99)),
                              "mean_iters": float(np.mean([res[i][1]["iters"]
                                                           for i in np.nonzero(sel)[0]]))})
    # plain FP64 single-RHS CG on each field (one of its requests' b) as the reference
    plain_s = []
    for k, F in enumerate(fields):
        B.eigcg_destroy(F["ctx"])
        i0 = int(np.nonzero(which == k)[0][0]) if (which == k).any() else 0
        b = reqs[i0][1] if which[i0] == k else torch.from_numpy(
            gaussian_rhs(F["dims"], 9000)).to("cuda:0")[None]
        p = B.eigcg_default_params(dims=F["dims"], mass=SERVE_MASS, max_iter=40000, check_every=32,
                                   max_bank=0)
        ctx = B.eigcg_create(p, F["g"])
        try:
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t = time.perf_counter()
            B.eigcg_solve(ctx, b, x, TOL, B.EIGCG_MODE_CG)
            torch.cuda.synchronize()
            plain_s.append(time.perf_counter() - t)
        finally:
            B.eigcg_destroy(ctx)
    for k, pf in enumerate(per_field):
        pf["plain_fp64_cg_s"] = plain_s[[list(F["dims"]) for F in fields].index(pf["dims"])]
    plain_mix = float(sum(plain_s[f] for f in which))
    growth = serving_from_empty_banks(B, torch, fields, which, reqs, plain_mix)
    out = {"requests": n_requests, "rhs_per_s": n_requests / (t1 - t0), "wall_s": t1 - t0,
           "plain_fp64_cg_same_mix_s": plain_mix, "speedup_vs_plain_fp64_cg": plain_mix / (t1 - t0),
           "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
           "half_load": light,
           "loads": loads,
           "isolated_request_s": {str(list(fields[k]["dims"])): v for k, v in iso.items()},
           "failed": int(len(ok) - sum(ok)),
           "max_true_rel_res": max(st["true_rel_res"] for _, st in res), "per_field": per_field,
           "from_empty_banks": growth}
    log(f"serving: {out['rhs_per_s']:.1f} RHS/s p50 {out['p50_s'] * 1e3:.0f} ms "
        f"p99 {out['p99_s'] * 1e3:.0f} ms failed {out['failed']}, "
        f"{out['speedup_vs_plain_fp64_cg']:.2f}x plain FP64 CG on the same mix")
    return out


SERVE_GROW_EIG = 8  # eigCG requests per field that grow its bank inside the server


def serving_from_empty_banks(B, torch, fields, which, reqs, plain_mix):
    """The same request mix served from empty banks: FP64 contexts, each
    field's first SERVE_GROW_EIG requests are eigCG requests (one step of
    Incremental eigCG each, growing the bank inside the server), the rest
    init-CG with the grown bank; all requests submitted at once, so RHS/s and
    p50/p99 include the bank building."""
    import numpy as np
    ctxs = []
    try:
        for F in fields:
            p = B.eigcg_default_params(dims=F["dims"], mass=SERVE_MASS, nev=NEV, m=M,
                                       max_bank=NBANK, max_batch=12, max_iter=SERVE_MAX_ITER,
                                       check_every=16, use_graphs=1)
            ctxs.append(B.eigcg_create(p, F["g"]))
        seen = [0] * len(fields)
        modes = []
        for f in which:
            modes.append(B.EIGCG_MODE_EIGCG if seen[f] < SERVE_GROW_EIG else B.EIGCG_MODE_INITCG)
            seen[f] += 1
        for _, _, x in reqs:
            x.zero_()
        torch.cuda.synchronize()
        srv = B.eigcg_server_create(0)
        try:
            fids = [B.eigcg_server_add(srv, c) for c in ctxs]
            t0 = t_log = time.perf_counter()
            tickets = [B.eigcg_submit_mode(srv, fids[f], b, x, TOL, modes[i])
                       for i, (f, b, x) in enumerate(reqs)]
            while True:
                ndone = sum(1 for t in tickets if B.eigcg_poll(srv, t)[0] != B.EIGCG_EBUSY)
                if ndone == len(tickets):
                    break
                if time.perf_counter() - t_log > 5.0:
                    t_log = time.perf_counter()
                    log(f"serving from empty banks: {ndone} of {len(tickets)} done")
                time.sleep(2e-3)
            wall = time.perf_counter() - t0
            res = [B.eigcg_poll(srv, t) for t in tickets]
        finally:
            B.eigcg_server_destroy(srv)
        banks = [len(B.eigcg_bank_info(c)[0]) for c in ctxs]
    finally:
        for c in ctxs:
            B.eigcg_destroy(c)
    lat = np.array([st["seconds"] for _, st in res])
    eig = np.array([m == B.EIGCG_MODE_EIGCG for m in modes])
    out = {"requests": len(reqs), "eigcg_requests_per_field": SERVE_GROW_EIG, "precision": "fp64",
           "rhs_per_s": len(reqs) / wall, "wall_s": wall, "banks": banks,
           "speedup_vs_plain_fp64_cg": plain_mix / wall,
           "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
           "eigcg_p50_s": float(np.percentile(lat[eig], 50)),
           "initcg_p50_s": float(np.percentile(lat[~eig], 50)),
           "mean_iters_eigcg": float(np.mean([res[i][1]["iters"] for i in np.nonzero(eig)[0]])),
           "mean_iters_initcg": float(np.mean([res[i][1]["iters"] for i in np.nonzero(~eig)[0]])),
           "failed": int(sum(1 for rc, st in res if rc != 0 or st["true_rel_res"] > TOL)),
           "max_true_rel_res": max(st["true_rel_res"] for _, st in res)}
    log(f"serving from empty banks: {out['rhs_per_s']:.1f} RHS/s (banks {banks}) p50 "
        f"{out['p50_s'] * 1e3:.0f} ms p99 {out['p99_s'] * 1e3:.0f} ms failed {out['failed']}, "
        f"{out['speedup_vs_plain_fp64_cg']:.2f}x plain FP64 CG on the same mix")
    return out


LARGE_LATTICE, LARGE_SEED, LARGE_MASS = (32, 32, 32, 64), 4, -0.58


def large_leg(B, torch, n_bank_rhs=6, n_rhs=12):
    """The largest configuration: 32^3 x 64, a bank grown by FP64 Incremental
    eigCG on n_bank_rhs right-hand sides and held in FP32, then n_rhs deflated
    solves to 1e-10 in one batch of 12 columns with 16-bit (half) inner
    storage, and with FP32 inner iterations, against plain FP64 CG."""
    from synthetic import gauge_field, gaussian_rhs
    dims = LARGE_LATTICE
    t0 = time.perf_counter()
    U = gauge_field(dims, EPS, LARGE_SEED)
    g = torch.from_numpy(U).to("cuda:0")
    del U
    log(f"large lattice {dims}: links in {time.perf_counter() - t0:.0f}s")
    shape = (dims[3], dims[2], dims[1], dims[0], 4, 3)
    p64 = B.eigcg_default_params(dims=dims, mass=LARGE_MASS, nev=NEV, m=M, max_bank=NBANK,
                                 max_iter=20000, check_every=16)
    ctx64 = B.eigcg_create(p64, g)
    t0 = time.perf_counter()
    try:
        for i in range(n_bank_rhs):
            b = torch.from_numpy(gaussian_rhs(dims, 7500 + i)).to("cuda:0")[None]
            rc, st = B.eigcg_solve(ctx64, b, torch.zeros_like(b), TOL, B.EIGCG_MODE_EIGCG)
            log(f"large lattice bank: RHS {i} {st[0]['iters']} iterations")
        l = len(B.eigcg_bank_info(ctx64)[0])
        vecs = torch.empty((l,) + shape, dtype=torch.complex128, device="cuda:0")
        B.eigcg_bank_vectors(ctx64, 0, l, vecs)
        # plain FP64 single-RHS CG reference on the first solve's right-hand side
        bt = torch.stack([torch.from_numpy(gaussian_rhs(dims, 9500 + i)) for i in range(n_rhs)]).to("cuda:0")
        x = torch.zeros_like(bt[:1])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rc, stp = B.eigcg_solve(ctx64, bt[:1], x, TOL, B.EIGCG_MODE_CG)
        torch.cuda.synchronize()
        plain_s = time.perf_counter() - t1
    finally:
        B.eigcg_destroy(ctx64)
    log(f"large lattice: bank {l} vectors in {time.perf_counter() - t0:.0f}s; plain FP64 CG "
        f"{plain_s:.2f} s ({stp[0]['iters']} iterations)")
    out = {"lattice": list(dims), "mass": LARGE_MASS, "bank": l, "rhs": n_rhs,
           "plain_fp64_cg_s_per_rhs": plain_s, "plain_fp64_cg_iters": stp[0]["iters"], "runs": []}
    for prec, name in ((2, "half storage, FP32 arithmetic"), (1, "FP32")):
        p = B.eigcg_default_params(dims=dims, mass=LARGE_MASS, precision=prec, max_batch=12,
                                   max_bank=NBANK, reliable_every=50, max_iter=20000,
                                   check_every=16, use_graphs=1)
        ctx = B.eigcg_create(p, g)
        try:
            B.eigcg_bank_load(ctx, vecs)
            x = torch.zeros_like(bt)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rc, st = B.eigcg_solve(ctx, bt, x, TOL, B.EIGCG_MODE_INITCG)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
        finally:
            B.eigcg_destroy(ctx)
        r = {"inner": name, "rhs_per_s": n_rhs / dt, "wall_s": dt,
             "speedup_vs_plain_fp64_cg": (n_rhs / dt) * plain_s,
             "mean_iters": sum(q["iters"] for q in st) / n_rhs,
             "mean_outer_steps": sum(q["outer_steps"] for q in st) / n_rhs,
             "max_true_rel_res": max(q["true_rel_res"] for q in st),
             "failed": sum(1 for q in st if q["status"] != 0 or q["true_rel_res"] > TOL)}
        log(f"large lattice, {name}, 12 columns, deflated: {r['rhs_per_s']:.2f} RHS/s "
            f"({r['speedup_vs_plain_fp64_cg']:.1f}x plain FP64 CG), mean iters {r['mean_iters']:.0f}, "
            f"outer {r['mean_outer_steps']:.1f}, max res {r['max_true_rel_res']:.1e}")
        out["runs"].append(r)
    del vecs, bt, g
    torch.cuda.empty_cache()
    return out


LARGE_FULL_MASSES = (-0.55, -0.58, -0.60)


def large_full_leg(B, torch, masses=LARGE_FULL_MASSES, n_bank_rhs=24, n_rhs=12, chunk=24):
    """The largest configuration at its full shape: 32^3 x 64, for each of three
    masses a 240-vector bank grown by FP64 Incremental eigCG(10,100) on 24
    right-hand sides and held in FP32 (about 48 GB), then 12 deflated solves
    to 1e-10 in one batch of 12 columns with 16-bit (half) inner storage and
    with FP32 inner iterations, against plain FP64 CG.  The bank moves chunk
    vectors at a time (each re-projected by the Section 4 update) from the
    FP64 context to the half context and from there to the FP32 one, each
    source released after the move, so at most the FP64 bank with its window
    and one FP32 bank are resident together."""
    from synthetic import gauge_field, gaussian_rhs
    dims = LARGE_LATTICE
    U = gauge_field(dims, EPS, LARGE_SEED)
    g = torch.from_numpy(U).to("cuda:0")
    del U
    shape = (dims[3], dims[2], dims[1], dims[0], 4, 3)
    bt = torch.stack([torch.from_numpy(gaussian_rhs(dims, 9500 + i)) for i in range(n_rhs)]).to("cuda:0")
    out = {"lattice": list(dims), "rhs_per_mass": n_rhs, "masses": []}
    for mass in masses:
        t0 = time.perf_counter()
        p64 = B.eigcg_default_params(dims=dims, mass=mass, nev=NEV, m=M, max_bank=NBANK,
                                     max_iter=20000, check_every=16)
        ctx64 = B.eigcg_create(p64, g)
        src = None
        try:
            its = []
            for i in range(n_bank_rhs):
                b = torch.from_numpy(gaussian_rhs(dims, 7500 + i)).to("cuda:0")[None]
                rc, st = B.eigcg_solve(ctx64, b, torch.zeros_like(b), TOL, B.EIGCG_MODE_EIGCG)
                its.append(st[0]["iters"])
                if i % 6 == 5:
                    log(f"large lattice (full shape) mass {mass}: {i + 1} eigCG solves, "
                        f"{time.perf_counter() - t0:.0f}s")
            vals, _ = B.eigcg_bank_info(ctx64)
            l = len(vals)
            t_bank = time.perf_counter() - t0
            log(f"large lattice (full shape) mass {mass}: bank {l} vectors in {t_bank:.0f}s "
                f"(eigCG iterations {its[0]}..{its[-1]})")
            x = torch.zeros_like(bt[:1])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rc, stp = B.eigcg_solve(ctx64, bt[:1], x, TOL, B.EIGCG_MODE_CG)
            torch.cuda.synchronize()
            plain_s = time.perf_counter() - t1
            src = ctx64
            entry = {"mass": mass, "bank": l, "bank_lambda_min": float(vals[0]),
                     "bank_build_s": t_bank, "eigcg_iters": its,
                     "plain_fp64_cg_s_per_rhs": plain_s, "plain_fp64_cg_iters": stp[0]["iters"],
                     "runs": []}
            for prec, name in ((2, "half storage, FP32 arithmetic"), (1, "FP32")):
                p = B.eigcg_default_params(dims=dims, mass=mass, precision=prec, max_batch=12,
                                           max_bank=NBANK, reliable_every=50, max_iter=20000,
                                           check_every=16, use_graphs=1)
                ctx = B.eigcg_create(p, g)
                try:
                    # the bank in chunks from the previous context (FP64 eigCG, then
                    # the half context's FP32 bank), each chunk re-projected by the
                    # Section 4 update; the previous context is then released
                    buf = torch.empty((min(chunk, l),) + shape, dtype=torch.complex128,
                                      device="cuda:0")
                    for q0 in range(0, l, chunk):
                        k = min(chunk, l - q0)
                        B.eigcg_bank_vectors(src, q0, k, buf[:k])
                        B.eigcg_bank_load(ctx, buf[:k])
                    del buf
                    B.eigcg_destroy(src)
                    src = ctx
                    torch.cuda.empty_cache()
                    x = torch.zeros_like(bt)
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    rc, st = B.eigcg_solve(ctx, bt, x, TOL, B.EIGCG_MODE_INITCG)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t1
                except BaseException:
                    if src is not ctx:
                        B.eigcg_destroy(ctx)
                    raise
                r = {"inner": name, "bank": len(B.eigcg_bank_info(ctx)[0]), "rhs_per_s": n_rhs / dt,
                     "wall_s": dt, "speedup_vs_plain_fp64_cg": (n_rhs / dt) * plain_s,
                     "mean_iters": sum(q["iters"] for q in st) / n_rhs,
                     "mean_outer_steps": sum(q["outer_steps"] for q in st) / n_rhs,
                     "max_true_rel_res": max(q["true_rel_res"] for q in st),
                     "failed": sum(1 for q in st if q["status"] != 0 or q["true_rel_res"] > TOL)}
                log(f"large lattice (full shape) mass {mass}, {name}: {r['rhs_per_s']:.2f} RHS/s "
                    f"({r['speedup_vs_plain_fp64_cg']:.1f}x plain FP64 CG, {stp[0]['iters']} "
                    f"iterations), mean iters {r['mean_iters']:.0f}, max res {r['max_true_rel_res']:.1e}")
                entry["runs"].append(r)
        finally:
            if src is not None:
                B.eigcg_destroy(src)
            elif ctx64 is not None:
                B.eigcg_destroy(ctx64)
            torch.cuda.empty_cache()
        out["masses"].append(entry)
    del bt, g
    torch.cuda.empty_cache()
    return out


def cpu_baseline(total_rhs, total_iters, total_restarts, total_deflations, budget_s=10.0):
    """The NumPy oracle timed on this host: the 4^4 workload in full (plain CG
    and eigCG(10, 40) to 1e-8), and bounded segments on the bench lattice: CG
    iterations, one eigCG(10, 100) restart (the oracle's restart coefficients
    and its V (QZ) product) and one init-CG deflation with 240 vectors (stand-in
    vectors for timing only).  RHS/s for the bench workload is extrapolated
    from the GPU run's counts of iterations, restarts and deflations."""
    import platform

    import numpy as np
    from oracle.cg import cg
    from oracle.dirac import WilsonOperator
    from oracle.eigcg import eigcg, restart_coefficients
    from oracle.initcg import galerkin_guess
    from synthetic import gauge_field, gaussian_rhs

    blas_threads = None
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max((d.get("num_threads", 0) for d in threadpool_info()
                            if d.get("user_api") == "blas"), default=None)
    except Exception:  # threadpoolctl missing or no BLAS found
        pass
    out = {"kind": "oracle", "unit": "RHS/s", "blas_threads": blas_threads,
           "host_cores_available": len(os.sched_getaffinity(0))}
    # 4^4 (the small configuration) in full
    U0 = gauge_field((4, 4, 4, 4), 0.3, 0)
    op0 = WilsonOperator(U0, -0.2)
    b0 = gaussian_rhs((4, 4, 4, 4), 1000).reshape(-1)
    t0 = time.perf_counter()
    _, i_cg = cg(op0.A, b0, tol=1e-10)
    t1 = time.perf_counter()
    _, _, _, i_eig = eigcg(op0.A, b0, 10, 40, tol=1e-8)
    t2 = time.perf_counter()
    out["small_4x4x4x4"] = {"cg_s": t1 - t0, "cg_iters": i_cg["iterations"],
                            "eigcg_10_40_s": t2 - t1, "eigcg_iters": i_eig["iterations"]}
    # bench lattice: CG iterations
    U = gauge_field(LATTICE, EPS, SEED)
    op = WilsonOperator(U, MASSES[0])
    b = gaussian_rhs(LATTICE, 1000).reshape(-1)
    n = b.shape[0]
    t0 = time.perf_counter()
    cg(op.A, b, tol=0.0, max_iter=1, true_residual_restarts=0)
    one = time.perf_counter() - t0
    n_it = max(2, min(40, int(budget_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    cg(op.A, b, tol=0.0, max_iter=n_it, true_residual_restarts=0)
    per_iter = (time.perf_counter() - t0) / (n_it + 2)  # + r0 and the final true residual
    # one eigCG(10, 100) restart: coefficients from a 100 x 100 window matrix
    # (built from the 4^4 run's CG scalars: the small eigenproblems cost the
    # same for any lattice), then V <- V (QZ) over 100 window columns of this
    # lattice
    al, be = np.array(i_cg["alpha"][:M]), np.array(i_cg["beta"][:M])
    d = 1.0 / al
    d[1:] += be[1:] / al[:-1]
    off = -np.sqrt(be[1:]) / al[:-1]
    Tm = (np.diag(d) + np.diag(off, 1) + np.diag(off, -1)).astype(np.complex128)
    V = np.empty((n, M), dtype=np.complex128)
    V[:] = (1.0 + 0.5j) / np.sqrt(n)
    t0 = time.perf_counter()
    QZ = restart_coefficients(Tm, NEV)[0]
    V[:, :2 * NEV] = V[:, :M] @ QZ
    t_restart = time.perf_counter() - t0
    del V
    # one init-CG deflation with 240 vectors (eq. (2.1)); the oracle's Galerkin guess
    Ub = np.empty((n, NBANK), dtype=np.complex128)
    Ub[:] = (1.0 - 0.25j) / np.sqrt(n)
    H = np.eye(NBANK, dtype=np.complex128)
    t0 = time.perf_counter()
    galerkin_guess(op.A, Ub, H, b, x_tilde=np.zeros_like(b))
    t_defl = time.perf_counter() - t0
    del Ub
    cpu_model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    total_s = total_iters * per_iter + total_restarts * t_restart + total_deflations * t_defl
    out.update({
        "value": total_rhs / total_s,
        "cores": blas_threads or 1,
        "cpu_model": cpu_model,
        "seconds_per_cg_iteration": per_iter,
        "seconds_per_eigcg_restart": t_restart,
        "seconds_per_deflation_240": t_defl,
        "extrapolated": True,
        "sample": f"4^4 CG + eigCG(10,40) in full; on 16^3x32: {n_it} FP64 CG iterations "
                  f"({per_iter:.3f} s each, A = M^H M; the NumPy stencil runs on one core), one "
                  f"eigCG(10,100) restart ({t_restart:.2f} s) and one 240-vector deflation "
                  f"({t_defl:.2f} s, BLAS threads {blas_threads}); RHS/s extrapolated with the "
                  f"GPU run's {total_iters} iterations, {total_restarts} restarts and "
                  f"{total_deflations} deflations for {total_rhs} RHS (bank updates not included)",
    })
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--baseline-rhs", type=int, default=4)
    ap.add_argument("--n-eig", type=int, default=N_EIG, help="phase-1 RHS per step (profiling)")
    ap.add_argument("--n-defl", type=int, default=N_DEFL, help="phase-2 RHS per step (profiling)")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-batching", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 32^3x64 half-precision leg")
    ap.add_argument("--large-full-only", action="store_true",
                    help="only the 32^3x64 leg at its full shape (240-vector FP32 bank, three "
                         "masses; several minutes)")
    ap.add_argument("--no-schur", action="store_true", help="skip the odd-even preconditioning leg")
    ap.add_argument("--no-auto", action="store_true", help="skip the automatic eigCG/init-CG leg")
    ap.add_argument("--no-bicgstab", action="store_true", help="skip the deflated BiCGSTAB leg")
    ap.add_argument("--bicgstab-only", action="store_true",
                    help="only the deflated BiCGSTAB leg (no timed steps)")
    ap.add_argument("--bicgstab-short", action="store_true",
                    help="with --bicgstab-only: one right-hand side, a bank from 4 eigCG "
                         "solves, BiCGSTAB on M only (short runs for counter collection)")
    ap.add_argument("--no-critical", action="store_true",
                    help="skip the critical-mass leg (m_q = -0.61)")
    ap.add_argument("--no-spectral", action="store_true",
                    help="skip the spectral preconditioning leg")
    ap.add_argument("--spectral-only", action="store_true",
                    help="only the spectral preconditioning leg (no timed steps)")
    ap.add_argument("--restart-rule", choices=tuple(RESTART_RULE), default="fixed",
                    help="init-CG restart threshold of the timed steps: the fixed "
                         "10 u ||A|| or the dynamic cost model")
    ap.add_argument("--serving-only", action="store_true",
                    help="only the serving leg (no timed steps)")
    ap.add_argument("--serve-bank-rhs", type=int, default=N_EIG)
    ap.add_argument("--serve-requests", type=int, default=120)
    ap.add_argument("--sample-every", type=int, default=SAMPLE_EVERY,
                    help="time the stencil passes of every n-th CG iteration of the timed steps")
    ap.add_argument("--defl-batch", type=int, default=DEFL_BATCH,
                    help="phase-2 init-CG right-hand sides solved together in lockstep "
                         "(phase 1 stays one right-hand side at a time)")
    ap.add_argument("--graphs", action="store_true",
                    help="timed steps replay captured CG segments (iterations not event-timed)")
    ap.add_argument("--stencil-variant", type=int, default=0,
                    help="with --roofline-only: force this stencil variant (counter runs "
                         "use the variant the full bench run picked)")
    ap.add_argument("--gemm-only", action="store_true",
                    help="only time the window and deflation contractions (MFMA) at the bench "
                         "lattice's vector length")
    ap.add_argument("--roofline-only", choices=("bench", "hbm"),
                    help="only time the stencil, copy and CG iteration on the bench lattice "
                         "or the 24^3x48 lattice (short runs for counter collection)")
    args = ap.parse_args()
    global restart_rule, sample_every, use_graphs, defl_batch
    restart_rule = RESTART_RULE[args.restart_rule]
    sample_every = args.sample_every
    use_graphs = 1 if args.graphs else 0
    defl_batch = args.defl_batch
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(this build runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0707_0131_amd import binding as B
    from synthetic import gauge_field, gaussian_rhs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.gemm_only:
        log("window and deflation contractions only")
        print(json.dumps({"gemm": gemm_roofline(B, torch)}))
        return
    if args.large_full_only:
        print(json.dumps({"large_lattice_full": large_full_leg(B, torch)}))
        return
    if args.roofline_only:
        dims, seed = (LATTICE, SEED) if args.roofline_only == "bench" else (HBM_LATTICE, HBM_SEED)
        log(f"stencil timings only ({dims})")
        U = gauge_field(dims, EPS, seed)
        g = torch.from_numpy(U).to("cuda:0")
        del U
        out = {"stencil": stencil_roofline(B, torch, dims, seed, 100, args.stencil_variant, g=g)}
        if args.roofline_only == "hbm":
            out["cg_samples"] = cg_pass_samples(B, torch, g, dims, HBM_CG_MASS, HBM_CG_ITERS,
                                                args.stencil_variant)
        print(json.dumps(out))
        return
    log(f"generating {LATTICE} links and {args.n_eig + args.n_defl} right-hand sides")
    U = gauge_field(LATTICE, EPS, SEED)
    g = torch.from_numpy(U).to("cuda:0")
    del U
    n_eig, n_defl = args.n_eig, args.n_defl
    nrhs = n_eig + n_defl
    shape = (LATTICE[3], LATTICE[2], LATTICE[1], LATTICE[0], 4, 3)
    bt = torch.empty((nrhs,) + shape, dtype=torch.complex128, device="cuda:0")
    for i in range(nrhs):
        bt[i].copy_(torch.from_numpy(gaussian_rhs(LATTICE, 1000 + i)))
    xt = torch.zeros_like(bt)
    torch.cuda.synchronize()

    if args.serving_only:
        del bt, xt, g
        torch.cuda.empty_cache()
        print(json.dumps({"serving": serving_leg(B, torch, args.serve_bank_rhs,
                                                 args.serve_requests)}))
        return

    if args.spectral_only:
        print(json.dumps({"spectral": spectral_leg(B, torch, g, bt, xt)}))
        return

    if args.bicgstab_only:
        kw = dict(n_eig=4, n_rhs=1, solvers=BICG_SOLVERS[:2]) if args.bicgstab_short else {}
        print(json.dumps({"bicgstab": bicgstab_leg(B, torch, g, bt, xt, **kw)}))
        return

    for w in range(args.warmup):
        log(f"warmup step {w}")
        run_step(B, torch, g, MASSES[w % len(MASSES)], bt, xt, n_eig)

    steps = []
    torch.cuda.synchronize()
    win0 = time.monotonic_ns()  # timed window on the clock kernel traces use
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = run_step(B, torch, g, MASSES[k % len(MASSES)], bt, xt, n_eig)
        steps.append(r)
        log(f"step {k}: mass {r['mass']} phase1 {r['phase1_s']:.2f}s "
            f"(iters {r['phase1_iters'][0]}..{r['phase1_iters'][-1]}) phase2 {r['phase2_s']:.2f}s "
            f"(mean iters {sum(r['phase2_iters']) / len(r['phase2_iters']):.0f}) "
            f"max res {r['max_true_rel_res']:.1e} failed {r['failed']}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    win1 = time.monotonic_ns()
    total_rhs = nrhs * args.steps
    value = total_rhs / elapsed

    # plain FP64 CG on a sample of the same right-hand sides, same masses
    base = []
    for k in range(min(args.steps, len(MASSES))):
        mass = MASSES[k]
        dt, its, res = plain_cg(B, torch, g, mass, bt[n_eig:], xt[n_eig:], args.baseline_rhs)
        base.append({"mass": mass, "s_per_rhs": dt / args.baseline_rhs, "iters": its,
                     "max_true_rel_res": res,
                     "lambda_max": lambda_max_est(B, torch, g, mass)})
        log(f"plain CG mass {mass}: {dt / args.baseline_rhs:.3f} s/RHS, iters {its}")
    # per-mass RHS/s of the deflated workload vs plain CG
    per_mass = []
    for k, s in enumerate(steps[: len(base)]):
        defl = nrhs / (s["phase1_s"] + s["phase2_s"])
        plain = 1.0 / base[k]["s_per_rhs"]
        per_mass.append({"mass": s["mass"], "deflated_rhs_per_s": defl, "plain_cg_rhs_per_s": plain,
                         "speedup": defl / plain,
                         "phase2_rhs_per_s": n_defl / s["phase2_s"],
                         "phase2_speedup": (n_defl / s["phase2_s"]) / plain,
                         "lambda_max": base[k]["lambda_max"],
                         "bank_lambda_min": s["bank_lambda_min"],
                         "kappa": (base[k]["lambda_max"] / s["bank_lambda_min"]
                                   if s["bank_lambda_min"] else None)})
    plain_all = len(base) / sum(b["s_per_rhs"] for b in base)

    batching = None
    if not args.no_batching:
        batching = batching_leg(B, torch, g, bt)

    auto = None
    if not args.no_auto:
        auto = auto_leg(B, torch, g, bt, xt)
        fixed = [s for s in steps if s["mass"] == auto["mass"]]
        if fixed:
            auto["fixed_plan_rhs_per_s"] = nrhs / (fixed[0]["phase1_s"] + fixed[0]["phase2_s"])

    critical = None
    if not args.no_critical:
        critical = critical_leg(B, torch, g, bt, xt, n_eig=n_eig)

    spectral = None
    if not args.no_spectral:
        spectral = spectral_leg(B, torch, g, bt, xt)

    bicg = None
    if not args.no_bicgstab:
        bicg = bicgstab_leg(B, torch, g, bt, xt)

    odd_even = None
    if not args.no_schur:
        odd_even = schur_leg(B, torch, g, bt, n_eig=n_eig, n_defl=n_defl)

    roof_small = roof_hbm = hbm_samples = None
    if not args.no_roofline:
        log("stencil roofline (bench lattice, MALL-resident)")
        roof_small = stencil_roofline(B, torch, LATTICE, SEED, 200, g=g)
        del g
        torch.cuda.empty_cache()
        log(f"stencil roofline ({HBM_LATTICE}, working set above the 256 MB MALL)")
        U = gauge_field(HBM_LATTICE, EPS, HBM_SEED)
        g_hbm = torch.from_numpy(U).to("cuda:0")
        del U
        roof_hbm = stencil_roofline(B, torch, HBM_LATTICE, HBM_SEED, 100, g=g_hbm)
        log(f"FP64 CG passes sampled on {HBM_LATTICE} ({HBM_CG_ITERS} iterations)")
        hbm_samples = cg_pass_samples(B, torch, g_hbm, HBM_LATTICE, HBM_CG_MASS, HBM_CG_ITERS)
        del g_hbm
        torch.cuda.empty_cache()

    serving = None
    if not args.no_serving:
        del bt, xt
        torch.cuda.empty_cache()
        serving = serving_leg(B, torch, args.serve_bank_rhs, args.serve_requests)

    large = None
    if not args.no_large:
        large = large_leg(B, torch)

    total_iters = sum(sum(s["phase1_iters"]) + sum(s["phase2_iters"]) for s in steps)
    total_restarts = sum(s["phase1_restarts"] for s in steps)
    # a deflation per init-CG solve and per init-CG restart, and one per eigCG solve
    # after the first (the bank is empty before it)
    total_deflations = sum(len(s["phase1_iters"]) - 1 + len(s["phase2_iters"])
                           + s["phase2_restarts"] for s in steps)
    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline (bounded sample)")
        cpu = cpu_baseline(total_rhs, total_iters, total_restarts, total_deflations)

    # dominant kernel: the second stencil pass of every CG iteration (M^H fused
    # with r -= alpha t and ||r||^2), timed live with events on the solver's
    # stream during the timed steps
    n_s = sum(s["samples"]["n"] for s in steps)
    pass2_ms = sum(s["samples"]["n"] * s["samples"]["pass2_ms"] for s in steps) / max(1, n_s)
    pass1_ms = sum(s["samples"]["n"] * s["samples"]["pass1_ms"] for s in steps) / max(1, n_s)
    V = LATTICE[0] * LATTICE[1] * LATTICE[2] * LATTICE[3]
    # per site: t in (192 B), two-row links (384 B), r in and out (2 x 192 B)
    pass2_bytes = V * (192 + 384 + 192 + 192)
    pass1_bytes = V * site_bytes_stencil(True)  # p in, links, t out
    achieved = pass2_bytes / pass2_ms / 1e6 if n_s else None
    traffic = measured_traffic(variant=steps[0]["samples"]["stencil_variant"] if steps else None)
    roof_mall = {
        "bound": "hbm",
        "mall_resident": True,
        "kernel": "k_wilson_pair FP64 M^H pass fused with the CG residual update "
                  "(960 algorithmic B/site, 16^3x32: links, p, t, r and x fit the 256 MB MALL)",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS if achieved else None,
        "traffic": traffic,
        "launch_ms": pass2_ms,
        "stencil_variant": steps[0]["samples"]["stencil_variant"] if steps else None,
        "sampled_launches": n_s,
        "algorithmic_bytes_per_launch": pass2_bytes,
        "timed_region": True,
    }
    roof = roof_mall
    if hbm_samples and hbm_samples["n"] > 0:
        V_h = HBM_LATTICE[0] * HBM_LATTICE[1] * HBM_LATTICE[2] * HBM_LATTICE[3]
        b2 = V_h * (192 + 384 + 192 + 192)
        a_h = b2 / hbm_samples["pass2_ms"] / 1e6
        roof = {
            "bound": "hbm",
            "mall_resident": False,
            "kernel": "k_wilson_pair FP64 M^H pass fused with the CG residual update "
                      "(960 algorithmic B/site) on 24^3x48: working set (links 255 MB + "
                      "4 fields of 127 MB) above the 256 MB MALL",
            "achieved": a_h,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": a_h / HBM_PEAK_GBS,
            "traffic": measured_traffic(TRAFFIC_SUMMARY_HBM, hbm_samples["stencil_variant"]),
            "launch_ms": hbm_samples["pass2_ms"],
            "stencil_variant": hbm_samples["stencil_variant"],
            "sampled_launches": int(hbm_samples["n"]),
            "algorithmic_bytes_per_launch": b2,
            "timed_region": False,
            "pass1_ms": hbm_samples["pass1_ms"],
            "pass1_GBs": V_h * site_bytes_stencil(True) / hbm_samples["pass1_ms"] / 1e6,
        }
    out = {
        "metric": "deflated RHS solves/sec at 1e-10 rel. residual vs plain CG; stencil HBM GB/s; p99",
        "value": value,
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / max(1, args.steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "Incremental eigCG(10,100) on 24 RHS + init-CG (240 vectors) on 100 RHS, "
                        "16^3x32 Wilson, synthetic SU(3) links eps 0.5, FP64, tol 1e-10; eigCG one "
                        f"RHS at a time, init-CG (and the plain-CG baseline) in lockstep batches "
                        f"of {defl_batch}",
            "lockstep_batch": defl_batch,
            "lattice": list(LATTICE),
            "masses": list(MASSES),
            "rhs_per_step": nrhs,
            "init_cg_restart": args.restart_rule,
        },
        "plain_cg_rhs_per_s": plain_all,
        "speedup_vs_plain_cg": value / plain_all,
        "per_mass": per_mass,
        "steps_detail": [{k: v for k, v in s.items()
                          if k not in ("phase1_iters", "phase2_iters", "phase2_first_leg_iters")}
                         | {"phase1_iters": s["phase1_iters"],
                            "phase2_mean_iters": sum(s["phase2_iters"]) / len(s["phase2_iters"]),
                            "phase2_mean_first_leg_iters":
                                sum(s["phase2_first_leg_iters"]) / len(s["phase2_first_leg_iters"])}
                         for s in steps],
        "plain_cg": base,
        "roofline": roof,
        "roofline_mall_resident": roof_mall,
        "timed_window_monotonic_ns": [win0, win1],
        "stencil_pass1": {"launch_ms": pass1_ms, "GBs": pass1_bytes / pass1_ms / 1e6 if n_s else None,
                          "algorithmic_bytes_per_launch": pass1_bytes},
        "batching": batching,
        "odd_even": odd_even,
        "auto_switch": auto,
        "bicgstab": bicg,
        "critical_mass": critical,
        "spectral_preconditioning": spectral,
        "serving": serving,
        "large_lattice": large,
        "stencil_bench_lattice": roof_small,
        "stencil_hbm_lattice": roof_hbm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
