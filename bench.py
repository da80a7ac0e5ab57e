"""Benchmark: converged eigenpairs/sec of nonlinear FEAST on one MI355X.

One step = one full nlfeast_solve of the workload (assembly of T(z_k) for all nodes, batched
LU of all T(z_k), and every NLFEAST iteration: projections, reduced problem, residuals,
triangular solves against the residual block, accumulation, orthonormalisation) with the
coefficient matrices and X0 already resident in HBM.  The factorisation cache is invalidated
before every step so each step pays the LU.

The headline is the largest single-GPU workload, delay8192 (T(l) = l^2 I + l C + K +
exp(-l) E, n = 8192, 24 nodes, m0 = 160) in FP64, with the FP32-LU + FP64-refinement form of
the same problem beside it, the roofline of the dominant kernel (the complex GEMMs of the LU
trailing updates at n = 8192 x 24 nodes, timed with HIP events on the solve stream inside the
timed region), and the CPU oracle timed on a bounded sample of the same workload.  Further
legs: damped4096 (the FP64 mass-spring-damper problem, graph-replayed factorisation), the
eight-region batched qep2048x8 in FP64 and in FP32 + refinement, the node-count sweep,
left eigenvectors and a caller-supplied function.  Every leg reports its converged eigenvalues'
largest relative error against the stored reference set.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--no-cpu] [--headline-only]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64_mfma_tflops": 78.6, "fp32_mfma_tflops": 157.3, "hbm_gbs": 8000.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="delay8192")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline workload in FP64 (the profiled command)")
    ap.add_argument("--leg-steps", type=int, default=5,
                    help="timed steps of every leg beside the headline (at most --steps; one "
                         "warm-up step each), so that the whole run stays within a few minutes")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the damped4096 and eight-region batched (qep2048x8) legs")
    ap.add_argument("--no-nc-sweep", action="store_true",
                    help="skip the sweep over the number of quadrature nodes (quartic1024)")
    ap.add_argument("--no-left", action="store_true",
                    help="skip the left-eigenvector leg on the headline workload")
    ap.add_argument("--no-user-fn", action="store_true",
                    help="skip delay8192 with its exponential supplied as a caller function")
    ap.add_argument("--panel-width", type=int, default=0,
                    help="LU panel width per workgroup, 4..32 (0 = library default)")
    ap.add_argument("--refine-eta", type=float, default=0.05,
                    help="FP32+refine: refinement target ||E_k|| <= eta ||R||")
    ap.add_argument("--graph", type=int, default=1,
                    help="headline and damped4096 legs: 1 (default) replays the factorisation as "
                         "captured hipGraph segments with the trailing updates launched (and timed) "
                         "between them; 0 launches every kernel eagerly")
    ap.add_argument("--lookahead", type=int, default=0,
                    help="blocked LU look-ahead: 1 on, -1 off, 0 library default")
    ap.add_argument("--lu-streams", type=int, default=0,
                    help="node-matrix groups factored on separate streams (0 = library default)")
    ap.add_argument("--fp32-only", action="store_true",
                    help="run only the FP32 LU + FP64 refinement leg of --workload (for kernel traces of "
                         "the precision form) and print its result")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched qep2048x8 leg (for kernel traces of it) and print its result")
    ap.add_argument("--probe-lu", action="store_true",
                    help="counter runs: one 1 GiB device copy (calibration), then one FP64 "
                         "batched blocked LU of the headline shape, nothing else")
    ap.add_argument("--probe-n", type=int, default=8192)
    ap.add_argument("--probe-batch", type=int, default=24)
    ap.add_argument("--probe-c64", action="store_true",
                    help="with --probe-lu: complex64 matrices (the FP32 + refinement factorisation)")
    return ap.parse_args()


def probe_lu(n, bt, c64=False):
    """Counter runs: a plain device copy of known size (to scale the HBM counters), then one
    batched blocked LU of n x n complex128 matrices (the headline: 24 of n = 8192), whose
    trailing-update launches are the dominant kernel's; complex64 with c64 (the factorisation
    of the FP32 + refinement form)."""
    import torch
    import paper_1801_09794_amd as nl
    torch.cuda.set_device(0)
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")     # 1 GiB
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    g = torch.Generator(device="cuda").manual_seed(7)
    dt = torch.complex64 if c64 else torch.complex128
    A = torch.randn((bt, n, n), dtype=dt, device="cuda", generator=g)
    ipiv = torch.empty((bt, n), dtype=torch.int32, device="cuda")
    perm = torch.empty_like(ipiv)
    info = torch.empty(bt, dtype=torch.int32, device="cuda")
    dinv = torch.empty(bt * nl.nlf_lu_inverse_elems(n), dtype=dt, device="cuda")
    nl.nlf_getrf_batched_blocked(A, ipiv, perm, info, dinv)
    torch.cuda.synchronize()
    print(json.dumps(dict(probe="blocked LU " + ("c64" if c64 else "c128"), copy_bytes=2 * (1 << 27) * 8,
                          n=n, batch=bt)))


def source_digest():
    """First 16 hex digits of the SHA-256 of the GEMM and LU sources (the probe's launches
    depend on both)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("gemm.hip", "lu.hip"):
        h.update(open(os.path.join(ROOT, "paper_1801_09794_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(n, batch):
    """HBM traffic per launch of the dominant kernel from the committed counter summary of
    that shape, or None when there is none or the GEMM or LU source changed after the counters
    were taken."""
    path = os.path.join(ROOT, "profiles", "lu_update_c128_n%d_b%d_traffic.txt" % (n, batch))
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256_16", "").split()[0:1] != [source_digest()]:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def load_workload(name):
    import numpy as np
    import workloads as wl
    cfg = wl.CONFIGS[name]
    terms, mats = wl.make_problem(name)
    regions_json = json.load(open(os.path.join(ROOT, "tests", "golden", "contours.json")))[name]["regions"]
    regions = []
    for g in regions_json:
        regions.append(dict(centre=complex(*g["centre"]), a=g["radius"], nc=cfg["nc"],
                            m0=g.get("m0", cfg.get("m0"))))
    X0 = np.concatenate([wl.initial_block(cfg["n"], r["m0"], 2000 + cfg["id"] + i)
                         for i, r in enumerate(regions)], axis=1)
    return cfg, terms, mats, regions, X0


def run_gpu(args, cfg, terms, mats, regions, X0, precision, profile, autotune=0, graph=0, user_fn=None,
            reduced_solver=0, region_streams=0):
    import torch
    import paper_1801_09794_amd as nl
    n = cfg["n"]
    S = nl.NLFEAST(n, 0)
    dmats = [nl.to_colmajor(M, "cuda:0") for M in mats]
    S.set_coeffs(terms, dmats)
    if user_fn is not None:
        S.set_user_function(user_fn)
    quad = nl.NLF_QUAD_TRAPEZOID if cfg.get("quad") == "trapezoid" else nl.NLF_QUAD_GAUSS_LEGENDRE
    S.set_contour(regions, quad_rule=quad)
    X0d = nl.to_colmajor(X0, "cuda:0")
    opts = nl.options(tol=cfg["tol"], precision=precision, max_refine=5, refine_eta=args.refine_eta,
                      lu_streams=args.lu_streams, panel_width=args.panel_width,
                      autotune=autotune, graph=graph, lookahead=args.lookahead, reduced_solver=reduced_solver,
                      region_streams=region_streams)
    for _ in range(args.warmup):
        S.set_contour(regions, quad_rule=quad)
        S.solve(opts, X0d)
    torch.cuda.synchronize()
    nl.nlfeast_set_profiling(S.h, profile)
    prof = None
    outs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S.set_contour(regions, quad_rule=quad)   # invalidate the cached factorisations
        outs.append(S.solve(opts, X0d))
        if profile:
            p = S.profile()
            if prof is None:
                prof = {k: dict(v) for k, v in p.items()}
            else:
                for k, v in p.items():
                    for f in v:
                        prof[k][f] += v[f]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nl.nlfeast_set_profiling(S.h, False)
    out = outs[-1]
    S.close()
    return (t1 - t0) / args.steps, out, prof


def matched_rel_errors(lam, ref, scale):
    """Relative differences |lam - ref| / max(|ref|, scale) of two equally long eigenvalue sets,
    paired by minimum-cost assignment; the pairs are returned in order of the reference values
    (real part, then imaginary part)."""
    import numpy as np
    from scipy.optimize import linear_sum_assignment
    cost = np.abs(lam[:, None] - ref[None, :]) / np.maximum(np.abs(ref)[None, :], scale)
    i, j = linear_sum_assignment(cost)
    order = np.lexsort((ref[j].imag, ref[j].real))
    return ref[j][order], cost[i, j][order]


def per_eigenpair(ref, err):
    """[[Re, Im, relative error], ...] with 2 significant digits in the error."""
    return [[round(float(v.real), 6), round(float(v.imag), 6), float("%.2g" % e)] for v, e in zip(ref, err)]


def reference_errors(name, regions, out, tol):
    """Relative errors of the converged eigenvalues of each region against the stored brute-force
    reference (tests/golden/contours.json, written by the FP64 oracle), min-cost matched, one
    entry per reference eigenvalue; None when a region's converged count differs from the
    reference count."""
    import numpy as np
    gs = json.load(open(os.path.join(ROOT, "tests", "golden", "contours.json")))[name]["regions"]
    col, rows = 0, []
    for r, g in zip(regions, gs):
        sl = slice(col, col + r["m0"])
        conv = out["inside"][sl] & (out["res"][sl] <= tol)
        lam = out["lam"][sl][conv]
        ref = np.array([complex(*v) for v in g["eigenvalues"]])
        if len(lam) != len(ref):
            return None
        if len(ref):
            rows += per_eigenpair(*matched_rel_errors(lam, ref, g["radius"]))
        col += r["m0"]
    return rows


def reference_error(name, regions, out, tol):
    """Largest of reference_errors (0 when no region holds an eigenvalue)."""
    rows = reference_errors(name, regions, out, tol)
    return None if rows is None else max([e for _, _, e in rows], default=0.0)


def leg_stats(args, name, key, n, nz, regions, cfg, t, o, p):
    c = converged_pairs(o, cfg["tol"])
    f = p["factor"]
    lu_ms = f["ms"] / max(f["launches"], 1)
    tf = 8.0 / 3.0 * n ** 3 * nz / (lu_ms * 1e-3) / 1e12 if lu_ms > 0 else None
    peak = PEAK["fp32_mfma_tflops"] if key == "fp32_refine" else PEAK["fp64_mfma_tflops"]
    g = p["lu_gemm"]
    gt = g["flops"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] > 0 else None
    return {"value": c / t, "unit": "eigenpairs/s", "ms_per_step": t * 1e3, "converged": c,
            "spurious_flagged": int(o["spurious"].sum()), "status": int(o["status"]),
            "iterations": [int(v) for v in o["iters"]], "factor_ms": lu_ms, "lu_tflops": tf,
            "lu_frac_peak": tf / peak if tf else None,
            "trailing_gemm_tflops": gt, "trailing_gemm_frac_peak": gt / peak if gt else None,
            # the trailing updates take 3M products in both precisions: 3/4 of the counted flops
            "trailing_gemm_executed_frac_peak": 0.75 * gt / peak if gt else None,
            "trailing_gemm_avg_launch_us": g["ms"] * 1e3 / g["launches"] if g["launches"] else None,
            "max_rel_err_vs_reference": reference_error(name, regions, o, cfg["tol"]),
            **({"rel_err_vs_reference_per_eigenpair": reference_errors(name, regions, o, cfg["tol"])}
               if key == "fp32_refine" else {}),
            "profile_ms_per_step": {k: v["ms"] / args.steps for k, v in p.items()},
            "hbm_kernels": hbm_kernels(p)}


def extra_leg(args, name, description, autotune, graph, plain_fp64=False, reduced_solver=0):
    """A workload beside the headline in FP64 and in FP32 LU + FP64 refinement (same inputs,
    same tolerance), with the speedup of the precision form over FP64 on this workload and the
    converged eigenvalues checked against the stored reference.  plain_fp64: also the plain
    FP64 path on the same inputs (regions one after another on one stream, eager launches, no
    tuner), the baseline the batched precision form is measured against."""
    import paper_1801_09794_amd as nl
    cfg, terms, mats, regions, X0 = load_workload(name)
    n, nz = cfg["n"], sum(r["nc"] for r in regions)
    out = {"workload": description % dict(n=n, m0=[r["m0"] for r in regions], nc=cfg["nc"], nz=nz,
                                          tol=cfg["tol"], inside=cfg.get("inside") or 0)}
    outs = {}
    for key, prec in (("fp64", nl.NLF_PREC_FP64), ("fp32_refine", nl.NLF_PREC_FP32_REFINE)):
        t, o, p = run_gpu(args, cfg, terms, mats, regions, X0, prec, True, autotune=autotune, graph=graph,
                          reduced_solver=reduced_solver)
        out[key] = leg_stats(args, name, key, n, nz, regions, cfg, t, o, p)
        outs[key] = o
    out["fp32_refine"]["max_rel_eig_diff_vs_fp64"] = eig_diff(outs["fp32_refine"], outs["fp64"], cfg["tol"],
                                                              min(r["a"] for r in regions))
    out["fp32_refine"]["rel_eig_diff_vs_fp64_per_eigenpair"] = eig_diffs(
        outs["fp32_refine"], outs["fp64"], cfg["tol"], min(r["a"] for r in regions))
    out["fp32_refine_speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / out["fp32_refine"]["ms_per_step"]
    out["fp32_refine_vs_fp64_eigenpairs_per_s"] = out["fp32_refine"]["value"] / out["fp64"]["value"]
    if plain_fp64:
        t, o, p = run_gpu(args, cfg, terms, mats, regions, X0, nl.NLF_PREC_FP64, True, autotune=0, graph=0,
                          region_streams=1)
        out["fp64_plain"] = leg_stats(args, name, "fp64", n, nz, regions, cfg, t, o, p)
        out["fp64_plain"]["launch"] = ("regions one after another on one stream, eager launches, default LU "
                                       "parameters, companion linearisation of the reduced problem")
        out["batched_fp32_refine_vs_plain_fp64_eigenpairs_per_s"] = out["fp32_refine"]["value"] / out["fp64_plain"]["value"]
    return out


def user_function_leg(args):
    """Caller-supplied scalar functions and the contour-integral reduced solve: delay8192 with its
    exponential handed over as a Python function through the C ABI (evaluated on the host at
    the nodes, the Ritz values and the reduced contour's points), FP32 LU + FP64 refinement;
    converged eigenvalues against the stored reference."""
    import numpy as np
    import paper_1801_09794_amd as nl
    cfg, terms, mats, regions, X0 = load_workload("delay8192")
    uterms = [(k, p) if k != "exp" else ("fn", p) for k, p in terms]

    def expo(j, tau, z, want_deriv):
        e = np.exp(-tau * z)
        return e, (-tau * e if want_deriv else None)

    t, o, p = run_gpu(args, cfg, uterms, mats, regions, X0, nl.NLF_PREC_FP32_REFINE, True, user_fn=expo)
    c = converged_pairs(o, cfg["tol"])
    return {"workload": "delay8192 with exp(-l) supplied as a caller function (contour-integral reduced "
                        "solve: 96 points on the 1.5x circle, block Hankel moments, Newton), FP32 LU + FP64 "
                        "refinement, n=%d, m0=%d, %d nodes" % (cfg["n"], regions[0]["m0"], cfg["nc"]),
            "value": c / t, "unit": "eigenpairs/s", "ms_per_step": t * 1e3, "converged": c,
            "iterations": [int(v) for v in o["iters"]],
            "max_rel_err_vs_reference": reference_error("delay8192", regions, o, cfg["tol"]),
            "host_reduced_ms_per_step": p["host_reduced"]["ms"] / args.steps,
            "factor_ms": p["factor"]["ms"] / args.steps}


def left_leg(args):
    """Left eigenvectors (eigentriples) of damped4096: after one right solve, each left
    solve runs Algorithm 1 on the adjoint function with the cached factors (no factorisation);
    left eigenpairs per second, the largest ||T(lambda)^H y||, and the distance of the left
    eigenvalues from the right ones."""
    import numpy as np
    import torch
    import paper_1801_09794_amd as nl
    cfg, terms, mats, regions, X0 = load_workload("damped4096")
    S = nl.NLFEAST(cfg["n"], 0)
    S.set_coeffs(terms, [nl.to_colmajor(M, "cuda:0") for M in mats])
    S.set_contour(regions)
    opts = nl.options(tol=cfg["tol"], precision=nl.NLF_PREC_FP64, graph=args.graph)
    right = S.solve(opts, nl.to_colmajor(X0, "cuda:0"))
    Y0 = nl.to_colmajor(np.conj(X0), "cuda:0")
    for _ in range(args.warmup):
        S.solve(opts, Y0, left=True)
    nl.nlfeast_set_profiling(S.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fac = 0
    for _ in range(args.steps):
        left = S.solve(opts, Y0, left=True)
        fac += S.profile()["factor"]["launches"]
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    S.close()
    ok = left["inside"] & (left["res"] <= cfg["tol"])
    c = int(np.sum(ok))
    return {"workload": "left eigenvectors of %s after its right solve (adjoint problem on the conjugate "
                        "contour, cached factors through adjoint solves), FP64" % "damped4096",
            "value": c / t, "unit": "left eigenpairs/s", "ms_per_step": t * 1e3, "converged": c,
            "iterations": [int(v) for v in left["iters"]], "factorisation_launches": fac,
            "max_left_residual": float(np.max(left["res"][ok])) if c else None,
            "max_rel_diff_vs_right_eigenvalues": eig_diff(left, right, cfg["tol"], regions[0]["a"])}


def nc_sweep(args):
    """Sec. 5's observation that more quadrature nodes cost fewer iterations: the quartic1024
    workload (degree 4, n = 1024, one circle holding 15 eigenvalues, m0 = 24) in FP64 with
    n_c = 4, 8, 16, 32 Gauss-Legendre nodes; per n_c the Step 4 executions, the converged
    pairs and the wall time per solve and per iteration."""
    import paper_1801_09794_amd as nl
    cfg, terms, mats, regions, X0 = load_workload("quartic1024")
    inside = len(json.load(open(os.path.join(ROOT, "tests", "golden", "contours.json")))["quartic1024"]
                 ["regions"][0]["eigenvalues"])
    out = {"workload": "quartic1024: T(l) = l^4 I + sum_{j<4} l^j A_j, A_j complex Gaussian/sqrt(n), "
                       "n=%d, circle enclosing %d eigenvalues, m0=%d, FP64, tol %.0e"
                       % (cfg["n"], inside, regions[0]["m0"], cfg["tol"]), "points": []}
    for nc in (4, 8, 16, 32):
        regs = [dict(r, nc=nc) for r in regions]
        t, o, p = run_gpu(args, cfg, terms, mats, regs, X0, nl.NLF_PREC_FP64, True)
        it = int(o["iters"][0])
        out["points"].append({"nc": nc, "iterations": it, "converged": converged_pairs(o, cfg["tol"]),
                              "status": nl.STATUS_NAMES.get(int(o["status"]), int(o["status"])),
                              "ms_per_solve": t * 1e3, "factor_ms": p["factor"]["ms"] / args.steps,
                              "ms_per_iteration": (t * 1e3 - p["factor"]["ms"] / args.steps) / max(it, 1)})
    return out


def hbm_kernels(prof):
    """Achieved bandwidth of the HBM-bound steps (assembly of T(z_k), Step 4 accumulation):
    algorithmic bytes of their launches over their summed event-timed duration."""
    out = {}
    for k, what in (("assemble", "T(z_k) = sum_j f_j(z_k) A_j: read each A_j once, write every node"),
                    ("accumulate", "Q = X rho(Lambda) - sum_k omega_k Y_k (z_k - Lambda)^-1: read n_c + 1 "
                                   "blocks, write one")):
        v = prof.get(k)
        if not v or v["ms"] <= 0 or v["bytes"] <= 0:
            continue
        gbs = v["bytes"] / (v["ms"] * 1e-3) / 1e9
        out[k] = {"what": what, "achieved": gbs, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                  "frac": gbs / PEAK["hbm_gbs"], "bytes_per_launch": v["bytes"] / max(v["launches"], 1),
                  "avg_launch_us": v["ms"] * 1e3 / max(v["launches"], 1)}
    return out


def eig_diffs(a, b, tol, scale):
    """Relative differences between the converged eigenvalues of two solves, matched by
    minimum-cost assignment, one entry per eigenvalue of b (None when the converged counts differ
    or nothing converged)."""
    ca, cb = a["inside"] & (a["res"] <= tol), b["inside"] & (b["res"] <= tol)
    la, lb = a["lam"][ca], b["lam"][cb]
    if len(la) != len(lb) or len(la) == 0:
        return None
    return per_eigenpair(*matched_rel_errors(la, lb, scale))


def eig_diff(a, b, tol, scale):
    """Largest of eig_diffs."""
    rows = eig_diffs(a, b, tol, scale)
    return None if rows is None else max(e for _, _, e in rows)


def converged_pairs(out, tol):
    import numpy as np
    ok = out["inside"] & (out["res"] <= tol)
    return int(np.sum(ok))


def cpu_baseline(cfg, terms, mats, regions, X0, gpu_iters, sample_nodes=2):
    """The oracle (numpy/scipy complex128, as it stands) on a bounded sample of the headline
    workload, extrapolated to the whole solve: the assembly + LU of `sample_nodes` of the n_c
    node matrices, one pass of Steps 1-3 (projections, the reduced problem by the oracle's own
    route, Ritz vectors, block residual), the Step 4 solves against the residual block at the
    sampled nodes, and the Step 5 QR.  Whole solve = n_c LUs + iterations x (Steps 1-3 +
    n_c solves + QR) + one final Steps 1-3."""
    import numpy as np
    import scipy.linalg
    from oracle import nlfeast as onl, problem as pb, quadrature as qd, reduced
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 0) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    P = pb.Problem(terms, mats)
    g = regions[0]
    C = qd.Contour(g["centre"], g["a"])
    z, w = qd.nodes_weights(C, g["nc"])
    m0 = g["m0"]
    t0 = time.perf_counter()
    facs = [scipy.linalg.lu_factor(P.T(zk), check_finite=False) for zk in z[:sample_nodes]]
    t_lu = (time.perf_counter() - t0) / sample_nodes
    Q = onl.orthonormalise(X0[:, :m0])
    t0 = time.perf_counter()
    Ahat = P.project(Q)
    lam_all, Y_all = reduced.solve_reduced(P.terms, Ahat, C)
    sel = reduced.select(lam_all, C, m0)
    lam, Y = lam_all[sel].astype(complex), Y_all[:, sel]
    if not P.is_polynomial:
        for i in range(m0):
            if np.isfinite(lam[i]):
                lam[i], Y[:, i] = reduced.newton_polish(P.terms, Ahat, lam[i], Y[:, i])
    lam = np.where(np.isfinite(lam), lam, 0.0)
    X = Q @ Y
    X /= np.linalg.norm(X, axis=0)
    R = P.block_residual(X, lam)
    t_123 = time.perf_counter() - t0
    t0 = time.perf_counter()
    Qn = onl.step4(facs, X, R, lam, z[:sample_nodes], w[:sample_nodes])
    t_solve = (time.perf_counter() - t0) / sample_nodes
    t0 = time.perf_counter()
    onl.orthonormalise(Qn)
    t_qr = time.perf_counter() - t0
    nodes = len(z)
    est = t_lu * nodes + gpu_iters * (t_123 + nodes * t_solve + t_qr) + t_123
    return est, cores, dict(t_lu=t_lu, t_123=t_123, t_solve=t_solve, t_qr=t_qr, nodes=nodes,
                            sample_lus=sample_nodes, iters=gpu_iters)


def oracle_full_run(name):
    """The oracle's complete run on this workload, if one is stored (tests/golden/oracle_runs.json:
    written once by tests/golden/make_oracle_runs.py on the build host, whose cores it states)."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_runs.json")
    if not os.path.exists(path):
        return None
    e = json.load(open(path)).get(name)
    if not e:
        return None
    return {k: e[k] for k in ("seconds", "converged", "iterations", "cores", "host") if k in e}


def batched_leg(args):
    """The eight-region quadratic: one batched factorisation of all 128 node matrices (tuned
    launch parameters, one hipGraph), regions iterating concurrently with contour-integral
    reduced solves; FP64, FP32 + refinement and the plain FP64 path."""
    return extra_leg(
        args, "qep2048x8",
        "qep2048x8: T(l) = l^2 I + l A1 + A0, n=%(n)d complex Gaussian/sqrt(n), 8 disjoint circles, "
        "m0 %(m0)s, %(nc)d trapezoid nodes each (%(nz)d LUs, one hipGraph, tuned launch "
        "parameters, contour-integral reduced solve with device moments), tol %(tol).0e",
        autotune=1, graph=1, plain_fp64=True, reduced_solver=3)


def main():
    args = parse()
    if args.probe_lu:
        probe_lu(args.probe_n, args.probe_batch, args.probe_c64)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1801_09794_amd as nl
    nl.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.batched_only:
        args.steps = max(1, min(args.steps, args.leg_steps))
        args.warmup = min(args.warmup, 1)
        print(json.dumps({"leg": "batched", "steps": args.steps, "warmup": args.warmup,
                          "result": batched_leg(args)}))
        return
    name = args.workload
    cfg, terms, mats, regions, X0 = load_workload(name)
    n = cfg["n"]
    nnodes = sum(r["nc"] for r in regions)
    if args.fp32_only:
        t32, out32, prof32 = run_gpu(args, cfg, terms, mats, regions, X0, nl.NLF_PREC_FP32_REFINE, True,
                                     graph=args.graph)
        st = leg_stats(args, name, "fp32_refine", n, nnodes, regions, cfg, t32, out32, prof32)
        print(json.dumps({"leg": "fp32_refine", "workload": name, "steps": args.steps, "warmup": args.warmup,
                          "result": st}))
        return

    t64, out64, prof = run_gpu(args, cfg, terms, mats, regions, X0, nl.NLF_PREC_FP64, True, graph=args.graph)
    conv64 = converged_pairs(out64, cfg["tol"])
    value = conv64 / t64
    lu = prof["lu_gemm"]
    lu_tflops = lu["flops"] / (lu["ms"] * 1e-3) / 1e12 if lu["ms"] > 0 else 0.0
    lu_flops_total = 8.0 / 3.0 * n ** 3 * nnodes
    # wall span of assembly + factorisation of all nodes (panels overlap the updates)
    lu_phase_ms = prof["factor"]["ms"] / args.steps
    kinds = ", ".join({"pow": "l^%d", "exp": "exp(-%gl)"}[k] % p for k, p in terms)
    result = {
        "metric": "converged eigenpairs/sec + LU TFLOP/s (% MFMA peak), FP32+refine vs FP64",
        "value": value,
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "%s: T(l) = sum_j f_j(l) A_j with f_j in {%s}, n=%d dense complex128, %d "
                        "region(s), circle enclosing %d eigenvalues, m0=%d, %d Gauss-Legendre nodes, "
                        "tol %.0e, FP64 LU" % (name, kinds, n, len(regions), conv64, regions[0]["m0"],
                                               regions[0]["nc"], cfg["tol"]),
            "n": n, "m0": regions[0]["m0"], "nodes": nnodes, "regions": len(regions),
            "parallelism": "single GPU, nodes batched",
            "launch": "factorisation replayed as hipGraph segments" if args.graph else "eager launches",
        },
        "converged": conv64,
        "spurious_flagged": int(out64["spurious"].sum()),
        "status": int(out64["status"]),
        "iterations": int(out64["iters"][0]),
        "max_rel_err_vs_reference": reference_error(name, regions, out64, cfg["tol"]),
        "lu": {"tflops_phase": lu_flops_total / (lu_phase_ms * 1e-3) / 1e12 if lu_phase_ms > 0 else None,
               "phase_ms": lu_phase_ms,
               "phase_frac_fp64_peak": (lu_flops_total / (lu_phase_ms * 1e-3) / 1e12) / PEAK["fp64_mfma_tflops"]
               if lu_phase_ms > 0 else None,
               "trailing_gemm_tflops": lu_tflops,
               "trailing_gemm_frac_fp64_peak": lu_tflops / PEAK["fp64_mfma_tflops"]},
        "roofline": {
            "kernel": "lu_update_dma_kernel (rank-512 trailing updates of the blocked LU, %d complex128 "
                      "matrices of n = %d: 64 x 64 tiles, operands loaded straight into LDS, complex "
                      "products by the 3M scheme)" % (nnodes, n),
            "bound": "mfma",
            "achieved": lu_tflops if lu["ms"] > 0 else None,
            "peak": PEAK["fp64_mfma_tflops"],
            "unit": "TFLOP/s",
            "frac": lu_tflops / PEAK["fp64_mfma_tflops"] if lu["ms"] > 0 else None,
            "flop_count": "algorithmic: 8 real flops per complex multiply-add (the 4M count); the kernel "
                          "executes 3 real MFMA products per complex one (3M), i.e. 3/4 of these",
            "executed_tflops": 0.75 * lu_tflops if lu["ms"] > 0 else None,
            "executed_frac": 0.75 * lu_tflops / PEAK["fp64_mfma_tflops"] if lu["ms"] > 0 else None,
            "traffic": load_traffic(n, nnodes),
            "traffic_note": "HBM bytes per launch, averaged over the trailing-update launches "
                            "of one FP64 factorisation of this shape, from FETCH_SIZE + "
                            "WRITE_SIZE counters scaled by a 1 GiB copy (profiles/)",
            "algorithmic_bytes_per_launch": lu["bytes"] / max(lu["launches"], 1),
            "launches_per_step": lu["launches"] / args.steps,
            "avg_launch_us": lu["ms"] * 1e3 / max(lu["launches"], 1),
            "flops_per_step": lu["flops"] / args.steps,
        },
        "profile_ms_per_step": {k: v["ms"] / args.steps for k, v in prof.items()},
        "hbm_kernels": hbm_kernels(prof),
    }
    if not args.headline_only and not args.no_fp32:
        t32, out32, prof32 = run_gpu(args, cfg, terms, mats, regions, X0, nl.NLF_PREC_FP32_REFINE, True,
                                     graph=args.graph)
        st = leg_stats(args, name, "fp32_refine", n, nnodes, regions, cfg, t32, out32, prof32)
        st["speedup_vs_fp64"] = t64 / t32
        st["max_rel_eig_diff_vs_fp64"] = eig_diff(out32, out64, cfg["tol"], regions[0]["a"])
        st["rel_eig_diff_vs_fp64_per_eigenpair"] = eig_diffs(out32, out64, cfg["tol"], regions[0]["a"])
        result["fp32_refine"] = st
    if not args.headline_only and not args.no_cpu:
        est, cores, d = cpu_baseline(cfg, terms, mats, regions, X0, int(out64["iters"][0]))
        result["cpu_baseline"] = {
            "value": conv64 / est, "unit": "eigenpairs/s", "cores": cores, "kind": "oracle",
            "sample": "oracle (numpy/scipy complex128) on %s: assembly + LU of %d of the %d node matrices "
                      "(%.2f s each), one pass of Steps 1-3 (%.2f s), the Step 4 solves at the sampled "
                      "nodes (%.2f s per node) and the Step 5 QR (%.2f s); extrapolated to %d LUs + %d "
                      "iterations (the GPU solve's count) + the final Steps 1-3 = %.1f s per solve"
                      % (name, d["sample_lus"], d["nodes"], d["t_lu"], d["t_123"], d["t_solve"], d["t_qr"],
                         d["nodes"], d["iters"], est),
        }
        full = oracle_full_run(name)
        if full:
            result["cpu_baseline"]["full_run_build_host"] = full
    del mats
    if not args.headline_only:
        import copy
        args = copy.copy(args)
        args.steps = max(1, min(args.steps, args.leg_steps))
        args.warmup = min(args.warmup, 1)
        result["legs_steps"] = {"steps": args.steps, "warmup": args.warmup}
        if not args.no_batched and name != "damped4096":
            result["damped4096"] = extra_leg(
                args, "damped4096",
                "damped4096: quadratic mass-spring-damper T(l) = l^2 A2 + l A1 + A0, n=%(n)d dense "
                "complex128, circle enclosing 40 eigenvalues, m0 %(m0)s, %(nc)d Gauss-Legendre nodes, "
                "factorisation replayed as hipGraph segments, tol %(tol).0e", autotune=0, graph=args.graph)
        if not args.no_batched and name != "qep2048x8":
            result["batched"] = batched_leg(args)
        if not args.no_nc_sweep and name != "quartic1024":
            result["nc_sweep"] = nc_sweep(args)
        if not args.no_left:
            result["left_eigenvectors"] = left_leg(args)
        if not args.no_user_fn:
            result["user_function"] = user_function_leg(args)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
