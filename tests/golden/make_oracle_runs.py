"""Write tests/golden/oracle_runs.json: the oracle's complete run of Algorithm 1 on each named
benchmark workload, with its wall time on the host it ran on.  Calls only the oracle and the
seeded generators; nothing here touches the GPU library.

    python tests/golden/make_oracle_runs.py [name ...]

For each workload and region: the same inputs as the benchmark (coefficients, contour from
contours.json, X0 = initial_block(n, m0, 2000 + id + region), Gauss-Legendre nodes or the
workload's own rule), oracle.nlfeast.solve with its defaults (Taylor reading for exp terms),
and the result: converged eigenvalues inside, spurious values flagged, iterations, largest
residual, seconds from the matrices in host memory to the converged set (factorisations
included), and the BLAS thread count and CPU model of the host.
"""
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as wl  # noqa: E402
from oracle import nlfeast as onl, problem as pb, quadrature as qd  # noqa: E402

OUT = os.path.join(HERE, "oracle_runs.json")


def host():
    model = platform.processor()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 0) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    return model, threads


def run(name):
    cfg = wl.CONFIGS[name]
    terms, mats = wl.make_problem(name)
    P = pb.Problem(terms, mats)
    gs = json.load(open(os.path.join(HERE, "contours.json")))[name]["regions"]
    rule = cfg.get("quad", "gauss")
    regions = []
    t_all = time.perf_counter()
    for ri, g in enumerate(gs):
        m0 = g.get("m0", cfg.get("m0"))
        C = qd.Contour(complex(*g["centre"]), g["radius"])
        z, w = qd.nodes_weights(C, cfg["nc"], rule)
        X0 = wl.initial_block(cfg["n"], m0, 2000 + cfg["id"] + ri)
        t0 = time.perf_counter()
        r = onl.solve(P, C, z, w, X0, m0, cfg["tol"])
        sec = time.perf_counter() - t0
        conv = r.inside & ~r.spurious & (r.res <= cfg["tol"])
        regions.append(dict(m0=m0, iterations=int(r.iters), converged=int(conv.sum()),
                            spurious=int(r.spurious.sum()), stopped=bool(r.converged),
                            max_residual=float(r.res[conv].max()) if conv.any() else None,
                            seconds=sec, eigenvalues=[[v.real, v.imag] for v in r.lam[conv]]))
        print("  %s region %d: %d converged, %d spurious, %d iterations, %.0f s"
              % (name, ri, conv.sum(), r.spurious.sum(), r.iters, sec), flush=True)
    model, threads = host()
    return dict(seconds=time.perf_counter() - t_all, converged=sum(g["converged"] for g in regions),
                iterations=[g["iterations"] for g in regions], cores=threads, host=model,
                regions=regions)


def main(names):
    for name in names:
        entry = run(name)
        data = json.load(open(OUT)) if os.path.exists(OUT) else {}
        data[name] = entry
        json.dump(data, open(OUT, "w"), indent=1)
        print(name, "%.0f s" % entry["seconds"], flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["damped4096", "qep2048x8", "delay8192"])
