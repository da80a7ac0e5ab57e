"""Write tests/golden/contours.json: the contour (centre, radius) of each named workload
and the brute-force eigenvalues inside it.  Calls only the oracle's brute-force routines
and the seeded generators; nothing here touches the GPU library.

    python tests/golden/make_contours.py [name ...]

Recipes (contour seed 3000 + id):
  qep200      all 400 companion eigenvalues; centre = a seeded pick among them; radius =
              midpoint between the 10th and 11th distances (the centre is the 1st); a
              draw is rejected when the relative gap at that boundary is under 5%.
  damped4096  centre = the eigenvalue nearest i y0, y0 ~ U(0.3, 1.5); the 64 eigenvalues
              nearest the centre from shift-invert Arnoldi on the companion pencil, of which
              the nearest 44 are sharpened by two-sided Rayleigh functional iteration on
              T(lambda) (Arnoldi's residual test on the non-normal companion operator
              leaves eigenvalue errors near 1e-6 here); radius = midpoint between the 40th
              and 41st distances; rejected under a 2% relative gap.
  qep2048x8   8 disjoint circles, region r enclosing p_r eigenvalues with p_r between
              0.55 m0_r and 0.7 m0_r: centre uniform in the disk |c| < 0.8 (the bulk of the
              spectrum); the nearest eigenvalues from shift-invert Arnoldi on the companion
              pencil, sharpened by two steps of two-sided Rayleigh functional iteration on T;
              p_r is the count in that range with the largest relative gap to the next
              eigenvalue, the radius the gap midpoint; rejected under a 2% gap or when two
              circles come closer than 10% of the larger radius.
  quartic1024 all 4n eigenvalues of the degree-4 companion matrix (dense; shift-invert
              Arnoldi is not accurate enough on this operator); centre = the eigenvalue nearest
              a point uniform in |c| < 0.8; the count between 12 and 16 with the largest relative
              gap, radius at the gap midpoint, rejected under a 2% gap; the count + 2 nearest
              sharpened by two steps of two-sided Rayleigh functional iteration on T.
  delay512, delay8192
              centre c = i y0, y0 ~ U(0.3, 1.5); the eigenvalues nearest c from shift-invert
              Arnoldi on the companion form of the Taylor surrogate of T(c + mu) (tail below
              1e-16 on |mu| <= rho, rho widened until it covers them); the count p within 10%
              of the configured count with the largest relative gap to the next eigenvalue,
              radius at the gap midpoint, rejected under a 1% gap; the nearest p + 2 sharpened
              by two steps of two-sided Rayleigh functional iteration on T itself.  delay512
              also stores the winding number of det T along the circle.

Certificates added to a stored entry without redoing its search (the reference values stay as
they are):
  --certify NAME   max_residual = the largest eigen_residual over the stored eigenvalues: the
                   residual of a unit vector taken by inverse iteration at each eigenvalue
                   itself, an upper bound of the smallest singular value of T there.
  --winding NAME   winding_count = the number of eigenvalues inside the circle by the argument
                   principle (det T from LU factors along the circle), with the stored values
                   deflated from the phase and its smooth cubic trend taken out, only to keep
                   the number of samples small without aliasing.
  rational300 A0 - l I + l/(l - sigma) C: all 2n companion eigenvalues of the quadratic
              (l - sigma) T(l); centre = a seeded pick among them with |c| <= 0.9; radius =
              midpoint between the 12th and 13th distances, rejected under a 5% gap.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as wl  # noqa: E402
from oracle import brute, problem as pb, quadrature as qd  # noqa: E402

OUT = os.path.join(HERE, "contours.json")


def ring(lam, centre, k):
    d = np.sort(np.abs(lam - centre))
    return d, 0.5 * (d[k - 1] + d[k]), (d[k] - d[k - 1]) / d[k]


def qep200():
    cfg = wl.CONFIGS["qep200"]
    terms, mats = wl.make_problem("qep200")
    lam = brute.companion_eigs(pb.Problem(terms, mats))
    rng = np.random.default_rng(3000 + cfg["id"])
    while True:
        c = lam[rng.integers(len(lam))]
        _, r, gap = ring(lam, c, cfg["inside"])
        if gap >= 0.05:
            break
    inside = lam[np.abs(lam - c) < r]
    return dict(regions=[dict(centre=[c.real, c.imag], radius=r, gap=gap,
                              eigenvalues=[[v.real, v.imag] for v in inside])])


def damped4096():
    cfg = wl.CONFIGS["damped4096"]
    terms, mats = wl.make_problem("damped4096")
    P = pb.Problem(terms, mats)
    rng = np.random.default_rng(3000 + cfg["id"])
    while True:
        y0 = rng.uniform(0.3, 1.5)
        near = brute.companion_eigs_near(P, 1j * y0, 8)
        c, _ = brute.refine_eigenvalue(P, near[0])
        lam = brute.companion_eigs_near(P, c, 64)[:44]
        ref = [brute.refine_eigenvalue(P, l) for l in lam]
        lam = np.array([l for l, _ in ref])
        resid = max(rr for _, rr in ref)
        d, r, gap = ring(lam, c, cfg["inside"])
        if gap >= 0.02:
            break
    inside = lam[np.abs(lam - c) < r]
    return dict(regions=[dict(centre=[c.real, c.imag], radius=r, gap=gap, max_residual=resid,
                              eigenvalues=[[v.real, v.imag] for v in inside])])


def qep2048x8():
    cfg = wl.CONFIGS["qep2048x8"]
    terms, mats = wl.make_problem("qep2048x8")
    P = pb.Problem(terms, mats)
    rng = np.random.default_rng(3000 + cfg["id"])
    regions = []
    for m0 in cfg["m0s"]:
        plo, phi = int(round(0.55 * m0)), int(round(0.7 * m0))
        while True:
            c = 0.8 * np.sqrt(rng.uniform()) * np.exp(2j * np.pi * rng.uniform())
            if any(abs(c - complex(*g["centre"])) < 1.1 * 2 * g["radius"] for g in regions):
                continue
            lam = brute.companion_eigs_near(P, c, phi + 8)
            lam = lam[np.argsort(np.abs(lam - c))]
            res = np.zeros(phi + 2)
            for i in range(phi + 2):
                lam[i], res[i] = brute.refine_eigenvalue(P, lam[i], steps=2, seed=i)
            best = max(range(plo, phi + 1), key=lambda k: ring(lam, c, k)[2])
            _, r, gap = ring(lam, c, best)
            if gap >= 0.02 and all(abs(c - complex(*g["centre"])) > 1.1 * (r + g["radius"]) for g in regions):
                break
        inside = lam[np.abs(lam - c) < r]
        regions.append(dict(centre=[c.real, c.imag], radius=r, gap=gap, m0=m0,
                            max_residual=float(res.max()),
                            eigenvalues=[[v.real, v.imag] for v in inside]))
        print("  region m0 %d: %d inside, r %.4g, gap %.3f" % (m0, len(inside), r, gap), flush=True)
    return dict(regions=regions)


def quartic1024():
    cfg = wl.CONFIGS["quartic1024"]
    terms, mats = wl.make_problem("quartic1024")
    P = pb.Problem(terms, mats)
    full = brute.companion_eigs(P)          # all 4n eigenvalues (dense companion, A_4 = I)
    rng = np.random.default_rng(3000 + cfg["id"])
    p0 = cfg["inside"]
    plo, phi = p0 - 2, p0 + 2
    while True:
        z = 0.8 * np.sqrt(rng.uniform()) * np.exp(2j * np.pi * rng.uniform())
        c = full[np.argmin(np.abs(full - z))]
        best = max(range(plo, phi + 1), key=lambda k: ring(full, c, k)[2])
        _, r, gap = ring(full, c, best)
        if gap >= 0.02:
            break
    lam = full[np.argsort(np.abs(full - c))][:best + 2]
    res = np.zeros(len(lam))
    for i in range(len(lam)):
        lam[i], res[i] = brute.refine_eigenvalue(P, lam[i], steps=2, seed=i)
    _, r, gap = ring(lam, c, best)
    inside = lam[np.abs(lam - c) < r]
    return dict(regions=[dict(centre=[c.real, c.imag], radius=r, gap=gap, max_residual=float(res.max()),
                              eigenvalues=[[v.real, v.imag] for v in inside])])


def rational300():
    """Brute force for the rational problem A0 - l I + l/(l - sigma) C: multiplied by
    (l - sigma) it is the quadratic -l^2 I + l (A0 + sigma I + C) - sigma A0 (no eigenvalue at
    sigma while C is non-singular), whose 2n companion eigenvalues are the truth.  The centre is
    a seeded eigenvalue of the cluster around the unit disk (away from the pole's cluster)."""
    cfg = wl.CONFIGS["rational300"]
    terms, mats = wl.make_problem("rational300")
    n, sig = cfg["n"], terms[2][1]
    A0, _, Cm = mats
    quad = pb.Problem([("pow", 2), ("pow", 1), ("pow", 0)], [-np.eye(n), A0 + sig * np.eye(n) + Cm, -sig * A0])
    full = brute.companion_eigs(quad)
    rng = np.random.default_rng(3000 + cfg["id"])
    k = cfg["inside"]
    while True:
        c = full[rng.integers(len(full))]
        if abs(c) > 0.9:
            continue
        _, r, gap = ring(full, c, k)
        if gap >= 0.05:
            break
    inside = full[np.abs(full - c) < r]
    res = [np.linalg.norm(np.linalg.svd(quad.T(v), compute_uv=False)[-1:]) for v in inside]
    return dict(regions=[dict(centre=[c.real, c.imag], radius=r, gap=gap, pole=sig,
                              max_smallest_singular_value=float(max(res)),
                              eigenvalues=[[v.real, v.imag] for v in inside])])


def delay(name, rho):
    cfg = wl.CONFIGS[name]
    terms, mats = wl.make_problem(name)
    P = pb.Problem(terms, mats)
    rng = np.random.default_rng(3000 + cfg["id"])
    p0 = cfg["inside"]
    plo, phi = int(round(0.9 * p0)), int(round(1.1 * p0))
    k = phi + max(10, phi // 8)
    while True:
        c = 1j * rng.uniform(0.3, 1.5)
        while True:
            t0 = time.time()
            lam = brute.eigs_near(P, c, k, rho)
            dmax = float(np.max(np.abs(lam - c)))
            print("  centre %s rho %.3g: %d nearest within %.4g (%.0fs)" % (c, rho, k, dmax, time.time() - t0),
                  flush=True)
            if dmax <= rho / 1.2:
                break
            rho = 1.5 * 1.2 * dmax          # the surrogate must cover the k nearest: widen it
        lam = lam[np.argsort(np.abs(lam - c))]
        p = max(range(plo, phi + 1), key=lambda q: ring(lam, c, q)[2])
        _, r, gap = ring(lam, c, p)
        if gap < 0.01:
            continue
        res = np.zeros(p + 2)
        for i in range(p + 2):
            lam[i], res[i] = brute.refine_eigenvalue(P, lam[i], steps=2, seed=i)
        _, r, gap = ring(lam, c, p)
        if gap >= 0.01:
            break
    inside = lam[np.abs(lam - c) < r]
    out = dict(centre=[c.real, c.imag], radius=r, gap=gap, max_residual=float(res.max()),
               eigenvalues=[[v.real, v.imag] for v in inside])
    if cfg["n"] <= 1024:
        out["winding_count"] = brute.winding_count(P, qd.Contour(c, r))
    return dict(regions=[out])


RECIPES = {"qep200": qep200, "damped4096": damped4096, "qep2048x8": qep2048x8, "quartic1024": quartic1024,
           "delay512": lambda: delay("delay512", 0.4), "delay8192": lambda: delay("delay8192", 0.15),
           "rational300": rational300}


def certify(name):
    terms, mats = wl.make_problem(name)
    P = pb.Problem(terms, mats)
    data = json.load(open(OUT))
    for g in data[name]["regions"]:
        t0 = time.time()
        res = [brute.eigen_residual(P, complex(*v), seed=i) for i, v in enumerate(g["eigenvalues"])]
        g["max_residual"] = float(max(res))
        print("  %s: %d certified, max residual %.3g (%.0fs)" % (name, len(res), max(res), time.time() - t0),
              flush=True)
    return data[name]


def winding(name):
    terms, mats = wl.make_problem(name)
    P = pb.Problem(terms, mats)
    data = json.load(open(OUT))
    for g in data[name]["regions"]:
        t0 = time.time()
        c = complex(*g["centre"])
        C = qd.Contour(c, g["radius"])
        mu = [complex(*v) for v in g["eigenvalues"]]
        # the smooth part of log g (cubic Taylor polynomial about the centre) is taken out of
        # the phase so that coarse samples do not alias (the count itself does not depend on it)
        trend = brute.phase_trend(P, c, 0.05 * g["radius"], deflate=mu)
        print("  %s: phase trend |a1| r = %.1f, |a2| r^2 = %.1f, |a3| r^3 = %.1f rad (%.0fs)"
              % (name, abs(trend[0]) * g["radius"], abs(trend[1]) * g["radius"] ** 2,
                 abs(trend[2]) * g["radius"] ** 3, time.time() - t0), flush=True)
        g["winding_count"] = brute.winding_count(
            P, C, npts=32, max_step=0.8, deflate=mu, trend=trend,
            log=lambda k: print("    %d evaluations of det T (%.0fs)" % (k, time.time() - t0), flush=True))
        print("  %s: winding count %d, %d stored (%.0fs)" % (name, g["winding_count"], len(mu), time.time() - t0),
              flush=True)
    return data[name]


def store(name, entry):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}   # re-read: merge, not clobber
    data[name] = entry
    json.dump(data, open(OUT, "w"), indent=1)


def main(names):
    for name in names:
        t0 = time.time()
        entry = RECIPES[name]()
        entry["seconds"] = time.time() - t0
        print(name, "regions", len(entry["regions"]),
              "inside", [len(g["eigenvalues"]) for g in entry["regions"]],
              "%.1fs" % entry["seconds"], flush=True)
        store(name, entry)


if __name__ == "__main__":
    if len(sys.argv) == 3 and sys.argv[1] in ("--certify", "--winding"):
        name = sys.argv[2]
        store(name, (certify if sys.argv[1] == "--certify" else winding)(name))
    else:
        main(sys.argv[1:] or list(RECIPES))
