"""Host logic of bench.py that needs no GPU: the refusal of several GPUs, the matching of two
eigenvalue sets behind the per-eigenpair error fields, and the gate that drops the committed
HBM-traffic figures once the GEMM or LU source has changed."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_matching_pairs_permuted_sets():
    rng = np.random.default_rng(3)
    ref = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    rel = 10.0 ** rng.uniform(-14, -9, 12)
    # each value moved by its own relative amount, then shuffled
    lam = ref * (1 + rel * np.exp(1j * rng.uniform(0, 2 * np.pi, 12)))
    order = rng.permutation(12)
    got_ref, err = bench.matched_rel_errors(lam[order], ref, 1e-3)
    # returned in order of the reference values (real part, then imaginary part)
    keys = [(v.real, v.imag) for v in got_ref]
    assert keys == sorted(keys)
    by_value = {complex(v): e for v, e in zip(got_ref, err)}
    for v, r in zip(ref, rel):
        assert by_value[complex(v)] == pytest.approx(r, rel=1e-6)


def test_matching_scale_floor_for_values_near_zero():
    ref = np.array([0.0 + 0.0j, 1.0 + 0.0j])
    lam = np.array([1e-8 + 0.0j, 1.0 + 1e-12j])
    _, err = bench.matched_rel_errors(lam, ref, 0.5)
    assert err[0] == pytest.approx(2e-8)      # |1e-8 - 0| / max(0, 0.5)
    assert err[1] == pytest.approx(1e-12)


def test_per_eigenpair_rows_and_count_mismatch():
    lam = np.array([0.25 + 0.5j, -0.125 + 1j, 3.0 + 0j])
    res = np.array([1e-12, 1e-12, 1.0])
    inside = np.array([True, True, True])
    a = {"lam": lam, "res": res, "inside": inside}
    b = {"lam": lam * (1 + 1e-11), "res": res, "inside": inside}
    rows = bench.eig_diffs(a, b, 1e-10, 0.1)
    assert [r[:2] for r in rows] == [[-0.125, 1.0], [0.25, 0.5]]   # the unconverged value is left out
    assert all(r[2] == pytest.approx(1e-11, rel=0.05) for r in rows)
    assert bench.eig_diff(a, b, 1e-10, 0.1) == max(r[2] for r in rows)
    c = dict(b, res=np.array([1e-12, 1.0, 1.0]))
    assert bench.eig_diffs(a, c, 1e-10, 0.1) is None
    assert bench.eig_diff(a, c, 1e-10, 0.1) is None


def test_reference_errors_against_stored_sets():
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "contours.json")))["damped4096"]["regions"][0]
    ref = np.array([complex(*v) for v in g["eigenvalues"]])
    m0 = len(ref) + 4
    lam = np.concatenate([ref[::-1] * (1 + 1e-12), np.full(4, 9.0 + 0j)])
    out = {"lam": lam, "res": np.full(m0, 1e-14),
           "inside": np.array([True] * len(ref) + [False] * 4)}
    rows = bench.reference_errors("damped4096", [{"m0": m0}], out, 1e-10)
    assert len(rows) == len(ref)
    assert bench.reference_error("damped4096", [{"m0": m0}], out, 1e-10) == pytest.approx(1e-12, rel=0.05)
    out["inside"][0] = False     # one converged value fewer than the reference count
    assert bench.reference_errors("damped4096", [{"m0": m0}], out, 1e-10) is None


def test_traffic_figures_follow_the_source_digest(monkeypatch):
    t = bench.load_traffic(8192, 24)
    # FETCH_SIZE + WRITE_SIZE per launch, scaled, at least the algorithmic bytes of the launches
    assert t is not None and t >= 1.82e10
    assert bench.load_traffic(8191, 24) is None                      # no summary for that shape
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 16)
    assert bench.load_traffic(8192, 24) is None                      # sources changed since
