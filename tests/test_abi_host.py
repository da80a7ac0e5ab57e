"""CPU tests of the C-ABI library: it loads without a GPU, exports every function that
include/nlfeast.h declares, and its host-side steps (quadrature, reduced eigenproblem) agree
with the oracle.  No device work is launched here."""
import ctypes

import numpy as np
import pytest

import workloads as wl
from oracle import quadrature as qd, reduced

nl = pytest.importorskip("paper_1801_09794_amd")


@pytest.fixture(scope="module")
def lib():
    try:
        return nl.lib()
    except RuntimeError as e:     # not built: the build check reports it separately
        pytest.skip(str(e))


def test_exports_every_header_function(lib):
    names = nl.header_functions()
    assert len(names) >= 20
    raw = ctypes.CDLL(nl.LIB_PATH)
    for name in names:
        assert hasattr(raw, name), name
    assert set(names) == set(nl._SIGS), "binding signatures out of sync with the header"


def test_options_struct_layout():
    # the C struct: double, 3 x int32, double, uint64, 8 x int32
    assert ctypes.sizeof(nl.Options) == 72
    assert nl.Options.refine_eta.offset == 24 and nl.Options.seed.offset == 32


@pytest.mark.parametrize("rule,name", [(0, "gauss"), (1, "trapezoid")])
@pytest.mark.parametrize("nc", [1, 8, 16, 24, 64])
def test_quadrature_matches_oracle(lib, rule, name, nc):
    C = qd.Contour(-1.55 + 0.1j, 0.05, 0.0035)
    z, w = nl.nlf_quadrature(C.c, C.a, C.b, nc, rule)
    z0, w0 = qd.nodes_weights(C, nc, name)
    assert np.max(np.abs(z - z0)) < 1e-14
    assert np.max(np.abs(w - w0)) < 1e-15 * max(1, np.max(np.abs(w0))) + 1e-17


@pytest.mark.parametrize("m,keep,seed", [(6, 6, 1), (20, 25, 2), (40, 40, 3)])
def test_reduced_quadratic_matches_oracle(lib, m, keep, seed):
    rng = np.random.default_rng(seed)
    A = [wl.cn(rng, (m, m)) for _ in range(3)]
    C = qd.Contour(0.1 + 0.2j, 0.8)
    lam, Y = nl.nlf_reduced_solve(wl.QUADRATIC, A, C.c, C.a, C.b, keep)
    lam0, _ = reduced.solve_reduced(wl.QUADRATIC, A, C)
    sel = reduced.select(lam0, C, keep)
    # same selection, in the same order up to ties of the normalised radius
    assert np.max(np.abs(np.sort_complex(lam) - np.sort_complex(lam0[sel]))) < 1e-11
    for i in range(keep):
        T = sum(lam[i] ** p * Aj for (_, p), Aj in zip(wl.QUADRATIC, A))
        assert np.linalg.norm(T @ Y[:, i]) < 1e-11 * np.linalg.norm(T)
        assert abs(np.linalg.norm(Y[:, i]) - 1) < 1e-13


def test_reduced_cubic_and_delay_match_oracle(lib):
    rng = np.random.default_rng(9)
    terms = [("pow", 3), ("pow", 1), ("pow", 0)]
    A = [wl.cn(rng, (12, 12)) for _ in range(3)]
    C = qd.Contour(0.2, 0.9, 0.5)
    lam, _ = nl.nlf_reduced_solve(terms, A, C.c, C.a, C.b, 10)
    lam0, _ = reduced.solve_reduced(terms, A, C)
    assert np.max(np.abs(np.sort_complex(lam) - np.sort_complex(lam0[reduced.select(lam0, C, 10)]))) < 1e-11
    A = [wl.cn(rng, (25, 25)) for _ in range(4)]
    C = qd.Contour(0.1 + 0.2j, 0.3)
    lam, Y = nl.nlf_reduced_solve(wl.DELAY, A, C.c, C.a, C.b, 8)
    lam0, Y0 = reduced.solve_reduced(wl.DELAY, A, C)
    sel = reduced.select(lam0, C, 8)
    inside = C.inside(lam0[sel])
    for l0, y0 in zip(lam0[sel][inside], Y0[:, sel][:, inside].T):
        l1, _ = reduced.newton_polish(wl.DELAY, A, l0, y0)
        assert np.min(np.abs(lam - l1)) < 1e-12


def test_argument_errors_are_reported(lib):
    with pytest.raises(nl.NLFError) as e:
        nl.nlf_quadrature(0.0, -1.0, 1.0, 8)
    assert e.value.status == nl.NLF_ERR_ARG
    with pytest.raises(nl.NLFError):
        nl.nlf_reduced_solve(wl.QUADRATIC, [np.eye(3)] * 3, 0.0, 1.0, 0.0, 2)
