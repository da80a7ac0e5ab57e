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


# ---- the contour-integral reduced solve (caller-supplied functions), host side

def _exp_fn():
    return nl.user_function(lambda j, p, z, d: (np.exp(-p * z), -p * np.exp(-p * z) if d else None))


def _pow_fn():
    """Every term handed over as a caller function z -> z^p."""
    def f(j, p, z, d):
        q = int(p)
        return z ** q, (q * z ** (q - 1) if q > 0 else np.zeros_like(z)) if d else None
    return nl.user_function(f)


def _oracle_exp(tau):
    from oracle import problem as pb
    return pb.ScalarFunction(lambda z: np.exp(-tau * z), lambda z: -tau * np.exp(-tau * z), "exp")


@pytest.mark.parametrize("route", ["user", "forced"])
@pytest.mark.parametrize("shape,m,seed", [((0.2 + 0.1j, 0.6, 0.6), 12, 41), ((-0.1 + 0.3j, 0.7, 0.3), 30, 42)])
def test_contour_reduced_matches_oracle(lib, route, shape, m, seed):
    """Library (pivoted QR of the Hankel matrix) and oracle (SVD) on the same reduced delay
    problem: the same eigenvalues well inside the enlarged ellipse, each a null vector."""
    rng = np.random.default_rng(seed)
    A = [np.eye(m, dtype=complex), wl.cn(rng, (m, m)) / np.sqrt(m), wl.cn(rng, (m, m)) / np.sqrt(m),
         0.3 * wl.cn(rng, (m, m)) / np.sqrt(m)]
    C = qd.Contour(*shape)
    if route == "user":
        terms, fn, method = [("pow", 2), ("pow", 1), ("pow", 0), ("fn", 1.0)], _exp_fn(), 0
    else:
        terms, fn, method = wl.DELAY, None, 1
    lam, Y, found = nl.nlf_reduced_solve_ex(terms, A, C.c, C.a, C.b, m, fn=fn, method=method)
    lam0, _, found0 = reduced.contour_reduced(wl.DELAY[:3] + [("fn", _oracle_exp(1.0))], A, C, m)
    well = lambda l: l[C.radius(l) < 1.2]
    a, b = np.sort_complex(well(lam[found])), np.sort_complex(well(lam0[found0]))
    assert len(a) == len(b) >= 3
    assert np.max(np.abs(a - b)) < 1e-12
    for l, y in zip(lam[found], Y[:, found].T):
        if C.radius(l) < 1.2:
            T = sum(f * Aj for f, Aj in zip([l * l, l, 1.0, np.exp(-l)], A))
            assert np.linalg.norm(T @ y) < 1e-12 * np.linalg.norm(T)
    assert np.linalg.norm(np.linalg.norm(Y, axis=0) - 1) < 1e-12


@pytest.mark.parametrize("m,seed", [(16, 51), (40, 52)])
def test_contour_route_on_a_polynomial_matches_the_companion(lib, m, seed):
    """reduced_solver = 3 takes the contour-integral solve for a polynomial reduced problem too:
    inside the contour its eigenvalues are the exact companion's (method 0), and the oracle's
    contour reading (SVD of the Hankel matrix) finds the same values."""
    rng = np.random.default_rng(seed)
    A = [np.eye(m, dtype=complex), wl.cn(rng, (m, m)) / np.sqrt(m), wl.cn(rng, (m, m)) / np.sqrt(m)]
    C = qd.Contour(0.15 - 0.1j, 0.55)
    lc, Yc, fc = nl.nlf_reduced_solve_ex(wl.QUADRATIC, A, C.c, C.a, C.b, m, method=3)
    lp, _, fp = nl.nlf_reduced_solve_ex(wl.QUADRATIC, A, C.c, C.a, C.b, m, method=0)
    assert fp.all()
    ins = lambda l: np.sort_complex(l[C.inside(l)])
    a, b = ins(lc[fc]), ins(lp)
    assert len(a) == len(b) >= 3
    assert np.max(np.abs(a - b)) < 1e-12
    lo, _, fo = reduced.contour_reduced(wl.QUADRATIC, A, C, m)
    o = ins(lo[fo])
    assert len(o) == len(a) and np.max(np.abs(o - a)) < 1e-12
    for l, y in zip(lc[fc], Yc[:, fc].T):
        if C.inside(l):
            T = l * l * A[0] + l * A[1] + A[2]
            assert np.linalg.norm(T @ y) < 1e-12 * np.linalg.norm(T)


def test_reduced_solver_choice(lib):
    """Method 2 keeps the Taylor route for exponential terms (every pair marked found, the same
    values as nlf_reduced_solve); method 0 takes the contour-integral solve."""
    rng = np.random.default_rng(43)
    m = 14
    A = [np.eye(m, dtype=complex), wl.cn(rng, (m, m)) / np.sqrt(m), wl.cn(rng, (m, m)) / np.sqrt(m),
         0.3 * wl.cn(rng, (m, m)) / np.sqrt(m)]
    C = qd.Contour(0.1 + 0.1j, 0.6)
    lt, _, ft = nl.nlf_reduced_solve_ex(wl.DELAY, A, C.c, C.a, C.b, m, method=2)
    lp, _ = nl.nlf_reduced_solve(wl.DELAY, A, C.c, C.a, C.b, m)
    assert ft.all() and np.max(np.abs(lt - lp)) == 0.0
    lc, _, fc = nl.nlf_reduced_solve_ex(wl.DELAY, A, C.c, C.a, C.b, m, method=0)
    well = lambda l: np.sort_complex(l[C.radius(l) < 1.0])
    assert len(well(lc[fc])) == len(well(lt)) >= 2
    assert np.max(np.abs(well(lc[fc]) - well(lt))) < 1e-12


def test_contour_reduced_solve_is_reproducible(lib):
    """The moments are summed in an order fixed by the point index and the thread count, so
    repeated calls give bitwise-identical pairs (iteration counts do not vary between runs)."""
    rng = np.random.default_rng(42)
    m = 40
    A = [np.eye(m, dtype=complex), wl.cn(rng, (m, m)) / np.sqrt(m), wl.cn(rng, (m, m)) / np.sqrt(m),
         0.3 * wl.cn(rng, (m, m)) / np.sqrt(m)]
    C = qd.Contour(0.1 + 0.1j, 0.6)
    runs = [nl.nlf_reduced_solve_ex(wl.DELAY, A, C.c, C.a, C.b, m, method=0) for _ in range(5)]
    for lam, Y, found in runs[1:]:
        assert np.array_equal(lam, runs[0][0]) and np.array_equal(Y, runs[0][1])
        assert np.array_equal(found, runs[0][2])


def test_contour_reduced_completion(lib):
    """lambda I - diag(d) through caller functions: three eigenvalues inside the enlarged
    circle are found (e_i vectors), seven completing pairs sit on the enlarged circle with
    vectors orthogonal to everything before them."""
    m = 10
    d = np.array([0.1, -0.5j, 0.9 + 0.3j, 3.0, -4.0, 5j, 2.5 + 2.5j, -3 - 3j, 6.0, 7.0])
    A = [np.eye(m, dtype=complex), -np.diag(d)]
    C = qd.Contour(0.0, 1.0)
    lam, Y, found = nl.nlf_reduced_solve_ex([("fn", 1), ("fn", 0)], A, C.c, C.a, C.b, m, fn=_pow_fn())
    assert found.sum() == 3 and found[:3].all()
    assert np.max(np.abs(np.sort_complex(lam[:3]) - np.sort_complex(d[:3]))) < 1e-13
    assert np.allclose(C.radius(lam[3:]), 1.5)
    assert np.allclose(Y.conj().T @ Y, np.eye(m), atol=1e-12)


def test_contour_reduced_completion_is_orthogonal_to_a_non_normal_span(lib):
    """lambda I - A with A = S diag(d) S^{-1} (S far from unitary): the three eigenvectors found
    are not orthogonal to each other, and every completing vector is orthogonal to their span."""
    m = 12
    rng = np.random.default_rng(31)
    d = np.array([0.1, -0.4j, 0.5 + 0.2j] + list(3.0 + 2.0 * rng.uniform(size=m - 3)))
    S = np.eye(m) + 0.8 * wl.cn(rng, (m, m))
    A = [np.eye(m, dtype=complex), -(S * d[None, :]) @ np.linalg.inv(S)]
    C = qd.Contour(0.0, 1.0)
    lam, Y, found = nl.nlf_reduced_solve_ex([("fn", 1), ("fn", 0)], A, C.c, C.a, C.b, m, fn=_pow_fn())
    assert found.sum() == 3
    assert np.max(np.abs(np.sort_complex(lam[found]) - np.sort_complex(d[:3]))) < 1e-12
    F = Y[:, found]
    assert abs(np.vdot(F[:, 0], F[:, 1])) > 1e-3           # not an orthogonal set
    Qf, _ = np.linalg.qr(F)
    P = Y[:, ~found]
    assert np.linalg.norm(Qf.conj().T @ P) < 1e-12
    assert np.allclose(P.conj().T @ P, np.eye(m - 3), atol=1e-12)


def test_user_function_errors(lib):
    A = [np.eye(4, dtype=complex), -np.diag([0.1, 0.2, 3.0, 4.0])]
    C = qd.Contour(0.0, 1.0)
    def boom(j, p, z, d):
        raise ValueError("no")
    with pytest.raises(nl.NLFError) as e:
        nl.nlf_reduced_solve_ex([("fn", 1), ("pow", 0)], A, C.c, C.a, C.b, 4, fn=nl.user_function(boom))
    assert e.value.status == nl.NLF_ERR_ARG
    with pytest.raises(nl.NLFError) as e:        # a user term with no function
        nl.nlf_reduced_solve_ex([("fn", 1), ("pow", 0)], A, C.c, C.a, C.b, 4)
    assert e.value.status == nl.NLF_ERR_ARG
    with pytest.raises(nl.NLFError) as e:        # the plain entry point takes built-in kinds only
        nl.nlf_reduced_solve([("fn", 1), ("pow", 0)], A, C.c, C.a, C.b, 4)
    assert e.value.status == nl.NLF_ERR_ARG
    with pytest.raises(nl.NLFError) as e:        # the contour solve completes to at most m pairs
        nl.nlf_reduced_solve_ex([("fn", 1), ("pow", 0)], A, C.c, C.a, C.b, 5, fn=_pow_fn())
    assert e.value.status == nl.NLF_ERR_ARG
