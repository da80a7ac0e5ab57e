"""Python binding of libnlfeast.so, the MI355X (gfx950) nonlinear FEAST library.

Argument marshalling only: every step of the computation runs in the HIP library.  The
functions carry the names of the C ABI in include/nlfeast.h.  PyTorch provides device memory
and streams: a column-major n x m complex device matrix is held as a contiguous torch tensor
of shape (m, n) (its transpose), see `to_colmajor` / `from_colmajor`.

The library must be built first (`python -m paper_1801_09794_amd.build`); importing this
package without it raises, so no CPU fallback can run in its place.
"""
import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnlfeast.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "nlfeast.h")

NLF_OK, NLF_ERR_ARG, NLF_ERR_NOMEM, NLF_ERR_DEVICE, NLF_ERR_STATE = 0, 1, 2, 3, 4
NLF_ERR_SINGULAR, NLF_ERR_M0_TOO_SMALL, NLF_ERR_NOT_CONVERGED, NLF_SPURIOUS = 5, 6, 7, 8
NLF_F_POW, NLF_F_EXP, NLF_F_USER = 0, 1, 2
NLF_PREC_FP64, NLF_PREC_FP32_REFINE = 0, 1
NLF_QUAD_GAUSS_LEGENDRE, NLF_QUAD_TRAPEZOID = 0, 1
NLF_C64, NLF_C128 = 0, 1
KERNEL_CLASSES = ["assemble", "lu_gemm", "lu_panel", "lu_trsm", "lu_laswp", "solve", "refine",
                  "residual", "accumulate", "orth", "project", "host_reduced", "factor",
                  "autotune", "lu_rec_gemm", "reduced"]

STATUS_NAMES = {0: "NLF_OK", 1: "NLF_ERR_ARG", 2: "NLF_ERR_NOMEM", 3: "NLF_ERR_DEVICE",
                4: "NLF_ERR_STATE", 5: "NLF_ERR_SINGULAR", 6: "NLF_ERR_M0_TOO_SMALL",
                7: "NLF_ERR_NOT_CONVERGED", 8: "NLF_SPURIOUS"}


class NLFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("refine_eta", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("autotune", ctypes.c_int32), ("verbose", ctypes.c_int32),
                ("lu_streams", ctypes.c_int32), ("panel_width", ctypes.c_int32),
                ("region_streams", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("lookahead", ctypes.c_int32), ("reduced_solver", ctypes.c_int32)]


def options(tol=1e-10, max_iter=50, precision=NLF_PREC_FP64, max_refine=5, refine_eta=0.05,
            seed=2024, autotune=0, verbose=0, lu_streams=0, panel_width=0, region_streams=0,
            graph=0, lookahead=0, reduced_solver=0):
    return Options(tol, max_iter, precision, max_refine, refine_eta, seed, autotune, verbose,
                   lu_streams, panel_width, region_streams, graph, lookahead, reduced_solver)


# nlfeast_user_fn: (user, term, param, count, z, f, df) -> int32
USER_FN = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                           ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))


def user_function(py_fn, errors=None):
    """Wraps py_fn(term, param, z, want_deriv) -> (f, df) (complex numpy arrays shaped like z;
    df may be None when want_deriv is False) as an nlfeast_user_fn.  Keep the returned object
    alive while the library may call it.  An exception inside py_fn is reported to the
    library as a failure (the call that asked returns NLF_ERR_ARG) and, when `errors` is a
    list, appended to it."""
    def tramp(_user, term, param, count, z, f, df):
        try:
            zz = np.ctypeslib.as_array(z, shape=(2 * count,))
            zc = zz[0::2] + 1j * zz[1::2]
            fv, dv = py_fn(int(term), float(param), zc, bool(df))
            fo = np.ctypeslib.as_array(f, shape=(2 * count,))
            fv = np.broadcast_to(np.asarray(fv, dtype=complex), zc.shape)
            fo[0::2], fo[1::2] = fv.real, fv.imag
            if df:
                do = np.ctypeslib.as_array(df, shape=(2 * count,))
                dv = np.broadcast_to(np.asarray(dv, dtype=complex), zc.shape)
                do[0::2], do[1::2] = dv.real, dv.imag
            return 0
        except Exception as e:   # noqa: BLE001 - reported to the library as a failure
            if errors is not None:
                errors.append(e)
            return 1
    return USER_FN(tramp)


_lib = None

c_i64, c_i32, c_dbl, c_vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
P_i32, P_dbl = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
P_vp = ctypes.POINTER(ctypes.c_void_p)

_SIGS = {
    "nlfeast_create": (c_i32, [ctypes.POINTER(c_vp), c_i64, ctypes.c_int, c_vp]),
    "nlfeast_set_coeffs": (c_i32, [c_vp, c_i32, P_i32, P_dbl, P_vp, c_i64]),
    "nlfeast_set_contour": (c_i32, [c_vp, c_i32, P_dbl, P_dbl, P_i32, P_i32, c_i32]),
    "nlfeast_workspace_size": (c_i32, [c_vp, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_size_t)]),
    "nlfeast_solve": (c_i32, [c_vp, ctypes.POINTER(Options), c_vp, ctypes.c_size_t, c_vp, c_vp,
                              P_dbl, P_dbl, P_i32, P_i32, P_i32]),
    "nlfeast_set_profiling": (c_i32, [c_vp, c_i32]),
    "nlfeast_get_profile": (c_i32, [c_vp, ctypes.POINTER(c_i64), P_dbl, P_dbl, P_dbl]),
    "nlfeast_last_error": (ctypes.c_char_p, [c_vp]),
    "nlfeast_destroy": (None, [c_vp]),
    "nlf_assemble": (c_i32, [c_i64, c_i32, P_i32, P_dbl, P_vp, c_i64, c_i32, P_dbl, c_vp, c_vp,
                             c_i64, c_i64, c_vp]),
    "nlf_getrf_batched": (c_i32, [c_i32, c_i64, c_i32, c_vp, c_i64, c_i64, c_vp, c_vp, c_vp, c_vp]),
    "nlf_getrf_batched_noalloc": (c_i32, [c_i32, c_i64, c_i32, c_vp, c_i64, c_i64, c_vp, c_vp, c_vp, c_vp]),
    "nlf_getrf_batched_blocked": (c_i32, [c_i32, c_i64, c_i32, c_vp, c_i64, c_i64, c_vp, c_vp, c_vp,
                                          c_vp, c_vp]),
    "nlf_getrs_batched": (c_i32, [c_i32, c_i64, c_i32, c_i32, c_vp, c_i64, c_i64, c_vp, c_vp,
                                  c_i64, c_i64, c_vp, c_i64, c_i64, c_vp]),
    "nlf_lu_inverse_elems": (c_i64, [c_i64]),
    "nlf_lu_block_inverses": (c_i32, [c_i32, c_i64, c_i32, c_vp, c_i64, c_i64, c_vp, c_vp]),
    "nlf_getrs_batched_inv": (c_i32, [c_i32, c_i64, c_i32, c_i32, c_vp, c_i64, c_i64, c_vp, c_vp,
                                      c_vp, c_i64, c_i64, c_vp, c_i64, c_i64, c_vp, c_vp]),
    "nlf_gemm_batched": (c_i32, [c_i32, ctypes.c_char, ctypes.c_char, c_i64, c_i64, c_i64, P_dbl,
                                 c_vp, c_i64, c_i64, c_vp, c_i64, c_i64, P_dbl, c_vp, c_i64, c_i64,
                                 c_i32, c_vp]),
    "nlf_gemm_batched_tile": (c_i32, [c_i32, ctypes.c_char, c_i64, c_i64, c_i64, P_dbl, c_vp, c_i64,
                                      c_i64, c_vp, c_i64, c_i64, P_dbl, c_vp, c_i64, c_i64, c_i32,
                                      c_i32, c_i32, c_vp]),
    "nlf_block_residual": (c_i32, [c_i64, c_i32, c_i32, P_i32, P_dbl, P_vp, c_i64, c_vp, c_i64,
                                   P_dbl, c_vp, c_i64, c_vp, c_vp, c_vp]),
    "nlf_accumulate": (c_i32, [c_i64, c_i32, c_i32, c_vp, c_vp, P_dbl, P_dbl, P_dbl, c_vp, c_vp]),
    "nlf_orth_workspace": (c_i64, [c_i64, c_i32]),
    "nlf_orthonormalize": (c_i32, [c_i64, c_i32, c_vp, c_vp, c_vp]),
    "nlf_project_workspace": (c_i64, [c_i64, c_i32, c_i32]),
    "nlf_project": (c_i32, [c_i64, c_i32, c_i32, P_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "nlf_quadrature": (c_i32, [c_dbl, c_dbl, c_dbl, c_dbl, c_i32, c_i32, P_dbl, P_dbl]),
    "nlf_reduced_solve": (c_i32, [c_i32, c_i32, P_i32, P_dbl, P_dbl, c_dbl, c_dbl, c_dbl, c_dbl,
                                  c_i32, P_dbl, c_i32, P_dbl, P_dbl]),
    "nlfeast_set_user_function": (c_i32, [c_vp, USER_FN, c_vp]),
    "nlfeast_solve_left": (c_i32, [c_vp, ctypes.POINTER(Options), c_vp, ctypes.c_size_t, c_vp, c_vp,
                                   P_dbl, P_dbl, P_i32, P_i32, P_i32]),
    "nlf_getrs_batched_inv_adjoint": (c_i32, [c_i32, c_i64, c_i32, c_i32, c_vp, c_i64, c_i64, c_vp, c_vp,
                                              c_vp, c_i64, c_i64, c_vp, c_vp, c_i64, c_i64, c_vp, c_vp]),
    "nlf_reduced_solve_ex": (c_i32, [c_i32, c_i32, P_i32, P_dbl, USER_FN, c_vp, c_i32, P_dbl, c_dbl,
                                     c_dbl, c_dbl, c_dbl, c_i32, P_dbl, c_i32, P_dbl, P_dbl, P_i32]),
}


def lib():
    """The loaded library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libnlfeast.so is not built (python -m paper_1801_09794_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/nlfeast.h."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nlf\w*)\s*\(", src)) - {"nlfeast_status"})


def _check(status, h=None):
    if status != NLF_OK:
        msg = lib().nlfeast_last_error(h)
        raise NLFError(status, msg.decode() if msg else "")


def _arr(a, ctype):
    a = np.ascontiguousarray(a)
    return a, a.ctypes.data_as(ctypes.POINTER(ctype))


def _cplx_pairs(v):
    v = np.asarray(v, dtype=complex).ravel()
    out = np.empty(2 * len(v))
    out[0::2] = v.real
    out[1::2] = v.imag
    return out


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def to_colmajor(A, device="cuda", dtype=None):
    """Device tensor holding the column-major copy of the 2-D array A (shape (cols, rows))."""
    import torch
    A = np.asarray(A)
    t = torch.from_numpy(np.ascontiguousarray(A.T))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device)


def from_colmajor(t):
    """numpy array of the matrix stored column-major in tensor t of shape (cols, rows)."""
    return t.detach().cpu().numpy().T


def _kinds(terms):
    kinds, params = [], []
    for k, p in terms:
        kinds.append({"pow": NLF_F_POW, "exp": NLF_F_EXP, "fn": NLF_F_USER}.get(k, k))
        params.append(float(p))
    return np.array(kinds, dtype=np.int32), np.array(params, dtype=np.float64)


# --------------------------------------------------------------------------- handle API

def nlfeast_create(n, device=0, stream=None):
    h = ctypes.c_void_p()
    _check(lib().nlfeast_create(ctypes.byref(h), int(n), int(device), _stream(stream)))
    return h


def nlfeast_destroy(h):
    lib().nlfeast_destroy(h)


def nlfeast_last_error(h=None):
    r = lib().nlfeast_last_error(h)
    return r.decode() if r else ""


def nlfeast_set_coeffs(h, terms, mats, lda=None):
    """terms: [(kind, param)], kind 'pow'/'exp'; mats: column-major device tensors."""
    kinds, params = _kinds(terms)
    ptrs = (ctypes.c_void_p * len(mats))(*[m.data_ptr() for m in mats])
    lda = lda if lda is not None else mats[0].shape[-1]
    _check(lib().nlfeast_set_coeffs(h, len(mats), kinds.ctypes.data_as(P_i32),
                                    params.ctypes.data_as(P_dbl), ptrs, int(lda)), h)


def nlfeast_set_user_function(h, fn):
    """fn: a USER_FN object (see user_function) or None; the caller keeps it alive."""
    _check(lib().nlfeast_set_user_function(h, fn if fn is not None else USER_FN(), None), h)


def nlfeast_set_contour(h, regions, quad_rule=NLF_QUAD_GAUSS_LEGENDRE):
    """regions: [dict(centre=complex, a=float, b=float (default a), nc=int, m0=int)]."""
    centre = _cplx_pairs([r["centre"] for r in regions])
    axes = np.array([[r["a"], r.get("b", r["a"])] for r in regions], dtype=np.float64).ravel()
    nn = np.array([r["nc"] for r in regions], dtype=np.int32)
    m0 = np.array([r["m0"] for r in regions], dtype=np.int32)
    _check(lib().nlfeast_set_contour(h, len(regions), centre.ctypes.data_as(P_dbl),
                                     axes.ctypes.data_as(P_dbl), nn.ctypes.data_as(P_i32),
                                     m0.ctypes.data_as(P_i32), int(quad_rule)), h)


def nlfeast_workspace_size(h, opts):
    out = ctypes.c_size_t()
    _check(lib().nlfeast_workspace_size(h, ctypes.byref(opts), ctypes.byref(out)), h)
    return out.value


def nlfeast_set_profiling(h, on=True):
    _check(lib().nlfeast_set_profiling(h, int(bool(on))), h)


def nlfeast_get_profile(h):
    K = len(KERNEL_CLASSES)
    la = (ctypes.c_int64 * K)()
    ms, fl, by = (ctypes.c_double * K)(), (ctypes.c_double * K)(), (ctypes.c_double * K)()
    _check(lib().nlfeast_get_profile(h, la, ms, fl, by), h)
    return {c: dict(launches=la[i], ms=ms[i], flops=fl[i], bytes=by[i])
            for i, c in enumerate(KERNEL_CLASSES)}


def nlfeast_solve(h, opts, ws, n, m_total, nreg, X0=None, X_out=None, left=False):
    """Runs Algorithm 1 on every region.  ws: device tensor of at least workspace_size bytes;
    X0: column-major device tensor (sum m0, n) or None.  Returns a dict with status,
    lam (complex), res, inside (bool: strictly inside the contour), spurious (bool: inside and
    identified as a spurious Ritz value), m and iters per region, and X (device tensor).
    left=True calls nlfeast_solve_left: X then holds the left eigenvectors."""
    import torch
    if X_out is None:
        X_out = torch.empty((m_total, n), dtype=torch.complex128, device=ws.device)
    lam = np.zeros(2 * m_total)
    res = np.zeros(m_total)
    ins = np.zeros(m_total, dtype=np.int32)
    mo = np.zeros(nreg, dtype=np.int32)
    it = np.zeros(nreg, dtype=np.int32)
    fn = lib().nlfeast_solve_left if left else lib().nlfeast_solve
    st = fn(h, ctypes.byref(opts), _ptr(ws), ws.numel() * ws.element_size(),
            _ptr(X0), _ptr(X_out), lam.ctypes.data_as(P_dbl),
            res.ctypes.data_as(P_dbl), ins.ctypes.data_as(P_i32),
            mo.ctypes.data_as(P_i32), it.ctypes.data_as(P_i32))
    if st not in (NLF_OK, NLF_SPURIOUS, NLF_ERR_NOT_CONVERGED, NLF_ERR_M0_TOO_SMALL):
        _check(st, h)
    return dict(status=st, lam=lam[0::2] + 1j * lam[1::2], res=res, inside=ins != 0,
                spurious=ins == 2, m=mo, iters=it, X=X_out)


# --------------------------------------------------------------------------- step-level API

def nlf_assemble(terms, mats, z, T64=None, T32=None, stream=None):
    kinds, params = _kinds(terms)
    n = mats[0].shape[-1]
    ptrs = (ctypes.c_void_p * len(mats))(*[m.data_ptr() for m in mats])
    zz = _cplx_pairs(z)
    _check(lib().nlf_assemble(n, len(mats), kinds.ctypes.data_as(P_i32), params.ctypes.data_as(P_dbl),
                              ptrs, n, len(zz) // 2, zz.ctypes.data_as(P_dbl), _ptr(T64), _ptr(T32),
                              n, n * n, _stream(stream)))


def nlf_getrf_batched(A, ipiv, perm, info, stream=None):
    """A: device tensor (batch, n, n) holding column-major matrices, factored in place."""
    import torch
    dtype = NLF_C128 if A.dtype == torch.complex128 else NLF_C64
    batch, n = A.shape[0], A.shape[-1]
    _check(lib().nlf_getrf_batched(dtype, n, batch, _ptr(A), n, n * n, _ptr(ipiv), _ptr(perm),
                                   _ptr(info), _stream(stream)))


def nlf_getrf_batched_noalloc(A, ipiv, perm, info, stream=None):
    """nlf_getrf_batched without any device allocation (the exchange lists use the library's
    fixed per-GPU scratch; 4 n batch <= NLF_NOALLOC_SCRATCH_INTS)."""
    import torch
    dtype = NLF_C128 if A.dtype == torch.complex128 else NLF_C64
    batch, n = A.shape[0], A.shape[-1]
    _check(lib().nlf_getrf_batched_noalloc(dtype, n, batch, _ptr(A), n, n * n, _ptr(ipiv), _ptr(perm),
                                           _ptr(info), _stream(stream)))


NLF_NOALLOC_SCRATCH_INTS = 1 << 20


def nlf_getrf_batched_blocked(A, ipiv, perm, info, dinv, stream=None):
    """Right-looking blocked LU of (batch, n, n) column-major matrices, in place; also writes the
    diagonal-block inverses (batch * nlf_lu_inverse_elems(n) elements) into dinv."""
    import torch
    dtype = NLF_C128 if A.dtype == torch.complex128 else NLF_C64
    batch, n = A.shape[0], A.shape[-1]
    _check(lib().nlf_getrf_batched_blocked(dtype, n, batch, _ptr(A), n, n * n, _ptr(ipiv), _ptr(perm),
                                           _ptr(info), _ptr(dinv), _stream(stream)))


def nlf_getrs_batched(LU, perm, B, X, shared_rhs=False, stream=None):
    """LU: (batch, n, n); B: (nrhs, n) if shared_rhs else (batch, nrhs, n); X: (batch, nrhs, n)."""
    import torch
    dtype = NLF_C128 if LU.dtype == torch.complex128 else NLF_C64
    batch, n = LU.shape[0], LU.shape[-1]
    nrhs = X.shape[-2]
    sB = 0 if shared_rhs else n * nrhs
    _check(lib().nlf_getrs_batched(dtype, n, nrhs, batch, _ptr(LU), n, n * n, _ptr(perm), _ptr(B),
                                   n, sB, _ptr(X), n, n * nrhs, _stream(stream)))


def nlf_lu_inverse_elems(n):
    return lib().nlf_lu_inverse_elems(n)


def nlf_lu_block_inverses(LU, dinv, stream=None):
    """LU: (batch, n, n) factors from nlf_getrf_batched; dinv: batch * nlf_lu_inverse_elems(n)."""
    import torch
    dtype = NLF_C128 if LU.dtype == torch.complex128 else NLF_C64
    batch, n = LU.shape[0], LU.shape[-1]
    _check(lib().nlf_lu_block_inverses(dtype, n, batch, _ptr(LU), n, n * n, _ptr(dinv),
                                       _stream(stream)))


def nlf_getrs_batched_inv(LU, perm, dinv, B, X, tmp, shared_rhs=False, stream=None):
    import torch
    dtype = NLF_C128 if LU.dtype == torch.complex128 else NLF_C64
    batch, n = LU.shape[0], LU.shape[-1]
    nrhs = X.shape[-2]
    sB = 0 if shared_rhs else n * nrhs
    _check(lib().nlf_getrs_batched_inv(dtype, n, nrhs, batch, _ptr(LU), n, n * n, _ptr(perm),
                                       _ptr(dinv), _ptr(B), n, sB, _ptr(X), n, n * nrhs, _ptr(tmp),
                                       _stream(stream)))


def nlf_getrs_batched_inv_adjoint(LU, perm, dinv, B, Z, X, tmp, shared_rhs=False, stream=None):
    """X_b = A_b^{-H} B_b from the factors; Z: scratch shaped like X (may be B when B is not
    shared)."""
    import torch
    dtype = NLF_C128 if LU.dtype == torch.complex128 else NLF_C64
    batch, n = LU.shape[0], LU.shape[-1]
    nrhs = X.shape[-2]
    sB = 0 if shared_rhs else n * nrhs
    _check(lib().nlf_getrs_batched_inv_adjoint(dtype, n, nrhs, batch, _ptr(LU), n, n * n, _ptr(perm),
                                               _ptr(dinv), _ptr(B), n, sB, _ptr(Z), _ptr(X), n, n * nrhs,
                                               _ptr(tmp), _stream(stream)))


def nlf_gemm_batched(opA, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch,
                     stream=None):
    import torch
    dtype = NLF_C128 if C.dtype == torch.complex128 else NLF_C64
    al = np.array([complex(alpha).real, complex(alpha).imag])
    be = np.array([complex(beta).real, complex(beta).imag])
    _check(lib().nlf_gemm_batched(dtype, opA.encode(), b"N", M, N, K, al.ctypes.data_as(P_dbl),
                                  _ptr(A), lda, sA, _ptr(B), ldb, sB, be.ctypes.data_as(P_dbl),
                                  _ptr(C), ldc, sC, batch, _stream(stream)))


def nlf_gemm_batched_tile(opA, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch,
                          tm, tn, stream=None):
    import torch
    dtype = NLF_C128 if C.dtype == torch.complex128 else NLF_C64
    al = np.array([complex(alpha).real, complex(alpha).imag])
    be = np.array([complex(beta).real, complex(beta).imag])
    _check(lib().nlf_gemm_batched_tile(dtype, opA.encode(), M, N, K, al.ctypes.data_as(P_dbl),
                                       _ptr(A), lda, sA, _ptr(B), ldb, sB, be.ctypes.data_as(P_dbl),
                                       _ptr(C), ldc, sC, batch, tm, tn, _stream(stream)))


def nlf_block_residual(terms, mats, X, lam, R, norms, ws, stream=None):
    kinds, params = _kinds(terms)
    n, m = mats[0].shape[-1], X.shape[0]
    ptrs = (ctypes.c_void_p * len(mats))(*[t.data_ptr() for t in mats])
    ll = _cplx_pairs(lam)
    _check(lib().nlf_block_residual(n, m, len(mats), kinds.ctypes.data_as(P_i32),
                                    params.ctypes.data_as(P_dbl), ptrs, n, _ptr(X), n,
                                    ll.ctypes.data_as(P_dbl), _ptr(R), n, _ptr(norms), _ptr(ws),
                                    _stream(stream)))


def nlf_accumulate(X, Y, z, omega, lam, Q, stream=None):
    m, n = X.shape
    zz, ww, ll = _cplx_pairs(z), _cplx_pairs(omega), _cplx_pairs(lam)
    _check(lib().nlf_accumulate(n, m, len(zz) // 2, _ptr(X), _ptr(Y), zz.ctypes.data_as(P_dbl),
                                ww.ctypes.data_as(P_dbl), ll.ctypes.data_as(P_dbl), _ptr(Q),
                                _stream(stream)))


def nlf_orth_workspace(n, m):
    return lib().nlf_orth_workspace(n, m)


def nlf_orthonormalize(Q, ws, stream=None):
    m, n = Q.shape
    _check(lib().nlf_orthonormalize(n, m, _ptr(Q), _ptr(ws), _stream(stream)))


def nlf_project_workspace(n, m, J):
    return lib().nlf_project_workspace(n, m, J)


def nlf_project(mats, Q, W, Ahat, ws, stream=None):
    m, n = Q.shape
    ptrs = (ctypes.c_void_p * len(mats))(*[t.data_ptr() for t in mats])
    _check(lib().nlf_project(n, m, len(mats), ptrs, n, _ptr(Q), _ptr(W), _ptr(Ahat), _ptr(ws),
                             _stream(stream)))


def nlf_quadrature(centre, a, b, nc, rule=NLF_QUAD_GAUSS_LEGENDRE):
    z = np.zeros(2 * nc)
    w = np.zeros(2 * nc)
    c = complex(centre)
    _check(lib().nlf_quadrature(c.real, c.imag, float(a), float(b), int(nc), int(rule),
                                z.ctypes.data_as(P_dbl), w.ctypes.data_as(P_dbl)))
    return z[0::2] + 1j * z[1::2], w[0::2] + 1j * w[1::2]


def nlf_reduced_solve(terms, Ahat, centre, a, b, m_keep, avoid=None):
    """Ahat: list of m x m complex numpy matrices; avoid: values the inversion shift keeps
    away from (e.g. the previous Ritz values).  Returns (lam, Y)."""
    kinds, params = _kinds(terms)
    m = Ahat[0].shape[0]
    A = np.concatenate([np.asfortranarray(M, dtype=complex).ravel(order="F") for M in Ahat])
    Af = np.empty(2 * len(A))
    Af[0::2], Af[1::2] = A.real, A.imag
    lam = np.zeros(2 * m_keep)
    Y = np.zeros(2 * m * m_keep)
    c = complex(centre)
    av = _cplx_pairs([] if avoid is None else avoid)
    _check(lib().nlf_reduced_solve(m, len(Ahat), kinds.ctypes.data_as(P_i32),
                                   params.ctypes.data_as(P_dbl), Af.ctypes.data_as(P_dbl), c.real,
                                   c.imag, float(a), float(b), int(m_keep),
                                   av.ctypes.data_as(P_dbl), len(av) // 2,
                                   lam.ctypes.data_as(P_dbl), Y.ctypes.data_as(P_dbl)))
    Yc = (Y[0::2] + 1j * Y[1::2]).reshape(m_keep, m).T
    return lam[0::2] + 1j * lam[1::2], Yc


def nlf_reduced_solve_ex(terms, Ahat, centre, a, b, m_keep, fn=None, method=0, avoid=None):
    """As nlf_reduced_solve with terms ('fn', param) evaluated by fn (a USER_FN object) and the
    reduced-solver choice `method`.  Returns (lam, Y, found)."""
    kinds, params = _kinds(terms)
    m = Ahat[0].shape[0]
    A = np.concatenate([np.asfortranarray(M, dtype=complex).ravel(order="F") for M in Ahat])
    Af = np.empty(2 * len(A))
    Af[0::2], Af[1::2] = A.real, A.imag
    lam = np.zeros(2 * m_keep)
    Y = np.zeros(2 * m * m_keep)
    found = np.zeros(m_keep, dtype=np.int32)
    c = complex(centre)
    av = _cplx_pairs([] if avoid is None else avoid)
    _check(lib().nlf_reduced_solve_ex(m, len(Ahat), kinds.ctypes.data_as(P_i32),
                                      params.ctypes.data_as(P_dbl), fn if fn is not None else USER_FN(),
                                      None, int(method), Af.ctypes.data_as(P_dbl), c.real, c.imag,
                                      float(a), float(b), int(m_keep), av.ctypes.data_as(P_dbl),
                                      len(av) // 2, lam.ctypes.data_as(P_dbl), Y.ctypes.data_as(P_dbl),
                                      found.ctypes.data_as(P_i32)))
    Yc = (Y[0::2] + 1j * Y[1::2]).reshape(m_keep, m).T
    return lam[0::2] + 1j * lam[1::2], Yc, found.astype(bool)


# --------------------------------------------------------------------------- convenience

class NLFEAST:
    """Handle lifecycle around the C ABI: coefficients and contours are set once; the
    workspace (and with it the cached factorisations) persists across solve() calls."""

    def __init__(self, n, device=0, stream=None):
        import torch
        self.n = n
        self.device = torch.device("cuda", device)
        self.h = nlfeast_create(n, device, stream)
        self.ws = None
        self.mats = None
        self.regions = None

    def set_coeffs(self, terms, mats):
        self.mats = list(mats)
        self.terms = list(terms)
        nlfeast_set_coeffs(self.h, terms, self.mats)

    def set_contour(self, regions, quad_rule=NLF_QUAD_GAUSS_LEGENDRE):
        self.regions = list(regions)
        nlfeast_set_contour(self.h, regions, quad_rule)

    def set_user_function(self, py_fn):
        """py_fn(term, param, z, want_deriv) -> (f, df) for the terms of kind 'fn'.  An exception
        raised by py_fn makes solve() raise NLFError(NLF_ERR_ARG) with that exception as its
        cause."""
        self._user_errors = []
        self._user_fn = user_function(py_fn, self._user_errors)
        nlfeast_set_user_function(self.h, self._user_fn)

    def solve(self, opts, X0=None, left=False):
        """Right eigenpairs (nlfeast_solve), or with left=True the left eigenvectors
        (nlfeast_solve_left; X then holds y with y^H T(lambda) = 0)."""
        import torch
        need = nlfeast_workspace_size(self.h, opts)
        if self.ws is None or self.ws.numel() < need:
            self.ws = None
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        m_total = sum(r["m0"] for r in self.regions)
        errors = getattr(self, "_user_errors", None)
        if errors:
            errors.clear()
        try:
            return nlfeast_solve(self.h, opts, self.ws, self.n, m_total, len(self.regions), X0, left=left)
        except NLFError as e:
            if errors:
                raise e from errors[0]
            raise

    def profile(self):
        return nlfeast_get_profile(self.h)

    def close(self):
        if self.h:
            nlfeast_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
