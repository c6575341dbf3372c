"""Serial CPU reference ("oracle") for Chebyshev time propagation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  The product library
never calls it, and the two share no code: the oracle has its own Hamiltonian
builders, Bessel routine, spectral bounds and loops (``chebtd_oracle.c``),
compiled with gcc into ``liboracle.so`` next to this file.

Every function follows Fehske et al., arXiv:0907.3022, Sect. 2.2 (Chebyshev
scheme, eq. (U_1), the Bessel coefficients, the recursion and the truncation
rule eq. (dec_Bessel)), eq. (CN) for Crank-Nicolson, and the models of
Sect. 3 (double well, eq. (model) honeycomb ribbon, eq. (ghm) Holstein
polaron).  hbar = 1.  The wrappers below only marshal numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chebtd_oracle.c")
# ORACLE_LIB names another build of the same source (the sanitizer build of
# the tests); by default the one next to this file
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, one thread, plain C11)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = C.CDLL(_LIB_PATH)
    d, i64, i32 = C.c_double, C.c_int64, C.c_int
    P = C.c_void_p
    sig = {
        "orc_bessel_j": (i32, [d, i32, P]),
        "orc_trunc_order": (i32, [d, d]),
        "orc_scale": (i32, [d, d, d, P, P]),
        "orc_coeffs": (i32, [d, d, d, i32, P]),
        "orc_free_matrix": (None, [i32]),
        "orc_matrix_nnz": (i64, [i32]),
        "orc_matrix_n": (i64, [i32]),
        "orc_matrix_export": (i32, [i32, P, P, P]),
        "orc_matrix_import": (i32, [i64, i64, P, P, P]),
        "orc_build_chain1d": (i32, [i64, d, P]),
        "orc_build_honeycomb": (i32, [i64, i64, i32, d, P]),
        "orc_holstein_nconf": (i64, [i32, i32]),
        "orc_holstein_occupations": (i32, [i32, i32, P]),
        "orc_build_holstein": (i32, [i32, i32, d, d, P, P, i32]),
        "orc_gershgorin": (i32, [i32, P, P]),
        "orc_apply": (i32, [i32, P, P]),
        "orc_propagate": (i32, [i32, d, d, i32, P, P, i64, P, P]),
        "orc_adjoint": (i32, [i32, d, d, i32, P, P, i64, P, P, P, P]),
        "orc_crank_nicolson_1d": (i32, [i64, d, P, d, i64, P]),
        "orc_density": (None, [i64, P, P]),
        "orc_region_sum": (d, [i64, P, P]),
        "orc_holstein_obs": (i32, [i32, i32, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c128(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.complex128)


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float64)


# --------------------------------------------------------------------------
# coefficients (Sect. 2.2)
# --------------------------------------------------------------------------
def bessel_j(z: float, kmax: int) -> np.ndarray:
    """J_0(z) .. J_kmax(z) by Miller's backward recurrence."""
    out = np.zeros(kmax + 1)
    if _load().orc_bessel_j(float(z), int(kmax), _ptr(out)) != 0:
        raise ValueError("bad Bessel arguments")
    return out


def trunc_order(z: float, tol: float = 1e-15) -> int:
    """M: last kept order; |J_k(z)| < tol for every k > M (eq. (dec_Bessel))."""
    M = _load().orc_trunc_order(float(z), float(tol))
    if M < 0:
        raise ValueError("bad truncation arguments")
    return M


def scale(emin: float, emax: float, alpha: float = 0.01):
    """(a, b) of H~ = (H - b)/a from the extreme eigenvalues (Sect. 2.2)."""
    a, b = C.c_double(), C.c_double()
    if _load().orc_scale(emin, emax, alpha, C.byref(a), C.byref(b)) != 0:
        raise ValueError("need emax > emin and alpha >= 0")
    return a.value, b.value


def coeffs(a: float, b: float, dt: float, M: int) -> np.ndarray:
    """gamma_k, k = 0..M: eq. (U_1) weights with e^{-i b dt} and the 2 folded in."""
    g = np.zeros(M + 1, dtype=np.complex128)
    if _load().orc_coeffs(a, b, dt, int(M), _ptr(g)) != 0:
        raise ValueError("bad coefficient arguments")
    return g


# --------------------------------------------------------------------------
# Hamiltonians (explicit CSR inside the oracle)
# --------------------------------------------------------------------------
class Matrix:
    """Handle of a CSR Hamiltonian held by the oracle library."""

    def __init__(self, handle: int):
        if handle < 0:
            raise ValueError("oracle could not build the matrix")
        self.h = handle
        self.n = int(_load().orc_matrix_n(handle))
        self.nnz = int(_load().orc_matrix_nnz(handle))

    def __del__(self):
        try:
            if self.h >= 0 and _lib is not None:
                _lib.orc_free_matrix(self.h)
                self.h = -1
        except Exception:
            pass

    def csr(self):
        rowptr = np.zeros(self.n + 1, dtype=np.int64)
        col = np.zeros(max(self.nnz, 1), dtype=np.int64)
        val = np.zeros(max(self.nnz, 1), dtype=np.complex128)
        _load().orc_matrix_export(self.h, _ptr(rowptr), _ptr(col), _ptr(val))
        return rowptr, col[: self.nnz], val[: self.nnz]

    def dense(self) -> np.ndarray:
        rowptr, col, val = self.csr()
        H = np.zeros((self.n, self.n), dtype=np.complex128)
        for i in range(self.n):
            for p in range(rowptr[i], rowptr[i + 1]):
                H[i, col[p]] += val[p]
        return H

    def apply(self, x) -> np.ndarray:
        x = _c128(x)
        y = np.zeros_like(x)
        _load().orc_apply(self.h, _ptr(x), _ptr(y))
        return y

    def gershgorin(self):
        lo, hi = C.c_double(), C.c_double()
        if _load().orc_gershgorin(self.h, C.byref(lo), C.byref(hi)) != 0:
            raise ValueError("empty matrix")
        return lo.value, hi.value


def chain1d(V, dx: float) -> Matrix:
    V = _f64(V)
    return Matrix(_load().orc_build_chain1d(V.size, float(dx), _ptr(V)))


def honeycomb(width: int, length: int, eps, edge: str = "zigzag", t: float = 1.0) -> Matrix:
    eps = _f64(eps)
    assert eps.size == width * length
    e = {"zigzag": 0, "armchair": 1}[edge]
    return Matrix(_load().orc_build_honeycomb(width, length, e, float(t), _ptr(eps)))


def holstein_nconf(L: int, nph: int) -> int:
    return int(_load().orc_holstein_nconf(L, nph))


def holstein_occupations(L: int, nph: int) -> np.ndarray:
    cnt = holstein_nconf(L, nph)
    occ = np.zeros(cnt * L, dtype=np.uint8)
    if _load().orc_holstein_occupations(L, nph, _ptr(occ)) != 0:
        raise ValueError("basis too large for the oracle")
    return occ.reshape(cnt, L)


def holstein(L: int, nph: int, t: float, w0: float, g, Delta, periodic: bool) -> Matrix:
    g = _f64(np.broadcast_to(np.asarray(g, dtype=np.float64), (L,)))
    Delta = _f64(np.broadcast_to(np.asarray(Delta, dtype=np.float64), (L,)))
    return Matrix(_load().orc_build_holstein(L, nph, float(t), float(w0), _ptr(g),
                                             _ptr(Delta), int(bool(periodic))))


def import_csr(rowptr, col, val) -> Matrix:
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int64)
    val = _c128(val)
    return Matrix(_load().orc_matrix_import(rowptr.size - 1, col.size, _ptr(rowptr),
                                            _ptr(col), _ptr(val)))


# --------------------------------------------------------------------------
# propagation, adjoint, Crank-Nicolson, observables
# --------------------------------------------------------------------------
class Plan:
    """Spectral scale (a, b), order M and weights gamma for one time step."""

    def __init__(self, emin, emax, dt, alpha=0.01, tol=1e-15, M=None):
        self.emin, self.emax, self.dt, self.alpha, self.tol = emin, emax, dt, alpha, tol
        self.a, self.b = scale(emin, emax, alpha)
        self.M = trunc_order(self.a * dt, tol) if M is None else int(M)
        self.gamma = coeffs(self.a, self.b, dt, self.M)


def propagate(H: Matrix, plan: Plan, psi, K: int, want_obs: bool = False):
    psi = _c128(psi).copy()
    nrm = np.zeros(max(K, 1))
    en = np.zeros(max(K, 1))
    rc = _load().orc_propagate(H.h, plan.a, plan.b, plan.M, _ptr(plan.gamma), _ptr(psi),
                               int(K), _ptr(nrm), _ptr(en))
    if rc != 0:
        raise ValueError("oracle propagate failed")
    if want_obs:
        return psi, nrm[:K], en[:K]
    return psi


def adjoint(H: Matrix, plan: Plan, psi0, K: int, mask):
    """Returns (L, dL/dV, adjoint of psi_0) for L = sum mask |psi_K|^2."""
    psi0 = _c128(psi0)
    mask = _f64(mask)
    g = np.zeros(H.n)
    gb = np.zeros(H.n, dtype=np.complex128)
    Lv = C.c_double()
    rc = _load().orc_adjoint(H.h, plan.a, plan.b, plan.M, _ptr(plan.gamma), _ptr(psi0), int(K),
                             _ptr(mask), _ptr(g), _ptr(gb), C.byref(Lv))
    if rc != 0:
        raise ValueError("oracle adjoint failed")
    return Lv.value, g, gb


def crank_nicolson_1d(V, dx: float, psi, dt: float, S: int) -> np.ndarray:
    V = _f64(V)
    psi = _c128(psi).copy()
    if _load().orc_crank_nicolson_1d(V.size, float(dx), _ptr(V), float(dt), int(S), _ptr(psi)) != 0:
        raise ValueError("oracle CN failed")
    return psi


def density(psi) -> np.ndarray:
    psi = _c128(psi)
    rho = np.zeros(psi.size)
    _load().orc_density(psi.size, _ptr(psi), _ptr(rho))
    return rho


def region_sum(psi, mask) -> float:
    psi = _c128(psi)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    return float(_load().orc_region_sum(psi.size, _ptr(psi), _ptr(mask)))


def holstein_obs(L: int, nph: int, psi):
    psi = _c128(psi)
    n_i, nph_i, chi = np.zeros(L), np.zeros(L), np.zeros(L)
    if _load().orc_holstein_obs(L, nph, _ptr(psi), _ptr(n_i), _ptr(nph_i), _ptr(chi)) != 0:
        raise ValueError("oracle Holstein observables failed")
    return n_i, nph_i, chi
