"""FP64 CPU oracle for SBQA (arXiv 2604.01050, Sec. II.A-B, Supplement S1).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check
and by the benchmark's CPU-baseline leg, never by the library's product path.
The arithmetic lives in ``sbqa_oracle.c`` (plain C, float64, no fused
multiply-add contraction); this module only builds it with gcc and marshals
numpy arrays through ctypes.

Layouts: state X, Y and fields are (N, C) float64 row-major with C = runs*R
and column c = r*R + k; spins are (count, N) int8 in {-1, +1}.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sbqa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

F_TERNARY, F_SIGN, F_BALLISTIC = 0, 1, 2

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared", "-march=x86-64-v2", "-Wall"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (seconds). Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ct.CDLL:
    global _lib
    if _lib is None:
        _lib = ct.CDLL(build())
        _declare(_lib)
    return _lib


class _Problem(ct.Structure):
    _fields_ = [("N", ct.c_int32), ("R", ct.c_int32), ("runs", ct.c_int32),
                ("dense", ct.c_void_p), ("row_ptr", ct.c_void_p), ("col", ct.c_void_p),
                ("val", ct.c_void_p), ("h", ct.c_void_p),
                ("dt", ct.c_double), ("a0", ct.c_double), ("c0", ct.c_double),
                ("fmode", ct.c_int32), ("n3", ct.c_int64), ("tri", ct.c_void_p), ("K", ct.c_void_p)]


def _declare(L):
    d, i32, i64, vp, f32 = ct.c_double, ct.c_int32, ct.c_int64, ct.c_void_p, ct.c_float
    L.orc_num_threads.restype = ct.c_int
    L.orc_set_threads.argtypes = [ct.c_int]
    L.orc_pump.argtypes, L.orc_pump.restype = [i64, i64], d
    L.orc_delta32.argtypes, L.orc_delta32.restype = [d, i64, i64], f32
    L.orc_gamma_x.argtypes, L.orc_gamma_x.restype = [d, d, d], d
    L.orc_jperp.argtypes, L.orc_jperp.restype = [d, d], d
    L.orc_jperp_paper_table.argtypes = [d, d, d, i64, vp]
    L.orc_jperp_linear_table.argtypes = [d, d, i64, vp]
    L.orc_energy_dense.argtypes = [i32, vp, vp, vp, i32, vp]
    L.orc_energy_csr.argtypes = [i32, vp, vp, vp, vp, vp, i32, vp]
    L.orc_bruteforce_dense.argtypes, L.orc_bruteforce_dense.restype = [i32, vp, vp, vp], d
    L.orc_apply_f.argtypes = [i32, f32, i64, vp, vp]
    L.orc_fields_dense.argtypes = [i32, i32, vp, vp, vp]
    L.orc_fields_csr.argtypes = [i32, i32, vp, vp, vp, vp, vp]
    L.orc_step.argtypes = [ct.POINTER(_Problem), vp, vp, d, f32, vp, vp, vp]
    L.orc_step_rows.argtypes = [ct.POINTER(_Problem), vp, vp, d, f32, vp, i32, vp, vp, vp, vp, vp]
    L.orc_run.argtypes = [ct.POINTER(_Problem), vp, vp, i64, vp, d, i64, vp, vp, vp]
    L.orc_run.restype = i32
    L.orc_auto_c0_dense.argtypes, L.orc_auto_c0_dense.restype = [i32, vp], d
    L.orc_auto_c0_csr.argtypes, L.orc_auto_c0_csr.restype = [i32, vp, vp, vp], d
    L.orc_energy3.argtypes = [i32, i64, vp, vp, vp, i32, vp]
    L.orc_bruteforce_hubo.argtypes, L.orc_bruteforce_hubo.restype = [i32, vp, vp, i64, vp, vp, vp], d
    L.orc_fields3.argtypes = [i32, i32, i64, vp, vp, vp, vp]
    L.orc_auto_c0_hubo.argtypes, L.orc_auto_c0_hubo.restype = [i32, vp, vp, vp, i64, vp], d


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ---------------------------------------------------------------- schedules
def pump(n: int, S: int) -> float:
    """a_n = n/S (Sec. II.A, a(t) = t/T)."""
    return lib().orc_pump(n, S)


def delta32(delta_max: float, n: int, S: int) -> np.float32:
    """Threshold of Eq. 8, rounded to binary32."""
    return np.float32(lib().orc_delta32(delta_max, n, S))


def gamma_x(gamma0: float, alpha: float, s: float) -> float:
    """Gamma_x(t) of Eq. 5 at s = t/T."""
    return lib().orc_gamma_x(gamma0, alpha, s)


def jperp(beta: float, gamma_x_over_R: float) -> float:
    """J_perp of Eq. 5 / Eq. S12 for a given Gamma_x/R."""
    return lib().orc_jperp(beta, gamma_x_over_R)


def jperp_paper_table(beta: float, alpha: float, gamma0_over_R: float, S: int) -> np.ndarray:
    out = np.empty(S)
    lib().orc_jperp_paper_table(beta, alpha, gamma0_over_R, S, _p(out))
    return out


def jperp_linear_table(start: float, end: float, S: int) -> np.ndarray:
    out = np.empty(S)
    lib().orc_jperp_linear_table(start, end, S, _p(out))
    return out


# ------------------------------------------------------------------ energies
def energy(spins, J=None, h=None, csr=None, tri=None, K=None) -> np.ndarray:
    """E(s) = -1/2 s^T J s - h^T s - sum_t K_t s_l s_m s_n for each row of
    spins (count, N); tri (n3, 3) lists each triple once."""
    s = np.ascontiguousarray(np.atleast_2d(spins), dtype=np.int8)
    count, N = s.shape
    E = np.empty(count)
    h = _f64(h)
    if csr is not None:
        rp, col, val = _i32(csr[0]), _i32(csr[1]), _f64(csr[2])
        lib().orc_energy_csr(N, _p(rp), _p(col), _p(val), _p(h), _p(s), count, _p(E))
    else:
        J = _f64(J)
        lib().orc_energy_dense(N, _p(J), _p(h), _p(s), count, _p(E))
    if tri is not None and len(tri):
        tri, K = _i32(tri), _f64(K)
        E3 = np.empty(count)
        lib().orc_energy3(N, len(K), _p(tri), _p(K), _p(s), count, _p(E3))
        E = E + E3
    return E


def bruteforce_hubo(J, h=None, tri=None, K=None):
    """Exhaustive minimum with three-body terms (N <= 24). Returns (E_min, spins)."""
    J = _f64(J)
    N = J.shape[0]
    tri = _i32(np.zeros((0, 3)) if tri is None else tri)
    K = _f64(np.zeros(0) if K is None else K)
    best = np.empty(N, dtype=np.int8)
    E = lib().orc_bruteforce_hubo(N, _p(J), _p(_f64(h)), len(K), _p(tri), _p(K), _p(best))
    return E, best


def bruteforce(J, h=None):
    """Exhaustive ground state (N <= 30). Returns (E_min, spins)."""
    J = _f64(J)
    N = J.shape[0]
    best = np.empty(N, dtype=np.int8)
    E = lib().orc_bruteforce_dense(N, _p(J), _p(_f64(h)), _p(best))
    return E, best


def auto_c0(J=None, csr=None, K=None) -> float:
    """c0 = 0.5 / (sqrt(N) * rms of off-diagonal J); with three-body weights K
    (CSR two-body part) the field-variance rule of orc_auto_c0_hubo."""
    if K is not None and len(K):
        rp, col, val = _i32(csr[0]), _i32(csr[1]), _f64(csr[2])
        K = _f64(K)
        return lib().orc_auto_c0_hubo(rp.size - 1, _p(rp), _p(col), _p(val), len(K), _p(K))
    if csr is not None:
        rp, col, val = _i32(csr[0]), _i32(csr[1]), _f64(csr[2])
        return lib().orc_auto_c0_csr(rp.size - 1, _p(rp), _p(col), _p(val))
    J = _f64(J)
    return lib().orc_auto_c0_dense(J.shape[0], _p(J))


# --------------------------------------------------------------- nonlinear f
def apply_f(fmode: int, delta, x) -> np.ndarray:
    x = _f64(x)
    g = np.empty_like(x)
    lib().orc_apply_f(fmode, float(np.float32(delta)), x.size, _p(x), _p(g))
    return g


def fields(G, J=None, csr=None, tri=None, K=None) -> np.ndarray:
    """Phi = J G (+ the three-body sums) for G of shape (N, C)."""
    G = _f64(G)
    N, C = G.shape
    Phi = np.empty_like(G)
    if csr is not None:
        rp, col, val = _i32(csr[0]), _i32(csr[1]), _f64(csr[2])
        lib().orc_fields_csr(N, C, _p(rp), _p(col), _p(val), _p(G), _p(Phi))
    else:
        J = _f64(J)
        lib().orc_fields_dense(N, C, _p(J), _p(G), _p(Phi))
    if tri is not None and len(tri):
        tri, K = _i32(tri), _f64(K)
        lib().orc_fields3(N, C, len(K), _p(tri), _p(K), _p(G), _p(Phi))
    return Phi


# ------------------------------------------------------------------ dynamics
class Problem:
    """An SBQA problem for the oracle: couplings, fields and constants."""

    def __init__(self, N, R, runs, J=None, csr=None, h=None, dt=0.5, a0=1.0, c0=None,
                 fmode=F_TERNARY, tri=None, K=None):
        self.N, self.R, self.runs = int(N), int(R), int(runs)
        self.C = self.R * self.runs
        self.J = _f64(J)
        self.csr = None if csr is None else (_i32(csr[0]), _i32(csr[1]), _f64(csr[2]))
        self.h = _f64(h)
        self.tri = _i32(np.zeros((0, 3)) if tri is None else tri)
        self.K = _f64(np.zeros(0) if K is None else K)
        self.dt, self.a0 = float(dt), float(a0)
        self.c0 = float(auto_c0(J=self.J, csr=self.csr, K=self.K) if c0 is None else c0)
        self.fmode = int(fmode)
        self._s = _Problem(self.N, self.R, self.runs, _p(self.J),
                           _p(self.csr[0]) if self.csr else None,
                           _p(self.csr[1]) if self.csr else None,
                           _p(self.csr[2]) if self.csr else None,
                           _p(self.h), self.dt, self.a0, self.c0, self.fmode,
                           len(self.K), _p(self.tri) if len(self.K) else None, _p(self.K) if len(self.K) else None)

    def step(self, X, Y, a_n, delta_n, jperp_r, want_phi=False):
        """One step (Eqs. 6-7 + wall) from (X, Y); returns new (X, Y[, Phi])."""
        X = np.array(X, dtype=np.float64, order="C", copy=True)
        Y = np.array(Y, dtype=np.float64, order="C", copy=True)
        jr = _f64(np.broadcast_to(np.asarray(jperp_r, dtype=np.float64), (self.runs,)))
        scratch = np.empty(3 * X.size)
        Phi = np.empty_like(X) if want_phi else None
        lib().orc_step(ct.byref(self._s), _p(X), _p(Y), float(a_n),
                       float(np.float32(delta_n)), _p(jr), _p(scratch), _p(Phi))
        return (X, Y, Phi) if want_phi else (X, Y)

    def step_rows(self, X, Y, a_n, delta_n, jperp_r, rows):
        """The step restricted to the given rows: returns (X', Y', Phi) of shape (len(rows), C)."""
        X = _f64(X)
        Y = _f64(Y)
        rows = _i32(rows)
        jr = _f64(np.broadcast_to(np.asarray(jperp_r, dtype=np.float64), (self.runs,)))
        n = rows.size
        Xo, Yo, Po = (np.empty((n, self.C)) for _ in range(3))
        scratch = np.empty(X.size)
        lib().orc_step_rows(ct.byref(self._s), _p(X), _p(Y), float(a_n), float(np.float32(delta_n)),
                            _p(jr), n, _p(rows), _p(scratch), _p(Xo), _p(Yo), _p(Po))
        return Xo, Yo, Po

    def run(self, X, Y, S, jperp_table, delta_max=0.7, energy_every=0):
        """S steps from (X, Y); jperp_table (runs, S). Returns dict of results."""
        X = np.array(X, dtype=np.float64, order="C", copy=True)
        Y = np.array(Y, dtype=np.float64, order="C", copy=True)
        jt = _f64(np.broadcast_to(np.asarray(jperp_table, dtype=np.float64), (self.runs, S)))
        bE = np.empty(self.runs)
        bs = np.empty((self.runs, self.N), dtype=np.int8)
        bstep = np.empty(self.runs, dtype=np.int64)
        rc = lib().orc_run(ct.byref(self._s), _p(X), _p(Y), int(S), _p(jt), float(delta_max),
                           int(energy_every), _p(bE), _p(bs), _p(bstep))
        if rc != 0:
            raise MemoryError("oracle run failed")
        return {"X": X, "Y": Y, "best_E": bE, "best_s": bs, "best_step": bstep}
