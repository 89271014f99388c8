"""FP64 CPU oracle for QAOA on k-NAE-SAT: Python access to ``oracle.c``.

TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU baseline leg
of the benchmark import this package. The GPU library and its binding never
import it, and it imports nothing from them.

``build()`` compiles ``oracle.c`` with gcc and OpenMP into ``liboracle.so``
beside it; the loaders below use what is built and build only when nothing is.
The dense checker in :mod:`oracle.dense` is a second, independent construction
(NumPy only) used to pin this one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_I32P = ctypes.POINTER(ctypes.c_int32)
_F64P = ctypes.POINTER(ctypes.c_double)
_U64P = ctypes.POINTER(ctypes.c_uint64)


def build() -> str:
    """Compile the oracle (gcc, -O2, OpenMP). Returns the library path."""
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_cost.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I32P, _I32P]
    lib.oracle_cost_at.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I32P, _U64P,
                                   ctypes.c_int64, _I32P]
    lib.oracle_count_solutions.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I32P, _U64P]
    lib.oracle_state.argtypes = [ctypes.c_int, _I32P, ctypes.c_int, _F64P, _F64P, _F64P]
    lib.oracle_qaoa.argtypes = [ctypes.c_int, _I32P, ctypes.c_int, _F64P, _F64P, _F64P, _F64P]
    lib.oracle_qaoa_grad.argtypes = [ctypes.c_int, _I32P, ctypes.c_int, _F64P, _F64P,
                                     ctypes.c_double, ctypes.c_double, _F64P, _F64P, _F64P]
    lib.oracle_cost_pred.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I32P, ctypes.c_int, _I32P]
    lib.oracle_cost_at_pred.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I32P, ctypes.c_int, _U64P,
                                        ctypes.c_int64, _I32P]
    lib.oracle_count_solutions_pred.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I32P, ctypes.c_int,
                                                _U64P]
    lib.oracle_sample.argtypes = [ctypes.c_int, _F64P, _F64P, ctypes.c_int64, _U64P]
    lib.oracle_num_threads.argtypes = []
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    for fn in (lib.oracle_cost, lib.oracle_cost_at, lib.oracle_count_solutions, lib.oracle_state,
               lib.oracle_qaoa, lib.oracle_qaoa_grad, lib.oracle_num_threads, lib.oracle_cost_pred,
               lib.oracle_cost_at_pred, lib.oracle_count_solutions_pred, lib.oracle_sample, lib.oracle_set_threads):
        fn.restype = ctypes.c_int
    _lib = lib
    return lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_I32P)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_F64P)


def _instance(clauses, n):
    cl = np.asarray(clauses, dtype=np.int32)
    if cl.ndim != 2:
        raise ValueError("clauses must be an [m, k] array of literals")
    m, k = cl.shape
    return np.ascontiguousarray(cl), m, max(k, 1)


PREDICATES = {"nae": 0, "sat": 1}


def _pred(predicate: str) -> int:
    if predicate not in PREDICATES:
        raise ValueError(f"predicate {predicate!r} is not 'nae' or 'sat'")
    return PREDICATES[predicate]


def cost(clauses, n: int, predicate: str = "nae") -> np.ndarray:
    """C(x) for all x in [0, 2^n) as int32: NAE-violated clauses (Section 3.2,
    eq. knaesatobj) or, with predicate "sat", SAT-violated ones (Section 2.2)."""
    cl, m, k = _instance(clauses, n)
    out = np.empty(1 << n, dtype=np.int32)
    rc = _load().oracle_cost_pred(n, m, k, cl.ctypes.data_as(_I32P), _pred(predicate), out.ctypes.data_as(_I32P))
    if rc:
        raise ValueError("oracle_cost: invalid instance")
    return out


def cost_at(clauses, n: int, xs, predicate: str = "nae") -> np.ndarray:
    """C(x) at the given basis states (int32)."""
    cl, m, k = _instance(clauses, n)
    x = np.ascontiguousarray(np.asarray(xs, dtype=np.uint64))
    out = np.empty(x.shape[0], dtype=np.int32)
    rc = _load().oracle_cost_at_pred(n, m, k, cl.ctypes.data_as(_I32P), _pred(predicate),
                                     x.ctypes.data_as(_U64P), x.shape[0], out.ctypes.data_as(_I32P))
    if rc:
        raise ValueError("oracle_cost_at: invalid arguments")
    return out


def count_solutions(clauses, n: int, predicate: str = "nae") -> int:
    """#{x : C(x) = 0}."""
    cl, m, k = _instance(clauses, n)
    c = ctypes.c_uint64(0)
    rc = _load().oracle_count_solutions_pred(n, m, k, cl.ctypes.data_as(_I32P), _pred(predicate), ctypes.byref(c))
    if rc:
        raise ValueError("oracle_count_solutions: invalid instance")
    return int(c.value)


def _angles(gammas, betas):
    g, gp = _f64(np.atleast_1d(np.asarray(gammas, dtype=np.float64)))
    b, bp = _f64(np.atleast_1d(np.asarray(betas, dtype=np.float64)))
    if g.shape != b.shape:
        raise ValueError("gammas and betas differ in length")
    return g, gp, b, bp


def state(cost_arr, n: int, gammas, betas) -> np.ndarray:
    """Final QAOA state as complex128[2^n]."""
    c, cp = _i32(cost_arr)
    g, gp, b, bp = _angles(gammas, betas)
    psi = np.empty(2 << n, dtype=np.float64)
    rc = _load().oracle_state(n, cp, len(g), gp, bp, psi.ctypes.data_as(_F64P))
    if rc:
        raise ValueError("oracle_state: invalid arguments")
    return psi.view(np.complex128)


def sample(psi, n: int, uniforms) -> np.ndarray:
    """Bitstrings drawn from |psi|^2 / norm by the inverse cumulative
    distribution in index order, one per uniform in [0, 1) (uint64)."""
    st = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
    if st.shape != (1 << n,):
        raise ValueError("psi must have 2^n entries")
    u, up = _f64(np.atleast_1d(np.asarray(uniforms, dtype=np.float64)))
    out = np.empty(u.shape[0], dtype=np.uint64)
    rc = _load().oracle_sample(n, st.view(np.float64).ctypes.data_as(_F64P), up, u.shape[0],
                               out.ctypes.data_as(_U64P))
    if rc:
        raise ValueError("oracle_sample: invalid arguments (uniforms must lie in [0, 1))")
    return out


def running_time(samples, cost_arr) -> int:
    """Instance running time (Section 4.2): the number of bitstrings drawn
    until the first satisfying one (C = 0); 0 if none of them satisfies."""
    c = np.asarray(cost_arr)[np.asarray(samples, dtype=np.int64)]
    hit = np.flatnonzero(c == 0)
    return int(hit[0]) + 1 if hit.size else 0


def qaoa(cost_arr, n: int, gammas, betas):
    """(p_succ, E[C], norm) of the depth-p QAOA state."""
    c, cp = _i32(cost_arr)
    g, gp, b, bp = _angles(gammas, betas)
    out = np.zeros(3, dtype=np.float64)
    rc = _load().oracle_qaoa(n, cp, len(g), gp, bp, None, out.ctypes.data_as(_F64P))
    if rc:
        raise ValueError("oracle_qaoa: invalid arguments")
    return float(out[0]), float(out[1]), float(out[2])


def qaoa_grad(cost_arr, n: int, gammas, betas, w_psucc: float = 1.0, w_energy: float = 0.0):
    """Adjoint gradient of w_psucc*p_succ + w_energy*E[C].

    Returns (dgammas, dbetas, (p_succ, E[C], norm))."""
    c, cp = _i32(cost_arr)
    g, gp, b, bp = _angles(gammas, betas)
    p = len(g)
    dg = np.zeros(p, dtype=np.float64)
    db = np.zeros(p, dtype=np.float64)
    out = np.zeros(3, dtype=np.float64)
    rc = _load().oracle_qaoa_grad(n, cp, p, gp, bp, float(w_psucc), float(w_energy),
                                  dg.ctypes.data_as(_F64P), db.ctypes.data_as(_F64P),
                                  out.ctypes.data_as(_F64P))
    if rc:
        raise ValueError("oracle_qaoa_grad: invalid arguments")
    return dg, db, (float(out[0]), float(out[1]), float(out[2]))


def finite_difference_grad(cost_arr, n: int, gammas, betas, w_psucc=1.0, w_energy=0.0, h=1e-4):
    """Central differences (F(theta + h e_i) - F(theta - h e_i)) / 2h on the
    oracle forward, for every gamma_i and beta_i."""
    g = np.asarray(gammas, dtype=np.float64)
    b = np.asarray(betas, dtype=np.float64)

    def F(gg, bb):
        ps, e, _ = qaoa(cost_arr, n, gg, bb)
        return w_psucc * ps + w_energy * e

    dg = np.zeros_like(g)
    db = np.zeros_like(b)
    for i in range(len(g)):
        e = np.zeros_like(g)
        e[i] = h
        dg[i] = (F(g + e, b) - F(g - e, b)) / (2 * h)
        db[i] = (F(g, b + e) - F(g, b - e)) / (2 * h)
    return dg, db


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_threads(threads: int) -> int:
    """OpenMP threads for the following oracle calls; returns the count in effect."""
    return int(_load().oracle_set_threads(int(threads)))
