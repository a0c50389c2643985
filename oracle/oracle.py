"""FP64 CPU oracle for the PANDA message-passing iteration (arXiv 1507.07039).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product library never does.

This is a thin ctypes binding over ``panda_oracle.c`` (built with gcc, FP64,
no fast-math, no FMA contraction, OpenMP over output entries).  All arithmetic
of the method lives in the C file; this module only moves numpy arrays in and
out.  Section / equation citations are in the C source next to each function.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "panda_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
# (CPU test of the oracle's memory and arithmetic safety); loaded instead of
# the plain build when ORACLE_SANITIZED=1 (the sanitizer runtime must then be
# preloaded into the process)
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")

OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_DEGENERATE, ERR_NONFINITE, ERR_NOMEM = -1, -2, -3, -5


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (plain IEEE FP64: -O2 -ffp-contract=off);
    sanitize: the AddressSanitizer + UndefinedBehaviorSanitizer build."""
    lib = _LIB_SAN if sanitize else _LIB
    if force or not os.path.exists(lib):
        tmp = lib + ".tmp%d" % os.getpid()
        san = (["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                "-fno-omit-frame-pointer", "-g"] if sanitize else [])
        cmd = (["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                "-fno-fast-math"] + san + ["-o", tmp, _SRC, "-lm"])
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
    return lib


class _Opts(ct.Structure):
    _fields_ = [("alpha", ct.c_double), ("tol", ct.c_double),
                ("max_iter", ct.c_int32), ("diag_alpha", ct.c_int32),
                ("sigma_from_T", ct.c_int32), ("n_own", ct.c_int32),
                ("h_undamped", ct.c_int32), ("update_last", ct.c_int32),
                ("sigma_ddof", ct.c_int32)]


@dataclass
class Options:
    """Run parameters and the readings of the paper (defaults in brackets).

    diag_alpha   [True]  Eq. 6 increment multiplied by alpha (False: literal).
    sigma_from_T [False] sigma from the fresh T row instead of the damped row.
    n_own        [False] Eq. 6 multiplier is the network's own dimension.
    h_undamped   [False] h = mean|(A+R)/2 - W| instead of Eq. 7 literal.
    update_last  [False] update P and C also on the converging iteration.
    sigma_ddof   [0]     Eq. 6 sigma: 0 population std, 1 sample std.
    """
    alpha: float = 0.1
    tol: float = 1e-3
    max_iter: int = 200
    diag_alpha: bool = True
    sigma_from_T: bool = False
    n_own: bool = False
    h_undamped: bool = False
    update_last: bool = False
    sigma_ddof: int = 0

    def _c(self) -> _Opts:
        return _Opts(self.alpha, self.tol, self.max_iter, int(self.diag_alpha),
                     int(self.sigma_from_T), int(self.n_own),
                     int(self.h_undamped), int(self.update_last), int(self.sigma_ddof))


_lib = None


def _load():
    global _lib
    if _lib is None:
        sanitized = os.environ.get("ORACLE_SANITIZED") == "1"
        path = _LIB_SAN if sanitized else _LIB
        if not os.path.exists(path):
            build(force=False, sanitize=sanitized)
        lib = ct.CDLL(path)
        dp = ct.POINTER(ct.c_double)
        lp = ct.POINTER(ct.c_int64)
        i64, i32 = ct.c_int64, ct.c_int32
        lib.oracle_T.restype = ct.c_double
        lib.oracle_T.argtypes = [dp, i64, dp, i64, i64]
        lib.oracle_tanimoto.argtypes = [dp, dp, i64, i64, i64, dp]
        lib.oracle_tanimoto_entries.argtypes = [dp, dp, i64, i64, i64, lp, lp, i64, dp]
        lib.oracle_set_threads.argtypes = [ct.c_int]
        lib.oracle_set_threads.restype = ct.c_int
        lib.oracle_normalize.argtypes = [dp, i64]
        lib.oracle_normalize_ex.argtypes = [dp, i64, i64, i32, i32]
        lib.oracle_step.argtypes = [dp, dp, dp, i64, i64, i32, ct.POINTER(_Opts),
                                    dp, ct.POINTER(i32)]
        lib.oracle_run.argtypes = [dp, dp, dp, i64, i64, i32, ct.POINTER(_Opts),
                                   ct.POINTER(i32), dp, dp]
        lib.oracle_step_w_entries.argtypes = [dp, dp, dp, i64, i64, ct.c_double,
                                              lp, lp, i64, dp]
        lib.oracle_pearson.argtypes = [dp, i64, i64, dp]
        lib.oracle_pearson_entries.argtypes = [dp, i64, i64, lp, lp, i64, dp]
        for f in ("oracle_tanimoto", "oracle_tanimoto_entries", "oracle_normalize",
                  "oracle_normalize_ex",
                  "oracle_step", "oracle_run", "oracle_step_w_entries",
                  "oracle_pearson", "oracle_pearson_entries"):
            getattr(lib, f).restype = ct.c_int
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _lp(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_int64))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def _check(code: int, what: str, allow=(OK,)) -> int:
    if code not in allow:
        raise OracleError(code, what)
    return code


def set_threads(n: int) -> int:
    """OpenMP threads of later oracle calls; returns the previous maximum."""
    return _load().oracle_set_threads(int(n))


def T(x, y) -> float:
    """Eq. 1 for two vectors."""
    x, y = _f64(x).ravel(), _f64(y).ravel()
    if x.size != y.size:
        raise ValueError("length mismatch")
    return _load().oracle_T(_dp(x), 1, _dp(y), 1, x.size)


def tanimoto(X, Y) -> np.ndarray:
    """Out[i, j] = T(X[i, :], Y[:, j]) entry by entry (Sec. II-C Tfunction)."""
    X, Y = _f64(X), _f64(Y)
    M, K = X.shape
    K2, N = Y.shape
    if K != K2:
        raise ValueError("inner dimension mismatch")
    out = np.empty((M, N), np.float64)
    _check(_load().oracle_tanimoto(_dp(X), _dp(Y), M, K, N, _dp(out)), "tanimoto")
    return out


def tanimoto_entries(X, Y, rows, cols) -> np.ndarray:
    X, Y = _f64(X), _f64(Y)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty(rows.size, np.float64)
    M, K = X.shape
    N = Y.shape[1]
    _check(_load().oracle_tanimoto_entries(_dp(X), _dp(Y), M, K, N, _lp(rows), _lp(cols),
                                           rows.size, _dp(out)), "tanimoto_entries")
    return out


def normalize(M) -> np.ndarray:
    """Global z-score (mean and population std over all entries)."""
    out = _f64(M).copy()
    _check(_load().oracle_normalize(_dp(out), out.size), "normalize")
    return out


ZSCORE_GLOBAL, ZSCORE_ROW, ZSCORE_ROWCOL = 0, 1, 2


def normalize_ex(M, mode: int = ZSCORE_GLOBAL, ddof: int = 0) -> np.ndarray:
    """Z-score with a scope (all entries / per row / row and column) and a
    standard-deviation normaliser (ddof 0 population, 1 sample)."""
    out = _f64(M).copy()
    rows, cols = out.shape
    _check(_load().oracle_normalize_ex(_dp(out), rows, cols, mode, ddof), "normalize_ex")
    return out


def step(W, P, C, t: int, opts: Options | None = None):
    """One iteration at step number t; returns (W, P, C, h, converged)."""
    opts = opts or Options()
    W, P, C = _f64(W).copy(), _f64(P).copy(), _f64(C).copy()
    Ne, Na = W.shape
    if P.shape != (Ne, Ne) or C.shape != (Na, Na):
        raise ValueError("shape mismatch")
    h = ct.c_double()
    conv = ct.c_int32()
    o = opts._c()
    _check(_load().oracle_step(_dp(W), _dp(P), _dp(C), Ne, Na, t, ct.byref(o),
                               ct.byref(h), ct.byref(conv)), "step")
    return W, P, C, h.value, bool(conv.value)


@dataclass
class RunResult:
    W: np.ndarray
    P: np.ndarray
    C: np.ndarray
    iters: int
    h: float
    status: int
    h_trace: np.ndarray


def run(W0, P0, C0, opts: Options | None = None, t0: int = 0) -> RunResult:
    """Message passing from already-normalised priors until h < tol."""
    opts = opts or Options()
    W, P, C = _f64(W0).copy(), _f64(P0).copy(), _f64(C0).copy()
    Ne, Na = W.shape
    if P.shape != (Ne, Ne) or C.shape != (Na, Na):
        raise ValueError("shape mismatch")
    trace = np.zeros(max(opts.max_iter, 1), np.float64)
    it = ct.c_int32()
    h = ct.c_double()
    o = opts._c()
    st = _check(_load().oracle_run(_dp(W), _dp(P), _dp(C), Ne, Na, t0, ct.byref(o),
                                   ct.byref(it), ct.byref(h), _dp(trace)),
                "run", allow=(OK, NOT_CONVERGED))
    n = it.value - t0
    return RunResult(W, P, C, it.value, h.value, st, trace[:n].copy())


def step_w_entries(W, P, C, alpha: float, rows, cols) -> np.ndarray:
    """Entries (rows[s], cols[s]) of W after one iteration from (W, P, C)."""
    W, P, C = _f64(W), _f64(P), _f64(C)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    Ne, Na = W.shape
    out = np.empty(rows.size, np.float64)
    _check(_load().oracle_step_w_entries(_dp(W), _dp(P), _dp(C), Ne, Na, alpha,
                                         _lp(rows), _lp(cols), rows.size, _dp(out)),
           "step_w_entries")
    return out


def pearson(E) -> np.ndarray:
    """Co-expression prior (Sec. II-A): Pearson correlation between the rows
    (genes) of E (genes x samples), entry by entry; 0 against a constant row,
    1 on the diagonal."""
    E = _f64(E)
    G, S = E.shape
    out = np.empty((G, G), np.float64)
    _check(_load().oracle_pearson(_dp(E), G, S, _dp(out)), "pearson")
    return out


def pearson_entries(E, rows, cols) -> np.ndarray:
    E = _f64(E)
    G, S = E.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty(rows.size, np.float64)
    _check(_load().oracle_pearson_entries(_dp(E), G, S, _lp(rows), _lp(cols), rows.size,
                                          _dp(out)), "pearson_entries")
    return out


def identity_prior(n: int) -> np.ndarray:
    """Identity network used when no interaction data exist (Sec. II-A)."""
    return np.eye(n, dtype=np.float64)
