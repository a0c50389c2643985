"""Thin Python binding of libpanda.so (argument marshalling only).

Every step of the message-passing path runs in the HIP kernels of the
library; this module checks tensor placement, passes device pointers and the
current HIP stream, and turns status codes into exceptions.  PyTorch is used
only to own device memory and streams.  There is no CPU fallback: if the
library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpanda.so")
# the host-sanitized build, for the sanitizer test (PANDA_LIB_SANITIZED=1)
if os.environ.get("PANDA_LIB_SANITIZED") == "1":
    LIB_PATH = os.path.join(HERE, "libpanda_san.so")

OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_DEGENERATE, ERR_NONFINITE, ERR_HIP, ERR_WORKSPACE = -1, -2, -3, -4, -5

# Every extern "C" entry point declared in include/panda.h.
EXPORTS = (
    "panda_default_options", "panda_normalize_workspace_bytes", "panda_normalize",
    "panda_normalize_ex_workspace_bytes", "panda_normalize_ex",
    "panda_tanimoto_workspace_bytes", "panda_tanimoto",
    "panda_pearson_workspace_bytes", "panda_pearson", "panda_pearson_noalloc",
    "panda_workspace_bytes",
    "panda_ctx_create", "panda_ctx_load", "panda_iterate", "panda_ctx_store",
    "panda_ctx_destroy", "panda_run", "panda_ctx_set_timing", "panda_ctx_phase_times",
    "panda_batch_workspace_bytes", "panda_batch_create", "panda_batch_destroy",
    "panda_batch_tile_candidates", "panda_batch_get_tiles", "panda_batch_set_tiles",
    "panda_batch_autotune", "panda_batch_load", "panda_batch_iterate", "panda_batch_run",
    "panda_batch_state", "panda_batch_store",
    "panda_ws_features_workspace_bytes", "panda_ws_features", "panda_mlp_forward",
    "panda_mlp_grad_workspace_bytes", "panda_mlp_grad", "panda_mlp_adam", "panda_mlp_train_step",
    "panda_ws_target", "panda_ws_predict", "panda_ws_init",
    "panda_permute_sym", "panda_null_workspace_bytes", "panda_null", "panda_null_zscore",
    "panda_status_string", "panda_last_error",
)

WS_FEATURES, WS_SKETCH, MLP_PARAMS = 16, 6, 5313

BATCH_TILES = ("R", "A+W", "P-partial", "C")

PHASES = ("R", "A+W", "h", "P-partial", "P-final", "C", "diag")


ZSCORE_GLOBAL, ZSCORE_ROW, ZSCORE_ROWCOL = 0, 1, 2


class PandaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"panda status {code}: {msg}")
        self.code = code


class Options(ct.Structure):
    """Mirror of panda_options (include/panda.h)."""
    _fields_ = [("alpha", ct.c_double), ("tol", ct.c_double), ("max_iter", ct.c_int32),
                ("diag_alpha", ct.c_int32), ("sigma_from_T", ct.c_int32),
                ("n_own", ct.c_int32), ("h_undamped", ct.c_int32),
                ("update_last", ct.c_int32), ("poll_every", ct.c_int32),
                ("precision", ct.c_int32), ("sigma_ddof", ct.c_int32),
                ("zscore_mode", ct.c_int32), ("packed_c", ct.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpanda.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1507_07039_amd/build.py")
    lib = ct.CDLL(path)
    vp, sz, i64, i32, dbl = ct.c_void_p, ct.c_size_t, ct.c_int64, ct.c_int32, ct.c_double
    op = ct.POINTER(Options)
    sig = {
        "panda_default_options": (None, [op]),
        "panda_normalize_workspace_bytes": (sz, []),
        "panda_normalize": (ct.c_int, [vp, i64, i64, vp, sz, vp]),
        "panda_normalize_ex_workspace_bytes": (sz, [i64, i64, i32]),
        "panda_normalize_ex": (ct.c_int, [vp, i64, i64, i32, i32, vp, sz, vp]),
        "panda_tanimoto_workspace_bytes": (sz, [i64, i64, i64]),
        "panda_tanimoto": (ct.c_int, [vp, vp, i64, i64, i64, vp, vp, sz, vp]),
        "panda_pearson_workspace_bytes": (sz, [i64, i64]),
        "panda_pearson": (ct.c_int, [vp, i64, i64, i64, vp, i64, vp, sz, vp]),
        "panda_pearson_noalloc": (ct.c_int, [vp, i64, i64, i64, vp, i64, vp]),
        "panda_workspace_bytes": (sz, [i64, i64, op]),
        "panda_ctx_create": (ct.c_int, [i64, i64, op, vp, sz, vp, ct.POINTER(vp)]),
        "panda_ctx_load": (ct.c_int, [vp, vp, vp, vp, i32]),
        "panda_iterate": (ct.c_int, [vp, ct.POINTER(dbl), ct.POINTER(i32)]),
        "panda_ctx_store": (ct.c_int, [vp, vp, vp, vp, ct.POINTER(dbl), ct.POINTER(i32)]),
        "panda_ctx_destroy": (None, [vp]),
        "panda_run": (ct.c_int, [vp, vp, vp, i64, i64, dbl, dbl, i32, vp, vp, vp, vp, sz, op,
                                 ct.POINTER(i32), ct.POINTER(dbl), vp]),
        "panda_ctx_set_timing": (ct.c_int, [vp, i32]),
        "panda_ctx_phase_times": (ct.c_int, [vp, ct.POINTER(dbl), ct.POINTER(i64)]),
        "panda_batch_workspace_bytes": (sz, [i32, ct.POINTER(i64), ct.POINTER(i64), op]),
        "panda_batch_create": (ct.c_int, [i32, ct.POINTER(i64), ct.POINTER(i64), op, vp, sz, vp,
                                          ct.POINTER(vp)]),
        "panda_batch_destroy": (None, [vp]),
        "panda_batch_tile_candidates": (i32, [i32]),
        "panda_batch_get_tiles": (ct.c_int, [vp, ct.POINTER(i32)]),
        "panda_batch_set_tiles": (ct.c_int, [vp, ct.POINTER(i32)]),
        "panda_batch_autotune": (ct.c_int, [vp, i32, ct.POINTER(ct.c_float)]),
        "panda_batch_load": (ct.c_int, [vp, i32, vp, vp, vp, i32]),
        "panda_batch_iterate": (ct.c_int, [vp, i32, i32, ct.POINTER(i32)]),
        "panda_batch_run": (ct.c_int, [vp, i32, ct.POINTER(i32)]),
        "panda_batch_state": (ct.c_int, [vp, i32, ct.POINTER(dbl), ct.POINTER(i32),
                                         ct.POINTER(i32)]),
        "panda_batch_store": (ct.c_int, [vp, i32, vp, vp, vp, ct.POINTER(dbl), ct.POINTER(i32)]),
        "panda_ws_features_workspace_bytes": (sz, [i64, i64]),
        "panda_ws_features": (ct.c_int, [vp, vp, vp, vp, ct.POINTER(dbl), vp, sz]),
        "panda_mlp_forward": (ct.c_int, [vp, vp, i64, vp, vp]),
        "panda_mlp_grad_workspace_bytes": (sz, [i64]),
        "panda_mlp_grad": (ct.c_int, [vp, vp, i64, vp, vp, i64, vp, vp, vp, sz, vp]),
        "panda_mlp_adam": (ct.c_int, [vp, vp, vp, vp, i32, ct.c_float, ct.c_float, ct.c_float,
                                      ct.c_float, vp]),
        "panda_mlp_train_step": (ct.c_int, [vp, vp, vp, i32, ct.c_float, vp, i64, vp, vp, i64, vp,
                                            vp, vp, sz, vp]),
        "panda_ws_target": (ct.c_int, [vp, vp, i64, i64, dbl, vp, vp]),
        "panda_ws_predict": (ct.c_int, [vp, vp, i64, i64, dbl, vp, vp]),
        "panda_ws_init": (ct.c_int, [vp, vp, i32]),
        "panda_permute_sym": (ct.c_int, [vp, i64, i64, vp, vp, i64, vp]),
        "panda_null_workspace_bytes": (sz, [i64, i64, op]),
        "panda_null": (ct.c_int, [vp, vp, vp, i64, i64, i32, vp, vp, op, vp, sz, vp, vp,
                                  ct.POINTER(i32), vp]),
        "panda_null_zscore": (ct.c_int, [vp, vp, vp, i64, i64, vp, vp]),
        "panda_status_string": (ct.c_char_p, [ct.c_int]),
        "panda_last_error": (ct.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def default_options(**kw) -> Options:
    o = Options()
    load_library().panda_default_options(ct.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _check(code: int, allow=(OK,)) -> int:
    if code not in allow:
        lib = load_library()
        raise PandaError(code, lib.panda_last_error().decode())
    return code


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libpanda needs a ROCm GPU; torch.cuda.is_available() is False")
    return torch


def _dev(t, name, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
        raise TypeError(f"{name} must be a float32 tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


def _stream():
    return ct.c_void_p(_torch().cuda.current_stream().cuda_stream)


def workspace(nbytes: int):
    """Caller-owned device workspace (256-byte aligned by the caching allocator)."""
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


def normalize(M, mode: int = 0, ddof: int = 0) -> None:
    """Z-score the network M in place: panda_normalize (all entries,
    population std) by default, else panda_normalize_ex with the scope
    mode (ZSCORE_GLOBAL / ZSCORE_ROW / ZSCORE_ROWCOL) and normaliser ddof."""
    lib = load_library()
    rows, cols = M.shape
    if mode == ZSCORE_GLOBAL and ddof == 0:
        ws = workspace(lib.panda_normalize_workspace_bytes())
        _check(lib.panda_normalize(_dev(M, "M"), rows, cols, ws.data_ptr(), ws.numel(),
                                   _stream()))
        return
    ws = workspace(lib.panda_normalize_ex_workspace_bytes(rows, cols, mode))
    _check(lib.panda_normalize_ex(_dev(M, "M"), rows, cols, mode, ddof, ws.data_ptr(),
                                  ws.numel(), _stream()))


def tanimoto(X, Y):
    """Out = T(X, Y) (panda_tanimoto, the paper's Tfunction)."""
    torch = _torch()
    lib = load_library()
    M, K = X.shape
    K2, N = Y.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    out = torch.empty((M, N), dtype=torch.float32, device="cuda")
    ws = workspace(lib.panda_tanimoto_workspace_bytes(M, K, N))
    _check(lib.panda_tanimoto(_dev(X, "X"), _dev(Y, "Y"), M, K, N, out.data_ptr(),
                              ws.data_ptr(), ws.numel(), _stream()))
    return out


def pearson(E):
    """C = Pearson correlation between the rows of the expression matrix E
    (genes x samples), the co-expression prior of Sec. II-A (panda_pearson).
    Not z-scored: pass it through normalize like any other prior."""
    torch = _torch()
    lib = load_library()
    G, S = E.shape
    out = torch.empty((G, G), dtype=torch.float32, device="cuda")
    ws = workspace(lib.panda_pearson_workspace_bytes(G, S))
    _check(lib.panda_pearson(_dev(E, "E"), G, S, S, out.data_ptr(), G,
                             ws.data_ptr(), ws.numel(), _stream()))
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def pearson_noalloc(E, C=None, ldc: int | None = None):
    """The same prior through panda_pearson_noalloc (no workspace: the
    library's per-GPU scratch array).  C (optional, device FP32, G rows of
    leading dimension ldc) receives the result; columns past G are left
    alone."""
    torch = _torch()
    lib = load_library()
    G, S = E.shape
    if C is None:
        C = torch.empty((G, G), dtype=torch.float32, device="cuda")
    ldc = C.shape[1] if ldc is None else ldc
    if C.shape[0] != G or C.shape[1] != ldc or ldc < G:
        raise ValueError("C must be G x ldc with ldc >= G")
    _check(lib.panda_pearson_noalloc(_dev(E, "E"), G, S, S, _dev(C, "C"), ldc, _stream()))
    return C


def workspace_bytes(Ne: int, Na: int, opts: Options | None = None) -> int:
    o = opts or default_options()
    return load_library().panda_workspace_bytes(Ne, Na, ct.byref(o))


class Context:
    """Message-passing state (W, P, C, t) held in a caller-owned workspace."""

    def __init__(self, Ne: int, Na: int, opts: Options | None = None, ws=None):
        self.lib = load_library()
        self.Ne, self.Na = int(Ne), int(Na)
        self.opts = opts or default_options()
        need = workspace_bytes(Ne, Na, self.opts)
        if need == 0:
            raise PandaError(ERR_ARG, "bad dimensions")
        self.ws = ws if ws is not None else workspace(need)
        h = ct.c_void_p()
        _check(self.lib.panda_ctx_create(self.Ne, self.Na, ct.byref(self.opts), self.ws.data_ptr(),
                                         self.ws.numel(), _stream(), ct.byref(h)))
        self.h = h

    def load(self, W, P=None, C=None, t: int = 0):
        pw = _dev(W, "W", (self.Ne, self.Na))
        pp = None if P is None else _dev(P, "P", (self.Ne, self.Ne))
        pc = None if C is None else _dev(C, "C", (self.Na, self.Na))
        _check(self.lib.panda_ctx_load(self.h, pw, pp, pc, int(t)))

    def iterate(self):
        """One iteration; returns (h, t)."""
        hv, tv = ct.c_double(), ct.c_int32()
        _check(self.lib.panda_iterate(self.h, ct.byref(hv), ct.byref(tv)))
        return hv.value, tv.value

    def store(self, W=None, P=None, C=None):
        """Copy the state into the given tensors; returns (h, t)."""
        hv, tv = ct.c_double(), ct.c_int32()
        pw = None if W is None else _dev(W, "W", (self.Ne, self.Na))
        pp = None if P is None else _dev(P, "P", (self.Ne, self.Ne))
        pc = None if C is None else _dev(C, "C", (self.Na, self.Na))
        _check(self.lib.panda_ctx_store(self.h, pw, pp, pc, ct.byref(hv), ct.byref(tv)))
        return hv.value, tv.value

    def set_timing(self, enable: bool = True):
        _check(self.lib.panda_ctx_set_timing(self.h, int(enable)))

    def phase_times(self):
        """{phase: (total ms, iterations timed)} since timing was enabled."""
        n = len(PHASES)
        ms = (ct.c_double * n)()
        cnt = (ct.c_int64 * n)()
        _check(self.lib.panda_ctx_phase_times(self.h, ms, cnt))
        return {PHASES[i]: (ms[i], cnt[i]) for i in range(n)}

    def features(self, omegaP, omegaC):
        """Warm-start features of the loaded priors: (F (Ne*Na x 16), tau)."""
        torch = _torch()
        F = torch.empty((self.Ne * self.Na, WS_FEATURES), dtype=torch.float32, device="cuda")
        ws = workspace(self.lib.panda_ws_features_workspace_bytes(self.Ne, self.Na))
        tau = ct.c_double()
        _check(self.lib.panda_ws_features(self.h, _dev(omegaP, "omegaP", (self.Ne, WS_SKETCH)),
                                          _dev(omegaC, "omegaC", (self.Na, WS_SKETCH)),
                                          F.data_ptr(), ct.byref(tau), ws.data_ptr(), ws.numel()))
        return F, tau.value

    def ws_init(self, Wpred, t0: int):
        """Warm state around a predicted W at iteration t0 (panda_ws_init)."""
        _check(self.lib.panda_ws_init(self.h, _dev(Wpred, "Wpred", (self.Ne, self.Na)), int(t0)))

    def state(self):
        torch = _torch()
        W = torch.empty((self.Ne, self.Na), dtype=torch.float32, device="cuda")
        P = torch.empty((self.Ne, self.Ne), dtype=torch.float32, device="cuda")
        C = torch.empty((self.Na, self.Na), dtype=torch.float32, device="cuda")
        h, t = self.store(W, P, C)
        return W, P, C, h, t

    def close(self):
        if self.h:
            self.lib.panda_ctx_destroy(self.h)
            self.h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class RunResult:
    W: object
    P: object
    C: object
    iters: int
    h: float
    status: int


def run(W0, P0=None, C0=None, alpha: float = 0.1, tol: float = 1e-3, max_iter: int = 200,
        opts: Options | None = None, ws=None, out=None) -> RunResult:
    """panda_run: message passing from normalised priors (P0/C0 None = identity)."""
    torch = _torch()
    lib = load_library()
    Ne, Na = W0.shape
    o = opts or default_options()
    if out is None:
        out = (torch.empty((Ne, Na), dtype=torch.float32, device="cuda"),
               torch.empty((Ne, Ne), dtype=torch.float32, device="cuda"),
               torch.empty((Na, Na), dtype=torch.float32, device="cuda"))
    W, P, C = out
    if ws is None:
        ws = workspace(workspace_bytes(Ne, Na, o))
    it, hv = ct.c_int32(), ct.c_double()
    code = lib.panda_run(_dev(W0, "W0", (Ne, Na)),
                         None if P0 is None else _dev(P0, "P0", (Ne, Ne)),
                         None if C0 is None else _dev(C0, "C0", (Na, Na)),
                         Ne, Na, alpha, tol, max_iter,
                         _dev(W, "W"), _dev(P, "P"), _dev(C, "C"), ws.data_ptr(), ws.numel(),
                         ct.byref(o), ct.byref(it), ct.byref(hv), _stream())
    _check(code, allow=(OK, NOT_CONVERGED))
    return RunResult(W, P, C, it.value, hv.value, code)


def _perm_dev(perm, n, name):
    torch = _torch()
    if not isinstance(perm, torch.Tensor) or not perm.is_cuda or perm.dtype != torch.int32:
        raise TypeError(f"{name} must be an int32 tensor on the GPU")
    if not perm.is_contiguous() or perm.shape[-1] != n:
        raise ValueError(f"{name} must be contiguous with rows of {n} entries")
    return perm.data_ptr()


def permute_sym(M, perm):
    """out[i][j] = M[perm[i]][perm[j]] (panda_permute_sym)."""
    torch = _torch()
    n = M.shape[0]
    out = torch.empty((n, n), dtype=torch.float32, device="cuda")
    _check(load_library().panda_permute_sym(_dev(M, "M", (n, n)), n, n, _perm_dev(perm, n, "perm"),
                                            out.data_ptr(), n, _stream()))
    return out


@dataclass
class NullResult:
    mean: object  # Ne x Na, FP32, per-edge mean over the null instances
    sd: object    # Ne x Na, FP32, population standard deviation
    iters: list
    status: int


def null(W0, P0=None, C0=None, gene_perm=None, tf_perm=None, opts: Options | None = None,
         ws=None) -> NullResult:
    """panda_null: PANDA() on K relabelled copies of the priors (genes of C0
    by the rows of gene_perm, TFs of P0 by the rows of tf_perm; int32 device
    tensors K x Na and K x Ne), folded into a per-edge mean and sd."""
    torch = _torch()
    lib = load_library()
    Ne, Na = W0.shape
    o = opts or default_options()
    perms = [p for p in (gene_perm, tf_perm) if p is not None]
    K = perms[0].shape[0] if perms else 1
    if any(p.shape[0] != K for p in perms):
        raise ValueError("gene_perm and tf_perm must have the same number of rows")
    mean = torch.empty((Ne, Na), dtype=torch.float32, device="cuda")
    sd = torch.empty((Ne, Na), dtype=torch.float32, device="cuda")
    if ws is None:
        ws = workspace(lib.panda_null_workspace_bytes(Ne, Na, ct.byref(o)))
    iters = (ct.c_int32 * K)()
    code = lib.panda_null(_dev(W0, "W0", (Ne, Na)),
                          None if P0 is None else _dev(P0, "P0", (Ne, Ne)),
                          None if C0 is None else _dev(C0, "C0", (Na, Na)), Ne, Na, K,
                          None if gene_perm is None else _perm_dev(gene_perm, Na, "gene_perm"),
                          None if tf_perm is None else _perm_dev(tf_perm, Ne, "tf_perm"),
                          ct.byref(o), ws.data_ptr(), ws.numel(), mean.data_ptr(), sd.data_ptr(),
                          iters, _stream())
    _check(code, allow=(OK, NOT_CONVERGED))
    return NullResult(mean, sd, list(iters), code)


def null_zscore(W, mean, sd):
    """z = (W - mean) / sd per edge, 0 where sd = 0 (panda_null_zscore)."""
    torch = _torch()
    Ne, Na = W.shape
    z = torch.empty((Ne, Na), dtype=torch.float32, device="cuda")
    _check(load_library().panda_null_zscore(_dev(W, "W", (Ne, Na)), _dev(mean, "mean", (Ne, Na)),
                                            _dev(sd, "sd", (Ne, Na)), Ne, Na, z.data_ptr(),
                                            _stream()))
    return z


def _shape_arrays(shapes):
    n = len(shapes)
    Ne = (ct.c_int64 * n)(*[int(a) for a, _ in shapes])
    Na = (ct.c_int64 * n)(*[int(b) for _, b in shapes])
    return n, Ne, Na


def batch_workspace_bytes(shapes, opts: Options | None = None) -> int:
    """Workspace of a batch of networks with shapes [(Ne, Na), ...]."""
    o = opts or default_options()
    n, Ne, Na = _shape_arrays(shapes)
    return load_library().panda_batch_workspace_bytes(n, Ne, Na, ct.byref(o))


class Batch:
    """Independent networks iterating together in grouped launches."""

    def __init__(self, shapes, opts: Options | None = None, ws=None):
        self.lib = load_library()
        self.shapes = [(int(a), int(b)) for a, b in shapes]
        self.opts = opts or default_options()
        need = batch_workspace_bytes(self.shapes, self.opts)
        if need == 0:
            raise PandaError(ERR_ARG, "bad batch shapes")
        self.ws = ws if ws is not None else workspace(need)
        n, Ne, Na = _shape_arrays(self.shapes)
        h = ct.c_void_p()
        _check(self.lib.panda_batch_create(n, Ne, Na, ct.byref(self.opts), self.ws.data_ptr(),
                                           self.ws.numel(), _stream(), ct.byref(h)))
        self.h = h

    def __len__(self):
        return len(self.shapes)

    @staticmethod
    def candidates():
        lib = load_library()
        return [lib.panda_batch_tile_candidates(p) for p in range(len(BATCH_TILES))]

    @property
    def tiles(self):
        c = (ct.c_int32 * len(BATCH_TILES))()
        _check(self.lib.panda_batch_get_tiles(self.h, c))
        return list(c)

    @tiles.setter
    def tiles(self, choice):
        c = (ct.c_int32 * len(BATCH_TILES))(*[int(x) for x in choice])
        _check(self.lib.panda_batch_set_tiles(self.h, c))

    def autotune(self, reps: int = 3):
        """Pick the fastest tile of every grouped product (before loading);
        returns {product: best ms}."""
        ms = (ct.c_float * len(BATCH_TILES))()
        _check(self.lib.panda_batch_autotune(self.h, int(reps), ms))
        return dict(zip(BATCH_TILES, list(ms)))

    def load(self, i: int, W, P=None, C=None, t: int = 0):
        Ne, Na = self.shapes[i]
        pw = _dev(W, "W", (Ne, Na))
        pp = None if P is None else _dev(P, "P", (Ne, Ne))
        pc = None if C is None else _dev(C, "C", (Na, Na))
        _check(self.lib.panda_batch_load(self.h, int(i), pw, pp, pc, int(t)))

    def iterate(self, steps: int = 1, graph: bool = False) -> int:
        """steps iterations; returns how many networks are still iterating."""
        a = ct.c_int32()
        _check(self.lib.panda_batch_iterate(self.h, int(steps), int(graph), ct.byref(a)))
        return a.value

    def run(self, graph: bool = True):
        """Iterate to convergence (or max_iter); returns (status, steps)."""
        st = ct.c_int32()
        code = self.lib.panda_batch_run(self.h, int(graph), ct.byref(st))
        _check(code, allow=(OK, NOT_CONVERGED))
        return code, st.value

    def status(self, i: int):
        """(h, t, still iterating) of network i at the last read-back."""
        hv, tv, av = ct.c_double(), ct.c_int32(), ct.c_int32()
        _check(self.lib.panda_batch_state(self.h, int(i), ct.byref(hv), ct.byref(tv),
                                          ct.byref(av)))
        return hv.value, tv.value, bool(av.value)

    def state(self, i: int):
        torch = _torch()
        Ne, Na = self.shapes[i]
        W = torch.empty((Ne, Na), dtype=torch.float32, device="cuda")
        P = torch.empty((Ne, Ne), dtype=torch.float32, device="cuda")
        C = torch.empty((Na, Na), dtype=torch.float32, device="cuda")
        hv, tv = ct.c_double(), ct.c_int32()
        _check(self.lib.panda_batch_store(self.h, int(i), W.data_ptr(), P.data_ptr(),
                                          C.data_ptr(), ct.byref(hv), ct.byref(tv)))
        return W, P, C, hv.value, tv.value

    def close(self):
        if self.h:
            self.lib.panda_batch_destroy(self.h)
            self.h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------- warm start ---

def mlp_forward(params, F):
    """y for every row of F (panda_mlp_forward)."""
    torch = _torch()
    n = F.shape[0]
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    _check(load_library().panda_mlp_forward(_dev(params, "params", (MLP_PARAMS,)),
                                            _dev(F, "F", (n, WS_FEATURES)), n, y.data_ptr(),
                                            _stream()))
    return y


def mlp_grad(params, F, target, idx=None, n=None, ws=None):
    """(gradient, loss as a device double) of the MSE over a batch (panda_mlp_grad)."""
    torch = _torch()
    lib = load_library()
    nrows = F.shape[0]
    if idx is not None:
        if idx.dtype != torch.int64 or not idx.is_cuda or not idx.is_contiguous():
            raise TypeError("idx must be a contiguous int64 tensor on the GPU")
        n = idx.numel() if n is None else n
    n = nrows if n is None else n
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    if ws is None:
        ws = workspace(lib.panda_mlp_grad_workspace_bytes(n))
    _check(lib.panda_mlp_grad(_dev(params, "params", (MLP_PARAMS,)), _dev(F, "F", (nrows, WS_FEATURES)),
                              nrows, _dev(target, "target", (nrows,)),
                              None if idx is None else idx.data_ptr(), n, grad.data_ptr(),
                              loss.data_ptr(), ws.data_ptr(), ws.numel(), _stream()))
    return grad, loss


def mlp_adam(params, m, v, grad, step: int, lr: float = 1e-3, beta1: float = 0.9,
             beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update of params in place (panda_mlp_adam)."""
    _check(load_library().panda_mlp_adam(
        _dev(params, "params", (MLP_PARAMS,)), _dev(m, "m", (MLP_PARAMS,)),
        _dev(v, "v", (MLP_PARAMS,)), _dev(grad, "grad", (MLP_PARAMS,)), int(step), lr, beta1,
        beta2, eps, _stream()))


def ws_target(W0, Wstar, tau: float):
    torch = _torch()
    rows, cols = W0.shape
    out = torch.empty_like(W0)
    _check(load_library().panda_ws_target(_dev(W0, "W0"), _dev(Wstar, "Wstar", (rows, cols)),
                                          rows, cols, float(tau), out.data_ptr(), _stream()))
    return out


def ws_predict(W0, y, tau: float):
    torch = _torch()
    rows, cols = W0.shape
    out = torch.empty_like(W0)
    _check(load_library().panda_ws_predict(_dev(W0, "W0"), _dev(y, "y"), rows, cols, float(tau),
                                           out.data_ptr(), _stream()))
    return out
