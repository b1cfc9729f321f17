"""ctypes binding of libfastpi.so: argument marshalling only.

Every step of the FastPI path runs inside the library (host reordering and planning in
C++, everything else in HIP kernels on the device). PyTorch supplies device memory and the
stream. There is no fallback: if the library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# FASTPI_LIBRARY names another build of the same library (the host-sanitizer build)
LIB_PATH = os.environ.get("FASTPI_LIBRARY") or os.path.join(HERE, "libfastpi.so")

FP64, MIXED = 0, 1

STATUS = {1: "WFLOOR", 0: "OK", -1: "EINVAL", -2: "ESHAPE", -3: "ENONFINITE", -4: "ENOMEM", -5: "EHIP",
          -6: "ENOCONV", -7: "EINTERNAL"}


class FastPIError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"fastpi {STATUS.get(code, code)}: {message}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class Split(ctypes.Structure):
    _fields_ = [(name, c_int64) for name in
                ("m", "n", "nnz", "m1", "n1", "m2", "n2", "B", "B_dense", "T_it", "s_b", "s", "r")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class Options(ctypes.Structure):
    _fields_ = [("precision", c_int), ("max_sweeps", c_int), ("tol", c_double),
                ("max_workspace_bytes", c_size_t)]


class Tuning(ctypes.Structure):
    _fields_ = [("block_lds", c_int32), ("block_wgs_per_cu", c_int32), ("gram_rows", c_int32),
                ("inner_sweeps", c_int32), ("precond", c_int32), ("eig_fused", c_int32)]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


# (name, restype, argtypes) of every symbol declared in include/fastpi.h
class Inner(ctypes.Structure):
    """Inner solver of the two updates: mode 0 exact, 1 randomized where t < ceil(0.3 q),
    2 randomized wherever t + oversample < q."""
    _fields_ = [("mode", ctypes.c_int32), ("oversample", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("seed", ctypes.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class CoreSolver(ctypes.Structure):
    """Core solver of the exact branch: mode 0 Jacobi on G, 1 subspace iteration where it
    applies (see include/fastpi.h)."""
    _fields_ = [("mode", c_int32), ("min_order", c_int32), ("k_factor", c_double), ("max_frac", c_double),
                ("iters_fp64", c_int32), ("iters_mixed", c_int32), ("orth_every", c_int32), ("pad", c_int32),
                ("res_tol_fp64", c_double), ("res_tol_mixed", c_double), ("k_factor_mixed", c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


class RankModel(ctypes.Structure):
    """Training statistics of the rank network's 16 block features (fastpi_rank_model)."""
    _fields_ = [("mean", c_void_p), ("std", c_void_p), ("lo", c_void_p), ("hi", c_void_p),
                ("margin", c_double)]


def _rank_model(mean, std, lo, hi, margin):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (mean, std, lo, hi)]
    for a in arrs:
        assert a.shape == (16,)
    return RankModel(*[_ptr(a) for a in arrs], float(margin)), arrs   # arrs keeps the memory alive


def rank_inputs(feats, mean, std, lo, hi, margin):
    """The rank network's standardised inputs (float32 [n, 16]) and range flags (bool [n])."""
    feats = np.ascontiguousarray(feats, dtype=np.float64).reshape(-1, 16)
    n = feats.shape[0]
    X = np.empty((n, 16), dtype=np.float32)
    ok = np.empty(n, dtype=np.int32)
    model, keep = _rank_model(mean, std, lo, hi, margin)
    _check(load().fastpi_rank_inputs(n, _ptr(feats), ctypes.byref(model), _ptr(X), _ptr(ok)))
    del keep
    return X, ok.astype(bool)


def rank_allocate(f, q, budget):
    """Integer ranks in [0, q_i] summing to min(budget, sum q), in proportion to f_i q_i."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.int64)
    assert f.shape == q.shape
    out = np.empty(q.shape, dtype=np.int64)
    _check(load().fastpi_rank_allocate(q.size, _ptr(f), _ptr(q), int(budget), _ptr(out)))
    return out


ROUTES = {0: "jacobi", 1: "subspace", 2: "subspace+jacobi", 3: "randomized"}

SIGNATURES = [
    ("fastpi_target_rank", c_int64, [c_double, c_int64]),
    ("fastpi_reorder", c_int, [c_int64, c_int64, c_void_p, c_void_p, c_void_p, c_double, c_void_p,
                               c_void_p, c_void_p, c_int64, POINTER(c_int64), POINTER(Split)]),
    ("fastpi_plan_create", c_int, [POINTER(c_void_p), c_int64, c_int64, c_void_p, c_void_p,
                                   c_void_p, c_double, c_double]),
    ("fastpi_plan_info", c_int, [c_void_p, POINTER(Split)]),
    ("fastpi_plan_permutation", c_int, [c_void_p, c_void_p, c_void_p]),
    ("fastpi_plan_blocks", c_int, [c_void_p, c_void_p]),
    ("fastpi_plan_block_ranks", c_int, [c_void_p, c_void_p]),
    ("fastpi_plan_destroy", None, [c_void_p]),
    ("fastpi_create", c_int, [POINTER(c_void_p), c_int, c_void_p, POINTER(Options)]),
    ("fastpi_set_precision", c_int, [c_void_p, c_int]),
    ("fastpi_destroy", None, [c_void_p]),
    ("fastpi_upload_plan", c_int, [c_void_p, c_void_p]),
    ("fastpi_svd", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("fastpi_apply", c_int, [c_void_p, c_int64, c_int64, c_int64, c_void_p, c_void_p, c_void_p,
                             c_int64, c_void_p, c_void_p]),
    ("fastpi_apply_noalloc", c_int, [c_void_p, c_int64, c_int64, c_int64, c_void_p, c_void_p, c_void_p,
                                     c_int64, c_void_p, c_void_p]),
    ("fastpi_stage_output", c_int, [c_void_p, c_int, c_void_p, c_int64]),
    ("fastpi_syev_top", c_int, [c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_void_p]),
    ("fastpi_sync", c_int, [c_void_p]),
    ("fastpi_last_sweeps", c_int, [c_void_p, c_void_p]),
    ("fastpi_block_features", c_int, [c_void_p, c_void_p, c_void_p]),
    ("fastpi_plan_set_block_ranks", c_int, [c_void_p, c_void_p]),
    ("fastpi_rank_inputs", c_int, [c_int64, c_void_p, POINTER(RankModel), c_void_p, c_void_p]),
    ("fastpi_rank_allocate", c_int, [c_int64, c_void_p, c_void_p, c_int64, c_void_p]),
    ("fastpi_plan_learned_ranks", c_int, [c_void_p, c_void_p, c_void_p, POINTER(RankModel), c_void_p, c_void_p]),
    ("fastpi_mlp_param_count", c_int, []),
    ("fastpi_mlp_forward", c_int, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
    ("fastpi_mlp_gradient", c_int, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("fastpi_mlp_adam", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int64,
                                ctypes.c_float]),
    ("fastpi_timing_start", c_int, [c_void_p, c_int]),
    ("fastpi_timing_read", c_int, [c_void_p, POINTER(c_int64), POINTER(c_double)]),
    ("fastpi_last_rotations", c_int, [c_void_p, c_void_p]),
    ("fastpi_batch_rotations", c_int, [c_void_p, c_void_p]),
    ("fastpi_set_graph", c_int, [c_void_p, c_int]),
    ("fastpi_last_graph_launches", c_int64, [c_void_p]),
    ("fastpi_set_tuning", c_int, [c_void_p, POINTER(Tuning)]),
    ("fastpi_get_tuning", c_int, [c_void_p, POINTER(Tuning)]),
    ("fastpi_set_tuning_cache", c_int, [c_void_p, ctypes.c_char_p]),
    ("fastpi_autotune", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_char_p,
                                c_int64]),
    ("fastpi_batch_create", c_int, [POINTER(c_void_p), c_void_p, c_int64, POINTER(c_void_p)]),
    ("fastpi_batch_destroy", None, [c_void_p]),
    ("fastpi_batch_svd", c_int, [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                 POINTER(c_void_p)]),
    ("fastpi_batch_sync", c_int, [c_void_p, c_void_p, c_void_p]),
    ("fastpi_batch_set_graph", c_int, [c_void_p, c_int]),
    ("fastpi_batch_last_graph_launches", c_int64, [c_void_p]),
    ("fastpi_batch_set_tuning", c_int, [c_void_p, POINTER(Tuning)]),
    ("fastpi_batch_get_tuning", c_int, [c_void_p, POINTER(Tuning)]),
    ("fastpi_batch_autotune", c_int, [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                      POINTER(c_void_p), ctypes.c_char_p, c_int64]),
    ("fastpi_labels_create", c_int, [POINTER(c_void_p), c_void_p, c_int64, c_int64, c_void_p, c_void_p,
                                     c_void_p]),
    ("fastpi_labels_destroy", None, [c_void_p]),
    ("fastpi_labels_nnz", c_int, [c_void_p, POINTER(c_int64)]),
    ("fastpi_apply_sparse", c_int, [c_void_p, c_int64, c_int64, c_int64, c_void_p, c_void_p, c_void_p,
                                    c_void_p, c_void_p]),
    ("fastpi_topk_hits", c_int, [c_void_p, c_int64, c_int64, c_int64, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p, ctypes.c_int32, c_void_p, c_void_p]),
    ("fastpi_set_block_route", c_int, [c_void_p, c_double]),
    ("fastpi_reorder_gpu", c_int, [c_void_p, c_int64, c_int64, c_int64, c_void_p, c_void_p, c_void_p, c_double,
                                   c_void_p, c_void_p, c_void_p, c_int64, POINTER(c_int64), POINTER(Split)]),
    ("fastpi_plan_create_gpu", c_int, [POINTER(c_void_p), c_void_p, c_int64, c_int64, c_void_p, c_void_p,
                                       c_void_p, c_double, c_double]),
    ("fastpi_batch_set_block_route", c_int, [c_void_p, c_double]),
    ("fastpi_set_inner", c_int, [c_void_p, POINTER(Inner)]),
    ("fastpi_get_inner", c_int, [c_void_p, POINTER(Inner)]),
    ("fastpi_batch_set_inner", c_int, [c_void_p, POINTER(Inner)]),
    ("fastpi_inner_applies", c_int, [POINTER(Inner), c_int64, c_int64]),
    ("fastpi_gaussian", c_int, [c_void_p, c_int64, ctypes.c_uint32, ctypes.c_uint32, c_void_p]),
    ("fastpi_set_core_solver", c_int, [c_void_p, POINTER(CoreSolver)]),
    ("fastpi_get_core_solver", c_int, [c_void_p, POINTER(CoreSolver)]),
    ("fastpi_batch_set_core_solver", c_int, [c_void_p, POINTER(CoreSolver)]),
    ("fastpi_last_core_routes", c_int, [c_void_p, c_void_p]),
    ("fastpi_batch_core_routes", c_int, [c_void_p, c_void_p]),
    ("fastpi_mfma_gemm", c_int, [c_void_p, c_int, c_int, c_int64, c_int64, c_int64, c_void_p, c_int64, c_void_p,
                                 c_int64, c_void_p, c_int64, c_int]),
    ("fastpi_last_error", ctypes.c_char_p, []),
]

_lib = None


def load(path: str = LIB_PATH):
    """Loads the library once; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FastPIError(-7, f"{path} is not built; run paper_2011_04235_amd/build.py")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(code):
    if code != 0:
        msg = load().fastpi_last_error()
        raise FastPIError(code, msg.decode() if msg else "")


def _ptr(a: np.ndarray):
    return c_void_p(a.ctypes.data) if a is not None else None


def inner_applies(mode, oversample, t, q):
    """Whether the inner-solver setting takes the randomized branch for target rank t and
    order q (the library's own rule)."""
    return bool(load().fastpi_inner_applies(ctypes.byref(Inner(int(mode), int(oversample), 0, 0)), int(t), int(q)))


def target_rank(alpha: float, x: int) -> int:
    return int(load().fastpi_target_rank(float(alpha), int(x)))


def reorder(m, n, indptr, indices, data=None, k=0.01):
    """Host reordering (Algorithm 2). Returns (piT, piF, blocks[B, 4], split dict)."""
    lib = load()
    indptr = np.ascontiguousarray(indptr, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.int32)
    data = None if data is None else np.ascontiguousarray(data, dtype=np.float64)
    piT = np.empty(m, dtype=np.int32)
    piF = np.empty(n, dtype=np.int32)
    nb = c_int64(0)
    sp = Split()
    _check(lib.fastpi_reorder(m, n, _ptr(indptr), _ptr(indices), _ptr(data), float(k), _ptr(piT),
                              _ptr(piF), None, 0, ctypes.byref(nb), ctypes.byref(sp)))
    blocks = np.empty((nb.value, 4), dtype=np.int64)
    _check(lib.fastpi_reorder(m, n, _ptr(indptr), _ptr(indices), _ptr(data), float(k), _ptr(piT),
                              _ptr(piF), _ptr(blocks), nb.value, ctypes.byref(nb), ctypes.byref(sp)))
    return piT, piF, blocks, sp.as_dict()


class Plan:
    """Reordering + ranks + value maps for one pattern and one alpha (host, C++)."""

    def __init__(self, m, n, indptr, indices, data=None, alpha=0.2, k=0.01, gpu=None):
        """gpu: a Handle to run the reordering on its device (the plan is the same)."""
        lib = load()
        indptr = np.ascontiguousarray(indptr, dtype=np.int64)
        indices = np.ascontiguousarray(indices, dtype=np.int32)
        data = None if data is None else np.ascontiguousarray(data, dtype=np.float64)
        h = c_void_p()
        if gpu is None:
            _check(lib.fastpi_plan_create(ctypes.byref(h), int(m), int(n), _ptr(indptr), _ptr(indices),
                                          _ptr(data), float(alpha), float(k)))
        else:
            _check(lib.fastpi_plan_create_gpu(ctypes.byref(h), gpu._h, int(m), int(n), _ptr(indptr),
                                              _ptr(indices), _ptr(data), float(alpha), float(k)))
        self._h = h
        self.alpha = alpha
        self.k = k
        sp = Split()
        _check(lib.fastpi_plan_info(h, ctypes.byref(sp)))
        self.info = sp.as_dict()

    def __getattr__(self, name):
        info = self.__dict__.get("info")
        if info is not None and name in info:
            return info[name]
        raise AttributeError(name)

    def permutation(self):
        piT = np.empty(self.info["m"], dtype=np.int32)
        piF = np.empty(self.info["n"], dtype=np.int32)
        _check(load().fastpi_plan_permutation(self._h, _ptr(piT), _ptr(piF)))
        return piT, piF

    def blocks(self):
        out = np.empty((self.info["B"], 4), dtype=np.int64)
        if self.info["B"]:
            _check(load().fastpi_plan_blocks(self._h, _ptr(out)))
        return out

    def block_ranks(self):
        out = np.empty(self.info["B"], dtype=np.int64)
        if self.info["B"]:
            _check(load().fastpi_plan_block_ranks(self._h, _ptr(out)))
        return out

    def block_features(self, data):
        """16 features of every dense diagonal block, in block order (host)."""
        data = np.ascontiguousarray(data, dtype=np.float64)
        out = np.empty((self.info["B_dense"], 16), dtype=np.float64)
        if out.size:
            _check(load().fastpi_block_features(self._h, _ptr(data), _ptr(out)))
        return out

    def learned_ranks(self, handle, data, theta, mean, std, lo, hi, margin):
        """Per-block ranks of the learned allocation (fastpi_plan_learned_ranks): theta is the
        network's packed parameters on the handle's device (float32 tensor)."""
        data = np.ascontiguousarray(data, dtype=np.float64)
        out = np.empty(self.info["B"], dtype=np.int64)
        model, keep = _rank_model(mean, std, lo, hi, margin)
        assert theta.dtype == handle.torch.float32 and theta.is_contiguous()
        _check(load().fastpi_plan_learned_ranks(self._h, handle._h, _ptr(data), ctypes.byref(model),
                                                _dptr(theta), _ptr(out)))
        del keep
        return out

    def set_block_ranks(self, ranks):
        """Per-block ranks (one per block of the block table); refreshes the shape info."""
        ranks = np.ascontiguousarray(ranks, dtype=np.int64)
        assert ranks.shape == (self.info["B"],)
        _check(load().fastpi_plan_set_block_ranks(self._h, _ptr(ranks)))
        sp = Split()
        _check(load().fastpi_plan_info(self._h, ctypes.byref(sp)))
        self.info = sp.as_dict()

    def __del__(self):
        h = self.__dict__.get("_h")
        if h is not None and _lib is not None:
            _lib.fastpi_plan_destroy(h)
            self._h = None


def _dptr(t):
    return c_void_p(t.data_ptr()) if t is not None else None


class Handle:
    """Device handle bound to a torch device and its current stream."""

    def __init__(self, device=0, precision="fp64", max_sweeps=0, tol=0.0, max_workspace_bytes=0,
                 stream=None):
        import torch
        lib = load()
        self.torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        opts = Options(FP64 if precision == "fp64" else MIXED, int(max_sweeps), float(tol),
                       int(max_workspace_bytes))
        h = c_void_p()
        _check(lib.fastpi_create(ctypes.byref(h), int(device), c_void_p(stream.cuda_stream),
                                 ctypes.byref(opts)))
        self._h = h
        self.plan = None

    def set_precision(self, precision):
        _check(load().fastpi_set_precision(self._h, FP64 if precision == "fp64" else MIXED))

    def upload_plan(self, plan: Plan):
        _check(load().fastpi_upload_plan(self._h, plan._h))
        self.plan = plan

    def svd(self, rowptr, col, val, out=None):
        """Low-rank SVD of the uploaded plan's matrix; device tensors in, (U, S, V) out."""
        torch = self.torch
        info = self.plan.info
        m, n, r = info["m"], info["n"], info["r"]
        if out is None:
            U = torch.empty((m, r), dtype=torch.float64, device=self.device)
            S = torch.empty((r,), dtype=torch.float64, device=self.device)
            V = torch.empty((n, r), dtype=torch.float64, device=self.device)
        else:
            U, S, V = out
        for t in (rowptr, col, val, U, S, V):
            assert t.is_contiguous() and t.device == self.device
        assert rowptr.dtype == torch.int64 and col.dtype == torch.int32 and val.dtype == torch.float64
        _check(load().fastpi_svd(self._h, _dptr(rowptr), _dptr(col), _dptr(val), _dptr(U), _dptr(S),
                                 _dptr(V)))
        return U, S, V

    def apply(self, U, S, V, Y, out=None):
        torch = self.torch
        m, r = U.shape
        n = V.shape[0]
        L = Y.shape[1]
        Z = torch.empty((n, L), dtype=torch.float64, device=self.device) if out is None else out
        for t in (U, S, V, Y, Z):
            assert t.is_contiguous() and t.dtype == torch.float64 and t.device == self.device
        _check(load().fastpi_apply(self._h, m, n, r, _dptr(U), _dptr(S), _dptr(V), L, _dptr(Y),
                                   _dptr(Z)))
        return Z

    def apply_noalloc(self, U, S, V, Y, out):
        """fastpi_apply without device allocation (the library's fixed per-GPU scratch); `out`
        must be given."""
        torch = self.torch
        m, r = U.shape
        n = V.shape[0]
        L = Y.shape[1]
        for t in (U, S, V, Y, out):
            assert t.is_contiguous() and t.dtype == torch.float64 and t.device == self.device
        _check(load().fastpi_apply_noalloc(self._h, m, n, r, _dptr(U), _dptr(S), _dptr(V), L, _dptr(Y),
                                           _dptr(out)))
        return out

    def reorder(self, m, n, rowptr, col, val=None, k=0.01):
        """Algorithm 2 on this handle's GPU from a device CSR (torch tensors); returns
        (piT, piF, blocks[B, 4], split dict) on the host, as reorder()."""
        nnz = int(col.shape[0])
        piT = np.empty(m, dtype=np.int32)
        piF = np.empty(n, dtype=np.int32)
        nb = c_int64(0)
        spl = Split()
        lib = load()
        _check(lib.fastpi_reorder_gpu(self._h, int(m), int(n), nnz, _dptr(rowptr), _dptr(col), _dptr(val),
                                      float(k), _ptr(piT), _ptr(piF), None, 0, ctypes.byref(nb), ctypes.byref(spl)))
        blocks = np.empty((nb.value, 4), dtype=np.int64)
        _check(lib.fastpi_reorder_gpu(self._h, int(m), int(n), nnz, _dptr(rowptr), _dptr(col), _dptr(val),
                                      float(k), _ptr(piT), _ptr(piF), _ptr(blocks), nb.value, ctypes.byref(nb),
                                      ctypes.byref(spl)))
        return piT, piF, blocks, spl.as_dict()

    def set_block_route(self, min_cost):
        """Blocks with p q^2 >= min_cost take the Gram route (default 1e6)."""
        _check(load().fastpi_set_block_route(self._h, float(min_cost)))

    def set_inner(self, mode=1, oversample=5, iters=11, seed=0):
        """Inner solver of the two updates (see Inner); kept across upload_plan."""
        _check(load().fastpi_set_inner(self._h, ctypes.byref(Inner(int(mode), int(oversample), int(iters),
                                                                     int(seed)))))

    def set_core_solver(self, **kw):
        """Updates the core-solver fields given (mode, min_order, k_factor, k_factor_mixed,
        max_frac, iters_fp64, iters_mixed, orth_every, res_tol_fp64, res_tol_mixed)."""
        c = CoreSolver()
        _check(load().fastpi_get_core_solver(self._h, ctypes.byref(c)))
        for key, v in kw.items():
            setattr(c, key, v)
        _check(load().fastpi_set_core_solver(self._h, ctypes.byref(c)))

    def get_core_solver(self):
        c = CoreSolver()
        _check(load().fastpi_get_core_solver(self._h, ctypes.byref(c)))
        return c.as_dict()

    def last_core_routes(self):
        """[row-update core, column-update core] route names of the last svd."""
        out = np.zeros(2, dtype=np.int32)
        _check(load().fastpi_last_core_routes(self._h, _ptr(out)))
        return [ROUTES[int(x)] for x in out]

    def get_inner(self):
        out = Inner()
        _check(load().fastpi_get_inner(self._h, ctypes.byref(out)))
        return out.as_dict()

    def gaussian(self, count, seed, stream):
        """The randomized branch's test-matrix draws for key (seed, stream) (device tensor)."""
        out = self.torch.empty((int(count),), dtype=self.torch.float64, device=self.device)
        _check(load().fastpi_gaussian(self._h, int(count), int(seed), int(stream), _dptr(out)))
        return out

    def apply_sparse(self, U, S, V, labels, out=None):
        """Z = V diag(S^+) U^T Y for a sparse label matrix (a Labels object)."""
        torch = self.torch
        m, r = U.shape
        n = V.shape[0]
        Z = torch.empty((n, labels.L), dtype=torch.float64, device=self.device) if out is None else out
        for t in (U, S, V, Z):
            assert t.is_contiguous() and t.dtype == torch.float64 and t.device == self.device
        _check(load().fastpi_apply_sparse(self._h, m, n, r, _dptr(U), _dptr(S), _dptr(V), labels._y,
                                          _dptr(Z)))
        return Z

    def topk_hits(self, rowptr, col, val, Z, y_rowptr, y_col, ks, out=None):
        """Top-k hit counts of held-out rows (device CSR features and labels); returns a
        device int32 tensor [rows, len(ks)]."""
        torch = self.torch
        rows = rowptr.shape[0] - 1
        n, L = Z.shape
        ks_h = np.ascontiguousarray(ks, dtype=np.int32)
        hits = torch.empty((rows, ks_h.size), dtype=torch.int32, device=self.device) if out is None else out
        for t in (rowptr, col, val, Z, y_rowptr, y_col, hits):
            assert t.is_contiguous() and t.device == self.device
        assert rowptr.dtype == torch.int64 and y_rowptr.dtype == torch.int64
        assert col.dtype == torch.int32 and y_col.dtype == torch.int32
        assert val.dtype == torch.float64 and Z.dtype == torch.float64
        _check(load().fastpi_topk_hits(self._h, rows, n, L, _dptr(rowptr), _dptr(col), _dptr(val), _dptr(Z),
                                       _dptr(y_rowptr), _dptr(y_col), int(ks_h.size), _ptr(ks_h),
                                       _dptr(hits)))
        return hits

    def stage_output(self, which):
        torch = self.torch
        info = self.plan.info
        sizes = {0: (info["s_b"],), 1: (info["s"],), 2: (info["n1"], info["s"]),
                 3: (info["m"], info["s"])}
        out = torch.empty(sizes[which], dtype=torch.float64, device=self.device)
        _check(load().fastpi_stage_output(self._h, int(which), _dptr(out), out.numel()))
        return out

    def mfma_gemm(self, A, B, ta=False, tb=False, fp32=False, out=None):
        """C = op(A) op(B) by the library's matrix-core product (a stage-level check)."""
        torch = self.torch
        M = A.shape[1] if ta else A.shape[0]
        K = A.shape[0] if ta else A.shape[1]
        N = B.shape[0] if tb else B.shape[1]
        C = torch.empty((M, N), dtype=torch.float64, device=self.device) if out is None else out
        _check(load().fastpi_mfma_gemm(self._h, int(ta), int(tb), M, N, K, _dptr(A), A.stride(0), _dptr(B),
                                       B.stride(0), _dptr(C), C.stride(0), int(fp32)))
        return C

    def syev_top(self, G, t):
        torch = self.torch
        q = G.shape[0]
        vals = torch.empty((t,), dtype=torch.float64, device=self.device)
        vecs = torch.empty((q, t), dtype=torch.float64, device=self.device)
        _check(load().fastpi_syev_top(self._h, q, _dptr(G), t, _dptr(vals), _dptr(vecs)))
        return vals, vecs

    def sync(self):
        """Waits; raises on an error code, returns "OK" or the warning "WFLOOR" (a kept singular
        value under the Gram floor, returned as 0)."""
        code = load().fastpi_sync(self._h)
        if code < 0:
            _check(code)
        return STATUS[code]

    def last_sweeps(self):
        out = np.zeros(3, dtype=np.int32)
        _check(load().fastpi_last_sweeps(self._h, _ptr(out)))
        return out.tolist()

    KERNELS = {"eig_gram": 0, "eig_solve": 1, "eig_update": 2, "block_svd": 3, "label_spmm": 4,
               "topk": 5, "gemm_nt": 6, "sub_gemm": 7, "cq_panel": 8, "eig_round": 9}

    def last_rotations(self):
        """Pair solves that ran in the last svd: [row-update core, column-update core]."""
        out = np.zeros(2, dtype=np.int64)
        _check(load().fastpi_last_rotations(self._h, _ptr(out)))
        return out.tolist()

    # ---- batching form: graphs and schedules ----
    def set_graph(self, enable=True):
        _check(load().fastpi_set_graph(self._h, 1 if enable else 0))

    def last_graph_launches(self):
        return int(load().fastpi_last_graph_launches(self._h))

    def set_tuning(self, **kw):
        t = Tuning(**{**self.get_tuning(), **kw})
        _check(load().fastpi_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self):
        t = Tuning()
        _check(load().fastpi_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning_cache(self, path):
        _check(load().fastpi_set_tuning_cache(self._h, None if path is None else str(path).encode()))

    def autotune(self, rowptr, col, val, out=None):
        """Times the candidate schedules on this matrix and keeps the fastest (synchronous).
        Returns the timing report."""
        U, S, V = out if out is not None else self._outputs()
        buf = ctypes.create_string_buffer(4096)
        _check(load().fastpi_autotune(self._h, _dptr(val), _dptr(U), _dptr(S), _dptr(V), buf, 4096))
        return buf.value.decode()

    def _outputs(self):
        torch = self.torch
        info = self.plan.info
        m, n, r = info["m"], info["n"], info["r"]
        return (torch.empty((m, r), dtype=torch.float64, device=self.device),
                torch.empty((r,), dtype=torch.float64, device=self.device),
                torch.empty((n, r), dtype=torch.float64, device=self.device))

    # ---- learned rank predictor (device float32 tensors) ----
    def mlp_forward(self, X, theta):
        f = self.torch.empty((X.shape[0],), dtype=self.torch.float32, device=self.device)
        _check(load().fastpi_mlp_forward(self._h, X.shape[0], _dptr(X), _dptr(theta), _dptr(f)))
        return f

    def mlp_gradient(self, X, y, theta, out=None):
        g = out if out is not None else self.torch.empty_like(theta)
        _check(load().fastpi_mlp_gradient(self._h, X.shape[0], _dptr(X), _dptr(y), _dptr(theta),
                                          _dptr(g)))
        return g

    def mlp_adam(self, theta, grad, m, v, step, lr):
        _check(load().fastpi_mlp_adam(self._h, _dptr(theta), _dptr(grad), _dptr(m), _dptr(v),
                                      int(step), float(lr)))

    def timing_start(self, kernel):
        _check(load().fastpi_timing_start(self._h, self.KERNELS[kernel] if kernel else -1))

    def timing_read(self):
        n = c_int64(0)
        ms = c_double(0.0)
        _check(load().fastpi_timing_read(self._h, ctypes.byref(n), ctypes.byref(ms)))
        return int(n.value), float(ms.value)

    def __del__(self):
        h = self.__dict__.get("_h")
        if h is not None and _lib is not None:
            _lib.fastpi_destroy(h)
            self._h = None


class Labels:
    """A sparse label matrix Y (m x L, host CSR; values default to one) on a handle's device."""

    def __init__(self, handle: Handle, m, L, indptr, indices, data=None):
        lib = load()
        self.m, self.L = int(m), int(L)
        indptr = np.ascontiguousarray(indptr, dtype=np.int64)
        indices = np.ascontiguousarray(indices, dtype=np.int32)
        data = None if data is None else np.ascontiguousarray(data, dtype=np.float64)
        y = c_void_p()
        _check(lib.fastpi_labels_create(ctypes.byref(y), handle._h, self.m, self.L, _ptr(indptr),
                                        _ptr(indices), _ptr(data)))
        self._y = y

    @property
    def nnz(self):
        out = c_int64(0)
        _check(load().fastpi_labels_nnz(self._y, ctypes.byref(out)))
        return out.value

    def __del__(self):
        if getattr(self, "_y", None) is not None and _lib is not None:
            _lib.fastpi_labels_destroy(self._y)
            self._y = None


def _ptr_array(tensors):
    arr = (c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = t.data_ptr()
    return arr


class Batch:
    """Several matrices run together on one handle (one persistent block-SVD launch, batched
    eigensolvers, optional graph replay). The plans' device copies are owned by the batch."""

    def __init__(self, handle: Handle, plans):
        lib = load()
        self.handle = handle
        self.plans = list(plans)
        arr = (c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        b = c_void_p()
        _check(lib.fastpi_batch_create(ctypes.byref(b), handle._h, len(self.plans), arr))
        self._b = b

    def __len__(self):
        return len(self.plans)

    def outputs(self):
        torch = self.handle.torch
        dev = self.handle.device
        out = []
        for p in self.plans:
            m, n, r = p.info["m"], p.info["n"], p.info["r"]
            out.append((torch.empty((m, r), dtype=torch.float64, device=dev),
                        torch.empty((r,), dtype=torch.float64, device=dev),
                        torch.empty((n, r), dtype=torch.float64, device=dev)))
        return out

    def svd(self, vals, out=None):
        """vals: one device float64 tensor of CSR values per matrix. Returns [(U, S, V)]."""
        out = out if out is not None else self.outputs()
        assert len(vals) == len(self.plans) == len(out)
        for v in vals:
            assert v.is_contiguous() and v.dtype == self.handle.torch.float64
        _check(load().fastpi_batch_svd(self._b, _ptr_array(vals), _ptr_array([o[0] for o in out]),
                                       _ptr_array([o[1] for o in out]), _ptr_array([o[2] for o in out])))
        self._keep = (vals, out)
        return out

    def sync(self):
        """Waits; returns (per-matrix status names, sweeps[count, 3]). Raises nothing."""
        st = np.zeros(len(self.plans), dtype=np.int32)
        sw = np.zeros((len(self.plans), 3), dtype=np.int32)
        load().fastpi_batch_sync(self._b, _ptr(st), _ptr(sw))
        return [STATUS.get(int(c), str(int(c))) for c in st], sw

    def set_core_solver(self, **kw):
        c = CoreSolver()
        _check(load().fastpi_get_core_solver(self.handle._h, ctypes.byref(c)))
        for key, v in kw.items():
            setattr(c, key, v)
        _check(load().fastpi_batch_set_core_solver(self._b, ctypes.byref(c)))

    def core_routes(self):
        """Per matrix [row-update, column-update] route names of the last svd."""
        out = np.zeros((len(self.plans), 2), dtype=np.int32)
        _check(load().fastpi_batch_core_routes(self._b, _ptr(out)))
        return [[ROUTES[int(x)] for x in row] for row in out]

    def rotations(self):
        """Pair solves that ran in the last svd, per matrix: array [count, 2]."""
        out = np.zeros((len(self.plans), 2), dtype=np.int64)
        _check(load().fastpi_batch_rotations(self._b, _ptr(out)))
        return out

    def set_graph(self, enable=True):
        _check(load().fastpi_batch_set_graph(self._b, 1 if enable else 0))

    def last_graph_launches(self):
        return int(load().fastpi_batch_last_graph_launches(self._b))

    def set_tuning(self, **kw):
        t = Tuning(**{**self.get_tuning(), **kw})
        _check(load().fastpi_batch_set_tuning(self._b, ctypes.byref(t)))

    def set_block_route(self, min_cost):
        _check(load().fastpi_batch_set_block_route(self._b, float(min_cost)))

    def set_inner(self, mode=1, oversample=5, iters=11, seed=0):
        _check(load().fastpi_batch_set_inner(self._b, ctypes.byref(Inner(int(mode), int(oversample), int(iters),
                                                                           int(seed)))))

    def get_tuning(self):
        t = Tuning()
        _check(load().fastpi_batch_get_tuning(self._b, ctypes.byref(t)))
        return t.as_dict()

    def autotune(self, vals, out=None):
        out = out if out is not None else self.outputs()
        buf = ctypes.create_string_buffer(8192)
        _check(load().fastpi_batch_autotune(self._b, _ptr_array(vals), _ptr_array([o[0] for o in out]),
                                            _ptr_array([o[1] for o in out]), _ptr_array([o[2] for o in out]),
                                            buf, 8192))
        return buf.value.decode()

    def __del__(self):
        b = self.__dict__.get("_b")
        if b is not None and _lib is not None:
            _lib.fastpi_batch_destroy(b)
            self._b = None
