"""Thin ctypes binding of libsgf.so (the C ABI declared in include/sgf.h).

Argument marshalling only: every step of the factorization, the apply and
CG runs in the HIP library.  PyTorch tensors provide device memory and the
stream (``torch.cuda.current_stream().cuda_stream``).  There is no fallback:
if the shared library is missing, importing this module raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgf.so")

SGF_OK, SGF_EINVAL, SGF_ENOTSPD, SGF_ENOMEM, SGF_EDEVICE, SGF_ENOCONV, SGF_ESTATE = range(7)
NEST_ALL_ALL, NEST_2_ALL, NEST_2_2, GEN_ALL_ALL = 0, 1, 2, 3
MAX_BASIS_COLS = 64
NOALLOC_SCRATCH_BYTES = 64 << 20
STOP_ROOT, STOP_PAPER = 0, 1
FP64, FP32, FP32_BF16N = 0, 1, 2

EXPORTED = ["sgf_default_options", "sgf_analyze", "sgf_factorize_numeric", "sgf_factorize", "sgf_autotune",
            "sgf_apply", "sgf_apply_noalloc", "sgf_multiply", "sgf_pcg_solve", "sgf_spmv", "sgf_get_info",
            "sgf_get_perm", "sgf_get_level", "sgf_plan_dry_run", "sgf_profile_enable", "sgf_profile_read", "sgf_profile_select",
            "sgf_set_apply_graph", "sgf_set_persistent", "sgf_set_basis", "sgf_set_low_rank", "sgf_set_pair_kernel", "sgf_set_device_coarsen", "sgf_block_count", "sgf_export_block", "sgf_set_band_apply", "sgf_set_small_apply", "sgf_set_band_elim", "sgf_set_small_compress", "sgf_release", "sgf_estimate_bytes",
            "sgf_server_default_options", "sgf_server_create", "sgf_server_add_operator", "sgf_server_submit",
            "sgf_server_wait", "sgf_server_get_stats", "sgf_server_clock", "sgf_server_destroy",
            "sgf_destroy", "sgf_status_str", "sgf_last_error"]

RANK_FN = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p)


class Options(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("grid", ctypes.c_int32 * 3), ("dofs_per_node", ctypes.c_int32),
                ("q", ctypes.c_int32), ("leaf", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("compress", ctypes.c_int32), ("compress_from_level", ctypes.c_int32),
                ("stop_rule", ctypes.c_int32), ("precision", ctypes.c_int32), ("tiled_min_rows", ctypes.c_int32),
                ("rank_tol", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("n", ctypes.c_int64), ("top_size", ctypes.c_int64),
                ("factor_entries", ctypes.c_int64), ("factor_bytes", ctypes.c_int64),
                ("compressed", ctypes.c_int64), ("factor_flops", ctypes.c_double),
                ("apply_bytes", ctypes.c_double), ("failed_cluster", ctypes.c_int32),
                ("failed_level", ctypes.c_int32), ("device_bytes", ctypes.c_int64)]


class Block(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("cell", ctypes.c_int32), ("m", ctypes.c_int32), ("k", ctypes.c_int32),
                ("r", ctypes.c_int32)]


BLOCK_ELIM, BLOCK_COMP, BLOCK_TOP = 0, 1, 2


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_int64), ("slots", ctypes.c_int32), ("max_batch_rhs", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("op", ctypes.c_int32), ("nrhs", ctypes.c_int32),
                ("status", ctypes.c_int32), ("factorized", ctypes.c_int32), ("batch_rhs", ctypes.c_int32),
                ("slot", ctypes.c_int32), ("iters_max", ctypes.c_int32), ("relres_max", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_end", ctypes.c_double),
                ("t_factor", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("held_bytes", ctypes.c_int64), ("peak_bytes", ctypes.c_int64), ("evictions", ctypes.c_int64),
                ("factorizations", ctypes.c_int64), ("batches", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("cached_operators", ctypes.c_int64)]


class SgfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1907_03406_amd.build`")
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    H = ctypes.c_void_p
    sig = {
        "sgf_default_options": (None, [ctypes.POINTER(Options)]),
        "sgf_analyze": (I32, [I64, P, P, P, ctypes.POINTER(Options), ctypes.POINTER(H)]),
        "sgf_factorize_numeric": (I32, [H, P, P]),
        "sgf_factorize": (I32, [I64, P, P, P, P, ctypes.POINTER(Options), P, ctypes.POINTER(H)]),
        "sgf_autotune": (I32, [H, P, I32, P, P]),
        "sgf_apply": (I32, [H, I32, P, I64, P, I64, P]),
        "sgf_apply_noalloc": (I32, [H, I32, P, I64, P, I64, P]),
        "sgf_multiply": (I32, [H, I32, P, I64, P, I64, P]),
        "sgf_pcg_solve": (I32, [H, I32, P, I64, P, I64, D, I32, P, P, P]),
        "sgf_spmv": (I32, [H, P, P, P]),
        "sgf_get_info": (I32, [H, ctypes.POINTER(Info)]),
        "sgf_get_perm": (I32, [H, P]),
        "sgf_get_level": (I32, [H, I32, P, P, P, P, P]),
        "sgf_plan_dry_run": (I32, [H, RANK_FN, P]),
        "sgf_profile_enable": (I32, [H, I32]),
        "sgf_profile_select": (I32, [H, ctypes.c_char_p]),
        "sgf_set_apply_graph": (I32, [H, I32]),
        "sgf_set_persistent": (I32, [H, I32]),
        "sgf_set_band_apply": (I32, [H, I32]),
        "sgf_set_small_apply": (I32, [H, I32]),
        "sgf_set_band_elim": (I32, [H, I32]),
        "sgf_set_small_compress": (I32, [H, I32]),
        "sgf_set_basis": (I32, [H, I32, P]),
        "sgf_block_count": (I32, [H, I32, P, P]),
        "sgf_export_block": (I32, [H, I32, I32, ctypes.POINTER(Block), P, P, P, P, P]),
        "sgf_set_low_rank": (I32, [H, I32]),
        "sgf_set_pair_kernel": (I32, [H, I32]),
        "sgf_set_device_coarsen": (I32, [H, I32]),
        "sgf_release": (I32, [H]),
        "sgf_estimate_bytes": (I32, [H, I32, P]),
        "sgf_server_default_options": (None, [ctypes.POINTER(ServerOptions)]),
        "sgf_server_create": (I32, [ctypes.POINTER(ServerOptions), ctypes.POINTER(H)]),
        "sgf_server_add_operator": (I32, [H, I64, P, P, P, P, ctypes.POINTER(Options), P]),
        "sgf_server_submit": (I32, [H, I32, I32, I32, P, I64, P, I64, D, I32, P]),
        "sgf_server_wait": (I32, [H, I64, ctypes.POINTER(RequestInfo), P, P]),
        "sgf_server_get_stats": (I32, [H, ctypes.POINTER(ServerStats)]),
        "sgf_server_clock": (D, []),
        "sgf_server_destroy": (I32, [H]),
        "sgf_profile_read": (I32, [H, ctypes.POINTER(KernelStat), I32, P]),
        "sgf_destroy": (I32, [H]),
        "sgf_status_str": (ctypes.c_char_p, [I32]),
        "sgf_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = load_library()


def _check(code):
    if code != SGF_OK:
        raise SgfError(code, _lib.sgf_last_error().decode())


def make_options(dim, grid, dofs_per_node=1, q=1, leaf=8, scheme=NEST_ALL_ALL, compress=True,
                 compress_from_level=1, stop_rule=STOP_ROOT, precision=FP64, rank_tol=0.0, tiled_min_rows=-1):
    o = Options()
    _lib.sgf_default_options(ctypes.byref(o))
    o.dim = dim
    for a in range(3):
        o.grid[a] = int(grid[a]) if a < len(grid) else 1
    o.dofs_per_node = dofs_per_node
    o.q, o.leaf, o.scheme = q, leaf, scheme
    o.compress = 1 if compress else 0
    o.compress_from_level = compress_from_level
    o.stop_rule, o.precision, o.rank_tol = stop_rule, precision, rank_tol
    o.tiled_min_rows = tiled_min_rows
    return o


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if isinstance(a, np.ndarray) else ctypes.c_void_p(a.data_ptr())


def _dev(t, n, what):
    """Checks that ``t`` is what the C ABI expects of a vector argument: a
    CUDA float64 tensor holding an n x nrhs column-major array with leading
    dimension n (1-D of length n, or 2-D of shape (n, nrhs) with strides
    (1, n), e.g. the transpose of a contiguous (nrhs, n) tensor).  Returns
    nrhs."""
    if isinstance(t, np.ndarray) or not hasattr(t, "device"):
        raise ValueError(f"{what}: a CUDA tensor is required, got {type(t).__name__}")
    if t.device.type != "cuda":
        raise ValueError(f"{what}: the tensor is on {t.device}, the library needs device memory")
    if str(t.dtype) != "torch.float64":
        raise ValueError(f"{what}: dtype {t.dtype}, float64 is required")
    if t.dim() == 1:
        if t.shape[0] != n or (n > 1 and t.stride(0) != 1):
            raise ValueError(f"{what}: a contiguous vector of length {n} is required")
        return 1
    if t.dim() != 2 or t.shape[0] != n:
        raise ValueError(f"{what}: shape {tuple(t.shape)}, (n, nrhs) with n = {n} is required")
    if t.shape[1] > 1 and (t.stride(0) != 1 or t.stride(1) != n):
        raise ValueError(f"{what}: strides {t.stride()}, column-major (1, {n}) are required")
    if t.shape[1] == 1 and t.stride(0) != 1:
        raise ValueError(f"{what}: the column must be contiguous")
    return t.shape[1]


def _pair(a, b, n, names):
    na, nb = _dev(a, n, names[0]), _dev(b, n, names[1])
    if na != nb:
        raise ValueError(f"{names[0]} has {na} columns, {names[1]} {nb}")
    return na


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream)


def _vals(v, nnz):
    """CSR values for a numeric factorization: a contiguous CUDA float64
    tensor with one entry per stored pattern entry."""
    if isinstance(v, np.ndarray) or not hasattr(v, "device"):
        raise ValueError("values: a CUDA tensor is required")
    if str(v.dtype) != "torch.float64" or v.numel() != nnz or not v.is_contiguous():
        raise ValueError(f"values: a contiguous float64 tensor of {nnz} entries is required")
    if v.device.type != "cuda":
        raise ValueError("values: pass a CUDA tensor or a numpy array")


class Solver:
    """One SGF factorization handle.

    ``Solver(problem_arrays, options)`` runs the symbolic analysis (host
    only).  ``factorize(vals)`` takes the CSR values as a device FP64 tensor.
    """

    def __init__(self, n, indptr, indices, coords, opt):
        self.n = int(n)
        self._indptr = np.ascontiguousarray(indptr, dtype=np.int64)
        self._indices = np.ascontiguousarray(indices, dtype=np.int32)
        self._coords = None if coords is None else np.ascontiguousarray(coords, dtype=np.float64)
        self.opt = opt
        h = ctypes.c_void_p()
        _check(_lib.sgf_analyze(self.n, _ptr(self._indptr), _ptr(self._indices),
                                None if self._coords is None else _ptr(self._coords),
                                ctypes.byref(opt), ctypes.byref(h)))
        self.h = h

    @classmethod
    def from_problem(cls, prob, coords=True, **kw):
        """coords=False analyzes without the node positions (q = 0, or a
        basis given next with set_basis)."""
        opt = make_options(prob.dim, prob.grid, prob.dpn, **kw)
        return cls(prob.n, prob.indptr, prob.indices, prob.coords if coords else None, opt)

    def set_basis(self, basis):
        """Near-kernel basis Pi (n x ncols, numpy) replacing the monomials;
        None returns to the monomials.  Drops the factor."""
        if basis is None:
            _check(_lib.sgf_set_basis(self.h, 0, None))
            return
        b = np.asfortranarray(basis, dtype=np.float64)
        if b.ndim != 2 or b.shape[0] != self.n:
            raise ValueError(f"basis: shape {b.shape}, (n, ncols) with n = {self.n} is required")
        _check(_lib.sgf_set_basis(self.h, int(b.shape[1]), ctypes.c_void_p(b.ctypes.data)))

    def set_low_rank(self, enable=True):
        """Standard low-rank equivalent (Eq. 7.5) at the ranks of the current
        polynomial factorization (enable), or back to the polynomial
        compression.  Drops the factor."""
        _check(_lib.sgf_set_low_rank(self.h, 1 if enable else 0))

    def close(self):
        if self.h:
            _lib.sgf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def factorize(self, vals, stream=None):
        _vals(vals, self._indices.size)
        _check(_lib.sgf_factorize_numeric(self.h, _ptr(vals), _stream(stream)))

    def autotune(self, vals, napply=30, stream=None):
        """Per-level elimination path / panel width by timing; returns the
        chosen mode per level (0 tiled, 8/16/32 panel width, -1 none)."""
        _vals(vals, self._indices.size)
        modes = np.zeros(64, dtype=np.int32)
        _check(_lib.sgf_autotune(self.h, _ptr(vals), int(napply), _ptr(modes), _stream(stream)))
        return modes[:self.info()["levels"]]

    def apply(self, r, z, stream=None):
        nrhs = _pair(r, z, self.n, ("r", "z"))
        _check(_lib.sgf_apply(self.h, nrhs, _ptr(r), self.n, _ptr(z), self.n, _stream(stream)))

    def apply_noalloc(self, r, z, stream=None):
        """sgf_apply_noalloc: the apply with its work vectors in the
        library's static device scratch (no device allocation)."""
        nrhs = _pair(r, z, self.n, ("r", "z"))
        _check(_lib.sgf_apply_noalloc(self.h, nrhs, _ptr(r), self.n, _ptr(z), self.n, _stream(stream)))

    def multiply(self, v, y, stream=None):
        nrhs = _pair(v, y, self.n, ("v", "y"))
        _check(_lib.sgf_multiply(self.h, nrhs, _ptr(v), self.n, _ptr(y), self.n, _stream(stream)))

    def spmv(self, v, y, stream=None):
        if _pair(v, y, self.n, ("v", "y")) != 1:
            raise ValueError("spmv takes one column")
        _check(_lib.sgf_spmv(self.h, _ptr(v), _ptr(y), _stream(stream)))

    def pcg(self, b, x, rtol=1e-8, maxit=500, stream=None, raise_on_noconv=True):
        nrhs = _pair(b, x, self.n, ("b", "x"))
        iters = np.zeros(nrhs, dtype=np.int32)
        rel = np.zeros(nrhs, dtype=np.float64)
        code = _lib.sgf_pcg_solve(self.h, nrhs, _ptr(b), self.n, _ptr(x), self.n, float(rtol), int(maxit),
                                  _ptr(iters), _ptr(rel), _stream(stream))
        if code != SGF_ENOCONV or raise_on_noconv:
            _check(code)
        return iters, rel

    def info(self):
        i = Info()
        _check(_lib.sgf_get_info(self.h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in Info._fields_}

    def perm(self):
        p = np.zeros(self.n, dtype=np.int64)
        _check(_lib.sgf_get_perm(self.h, _ptr(p)))
        return p

    def blocks(self, t):
        """Factor blocks of level t (sgf_export_block): a list of dicts with
        kind, cell, L and, for eliminations, W; for compressions V, tau, r."""
        ne, nc = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.sgf_block_count(self.h, int(t), ctypes.byref(ne), ctypes.byref(nc)))
        out = []
        for i in range(ne.value + nc.value):
            b = Block()
            _check(_lib.sgf_export_block(self.h, int(t), i, ctypes.byref(b), None, None, None, None, None))
            L = np.zeros((b.m, b.m), order="F")
            d = {"kind": b.kind, "cell": b.cell, "L": L}
            W = V = tau = rd = None
            if b.kind == BLOCK_ELIM:
                W = np.zeros((b.m, b.k), order="F")
                d["W"] = W
            elif b.kind == BLOCK_COMP:
                V = np.zeros((b.m, b.r), order="F")
                tau = np.zeros(b.r)
                rd = np.zeros(b.r)
                d.update(V=V, tau=tau, r=b.r, rdiag=rd)
            p = lambda a: None if a is None or a.size == 0 else ctypes.c_void_p(a.ctypes.data)
            _check(_lib.sgf_export_block(self.h, int(t), i, ctypes.byref(b), p(L), p(W), p(V), p(tau), p(rd)))
            out.append(d)
        return out

    def plan_dry_run(self, rank_of):
        """Host-only planning of every level with ranks from ``rank_of(level, cell, size)``."""
        cb = RANK_FN(lambda t, cell, size, ctx: int(rank_of(t, cell, size)))
        _check(_lib.sgf_plan_dry_run(self.h, cb, None))

    def set_persistent(self, max_workgroups=0):
        """Per-level work lists persistent on at most max_workgroups (0: one workgroup per item)."""
        _check(_lib.sgf_set_persistent(self.h, int(max_workgroups)))

    def set_band_elim(self, enable=True):
        """Banded one-wavefront elimination on levels with narrow M_II blocks (default on)."""
        _check(_lib.sgf_set_band_elim(self.h, int(bool(enable))))

    def set_small_compress(self, enable=True):
        """Compression of small separators in LDS (default on: four
        wavefronts per separator on levels of few separators, one otherwise);
        "one": one wavefront per separator on every level (same bits)."""
        mode = 2 if enable == "one" else int(bool(enable))
        _check(_lib.sgf_set_small_compress(self.h, mode))

    def set_pair_kernel(self, mode=-1):
        """Coarse couplings: -1 automatic, 0 one workgroup per pair, 1 one wavefront per pair."""
        _check(_lib.sgf_set_pair_kernel(self.h, int(mode)))

    def set_device_coarsen(self, enable=True):
        """Coarsening destinations computed on the device (default) or host copy lists."""
        _check(_lib.sgf_set_device_coarsen(self.h, 1 if enable else 0))

    def set_band_apply(self, enable=True):
        """Banded interior sweeps on levels with narrow M_II blocks: True / 1
        (default; one wavefront per front for one right-hand side on levels of
        the banded elimination), 2 (one workgroup per front always), False / 0
        (the blocked sweeps)."""
        mode = int(enable) if not isinstance(enable, bool) else int(enable)
        _check(_lib.sgf_set_band_apply(self.h, mode))

    def set_small_apply(self, enable=True):
        """One right-hand side on levels of fronts with at most 64 rows: one
        workgroup per front, all loads issued first (default), or the blocked
        sweeps."""
        _check(_lib.sgf_set_small_apply(self.h, 1 if enable else 0))

    def release(self):
        """Free all device memory of the handle (the analysis stays)."""
        _check(_lib.sgf_release(self.h))

    def estimate_bytes(self, nrhs=1):
        b = ctypes.c_int64()
        _check(_lib.sgf_estimate_bytes(self.h, int(nrhs), ctypes.byref(b)))
        return b.value

    def set_apply_graph(self, enable=True):
        """Replay the apply sweep as a captured HIP graph (default) or launch directly."""
        _check(_lib.sgf_set_apply_graph(self.h, 1 if enable else 0))

    def profile(self, enable=True):
        """Start (clear) or stop per-kernel event timing."""
        _check(_lib.sgf_profile_enable(self.h, 1 if enable else 0))

    def profile_select(self, kernel_class=None):
        """Time only the launches of one kernel class (None: every launch)."""
        _check(_lib.sgf_profile_select(self.h, kernel_class.encode() if kernel_class else None))

    def profile_read(self):
        """{kernel class: dict(launches, ms, flops, bytes)} since profile()."""
        cap = 1024
        arr = (KernelStat * cap)()
        cnt = ctypes.c_int32()
        _check(_lib.sgf_profile_read(self.h, arr, cap, ctypes.byref(cnt)))
        return {arr[i].name.decode(): dict(launches=arr[i].launches, ms=arr[i].ms, flops=arr[i].flops,
                                           bytes=arr[i].bytes) for i in range(min(cnt.value, cap))}

    def level(self, t):
        cnt = ctypes.c_int32()
        _check(_lib.sgf_get_level(self.h, t, ctypes.byref(cnt), None, None, None, None))
        c = cnt.value
        out = [np.zeros(c, dtype=np.int32) for _ in range(4)]
        _check(_lib.sgf_get_level(self.h, t, ctypes.byref(cnt), *[_ptr(a) for a in out]))
        return dict(zip(("cell", "type", "size", "rank"), out))


class Server:
    """Serving loop of the library (sgf_server_*): operators registered once,
    factorize / solve requests queued and run by worker streams under an HBM
    budget, solves of one operator coalesced into multi-column PCGs."""

    def __init__(self, hbm_budget=200 << 30, slots=4, max_batch_rhs=16):
        o = ServerOptions()
        _lib.sgf_server_default_options(ctypes.byref(o))
        o.hbm_budget, o.slots, o.max_batch_rhs = int(hbm_budget), int(slots), int(max_batch_rhs)
        h = ctypes.c_void_p()
        _check(_lib.sgf_server_create(ctypes.byref(o), ctypes.byref(h)))
        self.h = h
        self._keep = {}

    def add_operator(self, prob, **kw):
        """Register a problem (its CSR pattern, values and coordinates)."""
        opt = make_options(prob.dim, prob.grid, prob.dpn, **kw)
        ip = np.ascontiguousarray(prob.indptr, dtype=np.int64)
        ix = np.ascontiguousarray(prob.indices, dtype=np.int32)
        va = np.ascontiguousarray(prob.data, dtype=np.float64)
        co = np.ascontiguousarray(prob.coords, dtype=np.float64)
        op = ctypes.c_int32()
        _check(_lib.sgf_server_add_operator(self.h, prob.n, _ptr(ip), _ptr(ix), _ptr(va), _ptr(co), ctypes.byref(opt),
                                            ctypes.byref(op)))
        return op.value

    def submit(self, op, b, x, rtol=1e-8, maxit=1000, refactor=False):
        """b, x: device float64 tensors of shape (nrhs, n) (contiguous rows =
        columns of the n x nrhs problem); kept alive until wait()."""
        nrhs, n = (1, b.shape[0]) if b.dim() == 1 else (b.shape[0], b.shape[1])
        for t_, name in ((b, "b"), (x, "x")):
            if t_.device.type != "cuda" or str(t_.dtype) != "torch.float64" or not t_.is_contiguous() \
                    or tuple(t_.shape) != tuple(b.shape):
                raise ValueError(f"{name}: a contiguous CUDA float64 tensor shaped like b is required")
        t = ctypes.c_int64()
        _check(_lib.sgf_server_submit(self.h, int(op), 1 if refactor else 0, nrhs, _ptr(b), n, _ptr(x), n,
                                      float(rtol), int(maxit), ctypes.byref(t)))
        self._keep[t.value] = (b, x, nrhs)
        return t.value

    def wait(self, ticket):
        b, x, nrhs = self._keep.pop(ticket)
        info = RequestInfo()
        it = np.zeros(nrhs, dtype=np.int32)
        rel = np.zeros(nrhs, dtype=np.float64)
        _check(_lib.sgf_server_wait(self.h, int(ticket), ctypes.byref(info), _ptr(it), _ptr(rel)))
        d = {f: getattr(info, f) for f, _ in RequestInfo._fields_}
        d["iters"], d["relres"] = it, rel
        return d

    def stats(self):
        st = ServerStats()
        _check(_lib.sgf_server_get_stats(self.h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    @staticmethod
    def clock():
        return _lib.sgf_server_clock()

    def close(self):
        if self.h:
            _lib.sgf_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
