"""Thin ctypes binding of the C ABI in include/mlfma.h.

Argument marshalling only: every step of the product runs in the HIP
library.  torch provides device memory and the current stream; it is
imported before the library is loaded so both use one HIP runtime.
"""
import ctypes
import math
import os
import threading
import time

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_mlfma.so")

OP_C, OP_EM = 0, 1
C128, C64 = 0, 1
PART_NEAR, PART_FAR, PART_ALL, PART_LEVEL = 1, 2, 3, 16
PRECOND_NONE, PRECOND_SAI = 0, 1
STAGES = ("permute_in", "near", "radiate", "aggregate", "translate", "disaggregate", "receive", "permute_out")
_OPS = {"C": OP_C, "EM": OP_EM, OP_C: OP_C, OP_EM: OP_EM}
ERRORS = {-1: "MLFMA_ERR_ARG", -2: "MLFMA_ERR_MESH", -3: "MLFMA_ERR_OOM", -4: "MLFMA_ERR_HIP",
          -5: "MLFMA_ERR_STATE", -6: "MLFMA_ERR_TREE", -7: "MLFMA_ERR_UNSUPPORTED"}


class MlfmaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERRORS.get(code, code), msg))
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("wavenumber", ctypes.c_double), ("leaf_size", ctypes.c_double), ("digits", ctypes.c_int),
                ("interp_order", ctypes.c_int), ("leaf_extra_L", ctypes.c_int), ("max_rhs", ctypes.c_int),
                ("device", ctypes.c_int), ("hbm_budget_bytes", ctypes.c_ulonglong), ("trans_kernel", ctypes.c_int),
                ("level_kernel", ctypes.c_int), ("near_precision", ctypes.c_int), ("far_precision", ctypes.c_int)]


class BatchItem(ctypes.Structure):
    _fields_ = [("h", ctypes.c_void_p), ("op", ctypes.c_int), ("dtype", ctypes.c_int), ("nrhs", ctypes.c_longlong),
                ("x", ctypes.c_void_p), ("ldx", ctypes.c_longlong), ("y", ctypes.c_void_p), ("ldy", ctypes.c_longlong)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_int), ("max_batch_rhs", ctypes.c_int), ("device", ctypes.c_int),
                ("hbm_budget_bytes", ctypes.c_ulonglong), ("use_graphs", ctypes.c_int)]


# int solve(void *user, int dtype, long long n, long long nrhs, const void *b, long long ldb,
#           void *xq, long long ldxq, void *hip_stream)
QSOLVE = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_longlong,
                          ctypes.c_void_p, ctypes.c_longlong, ctypes.c_void_p, ctypes.c_longlong, ctypes.c_void_p)

_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is missing: run __graft_entry__.build() first" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, LL = ctypes.c_void_p, ctypes.c_longlong
        L.mlfma_options_default.argtypes = [ctypes.POINTER(Options)]
        L.mlfma_build_tree.argtypes = [P, LL, P, LL, ctypes.POINTER(Options), ctypes.POINTER(P)]
        L.mlfma_precompute_nearfield.argtypes = [P]
        L.mlfma_matvec_LK.argtypes = [P, ctypes.c_int, ctypes.c_int, LL, P, LL, P, LL, P]
        L.mlfma_matvec_part.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, LL, P, LL, P, LL, P]
        L.mlfma_matvec_LK_noalloc.argtypes = [P, ctypes.c_int, ctypes.c_int, LL, P, LL, P, LL, P]
        L.mlfma_release.argtypes = [P]
        L.mlfma_query.argtypes = [P, ctypes.POINTER(LL), ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_ulonglong)]
        L.mlfma_rwg_table.argtypes = [P, P, P]
        L.mlfma_level_info.argtypes = [P, ctypes.c_int, P]
        L.mlfma_last_error.restype = ctypes.c_char_p
        L.mlfma_translation_operator.argtypes = [ctypes.c_double, ctypes.c_int, P, LL, P, P]
        L.mlfma_near_info.argtypes = [P, P]
        L.mlfma_tuning.argtypes = [P, ctypes.c_int, P, P]
        L.mlfma_tuning_steps.argtypes = [P, ctypes.POINTER(ctypes.c_int), P]
        L.mlfma_tuning_level.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
        L.mlfma_graph_create.argtypes = [P, ctypes.c_int, ctypes.c_int, LL, P, LL, P, LL, ctypes.POINTER(P)]
        L.mlfma_graph_launch.argtypes = [P, P]
        L.mlfma_graph_destroy.argtypes = [P]
        L.mlfma_gmres.argtypes = [P, ctypes.c_int, ctypes.c_int, LL, P, LL, P, LL, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double, ctypes.POINTER(ctypes.c_int), P, P]
        L.mlfma_gmres_precond.argtypes = [P, ctypes.c_int, ctypes.c_int, LL, P, LL, P, LL, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int), P, P]
        L.mlfma_sai_build.argtypes = [P, ctypes.c_int, ctypes.c_int]
        L.mlfma_sai_apply.argtypes = [P, ctypes.c_int, ctypes.c_int, LL, P, LL, P, LL, P]
        L.mlfma_sai_info.argtypes = [P, ctypes.c_int, ctypes.POINTER(LL), ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_ulonglong)]
        L.mlfma_matvec_batch.argtypes = [P, ctypes.c_int, P]
        L.mlfma_matvec_batch_fused.argtypes = [P, ctypes.c_int, P]
        L.mlfma_plane_wave_rhs.argtypes = [P, ctypes.c_int, LL, P, P, P, LL, P]
        L.mlfma_far_field.argtypes = [P, ctypes.c_int, LL, P, LL, LL, P, P, P]
        L.mlfma_server_opts_default.argtypes = [ctypes.POINTER(ServerOptions)]
        L.mlfma_server_create.argtypes = [ctypes.POINTER(ServerOptions), ctypes.POINTER(P)]
        L.mlfma_server_submit.argtypes = [P, P, ctypes.c_int, ctypes.c_int, LL, P, LL, P, LL, P, ctypes.POINTER(LL)]
        L.mlfma_server_wait.argtypes = [P, LL, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int)]
        L.mlfma_server_stats.argtypes = [P, P]
        L.mlfma_server_destroy.argtypes = [P]
        L.mlfma_peak_probe.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        L.mlfma_hybrid_create.argtypes = [P, LL, P, P, P, P, P, P, QSOLVE, P, P, P, LL, LL, ctypes.POINTER(P)]
        L.mlfma_hybrid_matvec.argtypes = [P, ctypes.c_int, LL, P, LL, P, LL, P]
        L.mlfma_hybrid_gmres.argtypes = [P, ctypes.c_int, LL, P, LL, P, LL, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int), P, P]
        L.mlfma_hybrid_destroy.argtypes = [P]
        L.mlfma_profile.argtypes = [P, ctypes.c_int]
        L.mlfma_profile_read.argtypes = [P, P, ctypes.POINTER(LL)]
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise MlfmaError(rc, lib().mlfma_last_error().decode())


def default_options():
    o = Options()
    _check(lib().mlfma_options_default(ctypes.byref(o)))
    return o


class Geometry:
    """A closed triangulated surface with its octree, tables and near field
    resident on one GPU (mlfma_build_tree / mlfma_precompute_nearfield)."""

    def __init__(self, verts, tris, k=2 * math.pi, leaf=0.25, digits=3, interp_order=8, leaf_extra_L=2,
                 max_rhs=1, device=None, hbm_budget_bytes=0, trans_kernel="auto", level_kernel="auto",
                 near_precision="fp64", far_precision="fp64"):
        o = default_options()
        o.trans_kernel = {"auto": 0, "tiled": 1, "groups": 2, "matrix": 3, "lds": 4}[trans_kernel]
        o.level_kernel = {"auto": 0, "vector": 1, "matrix": 2, "blocked": 3, "pipelined": 4}[level_kernel]
        # arithmetic of the near and far parts of complex128 products
        o.near_precision = {"fp64": 1, "fp32": 2}[near_precision]
        o.far_precision = {"fp64": 1, "fp32": 2}[far_precision]
        o.wavenumber = k
        o.leaf_size = leaf
        o.digits = digits
        o.interp_order = interp_order
        o.leaf_extra_L = leaf_extra_L
        o.max_rhs = max_rhs
        o.device = torch.cuda.current_device() if device is None else int(device)
        o.hbm_budget_bytes = hbm_budget_bytes
        self.device = o.device
        v = np.ascontiguousarray(verts, dtype=np.float64)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().mlfma_build_tree(v.ctypes.data, len(v), t.ctypes.data, len(t), ctypes.byref(o),
                                          ctypes.byref(h)))
        self._h = h
        n = ctypes.c_longlong()
        lev = ctypes.c_int()
        _check(lib().mlfma_query(self._h, ctypes.byref(n), ctypes.byref(lev), None))
        self.n_rwg = n.value
        self.levels = lev.value

    def precompute(self):
        with torch.cuda.device(self.device):
            _check(lib().mlfma_precompute_nearfield(self._h))
        return self

    @property
    def hbm_bytes(self):
        b = ctypes.c_ulonglong()
        _check(lib().mlfma_query(self._h, None, None, ctypes.byref(b)))
        return b.value

    def rwg_table(self):
        e = np.zeros((self.n_rwg, 2), np.int32)
        pm = np.zeros((self.n_rwg, 2), np.int32)
        _check(lib().mlfma_rwg_table(self._h, e.ctypes.data, pm.ctypes.data))
        return e, pm

    def level_info(self, level):
        info = np.zeros(6, np.int64)
        _check(lib().mlfma_level_info(self._h, level, info.ctypes.data))
        return {"boxes": int(info[0]), "L": int(info[1]), "K": int(info[2]), "translations": int(info[3]),
                "box_edge": info[4] * 1e-6}

    def plane_wave_rhs(self, khat, pol, dtype=torch.complex128):
        """[b^J; b^M] (eqs. 49-50) for plane waves khat, pol (nrhs x 3) as a
        (2N, nrhs) CUDA tensor."""
        kh = np.ascontiguousarray(np.atleast_2d(khat), np.float64)
        po = np.ascontiguousarray(np.atleast_2d(pol), np.float64)
        nrhs = len(kh)
        bt = torch.empty((nrhs, 2 * self.n_rwg), dtype=dtype, device="cuda:%d" % self.device)
        dt = C128 if dtype == torch.complex128 else C64
        s = torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            _check(lib().mlfma_plane_wave_rhs(self._h, dt, nrhs, kh.ctypes.data, po.ctypes.data, bt.data_ptr(),
                                              2 * self.n_rwg, s.cuda_stream))
        return bt.t()

    def far_field(self, x, dirs):
        """mlfma_far_field: (F . theta_hat, F . phi_hat) of the currents x
        (complex CUDA tensor (2N,) or (2N, nrhs)) in the directions dirs
        (ndir x 3 unit vectors): tensor (ndir, 2, nrhs) of x's dtype.  The radar
        cross section is 4 pi |F|^2."""
        if x.dtype == torch.complex128:
            dt = C128
        elif x.dtype == torch.complex64:
            dt = C64
        else:
            raise TypeError("x must be complex128 or complex64")
        X = x[:, None] if x.dim() == 1 else x
        nrhs = X.shape[1]
        xt = X.t().contiguous()
        d = np.ascontiguousarray(np.atleast_2d(dirs), np.float64)
        F = torch.empty((len(d), 2, nrhs), dtype=x.dtype, device=x.device)
        s = torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            _check(lib().mlfma_far_field(self._h, dt, nrhs, xt.data_ptr(), 2 * self.n_rwg, len(d), d.ctypes.data,
                                         F.data_ptr(), s.cuda_stream))
        return F

    def near_info(self):
        info = np.zeros(4, np.int64)
        _check(lib().mlfma_near_info(self._h, info.ctypes.data))
        return {"slots": int(info[0]), "identity": int(info[1]), "touching_pairs": int(info[2]),
                "leaf_boxes": int(info[3])}

    def tuning(self):
        """Translation kernel and shape picked by the autotuner, per precision:
        {"c64": (targets per tile or group, sources per LDS batch (0 = the
        sibling-group kernel, -1 = it on merged sibling sets), rhs per lane,
        ms, lanes over the rhs (0 for the tiled kernel)), "c128": ...}."""
        out = {}
        for name, dt in (("c64", C64), ("c128", C128)):
            sh = np.zeros(4, np.int32)
            ms = ctypes.c_double(0)
            _check(lib().mlfma_tuning(self._h, dt, sh.ctypes.data, ctypes.byref(ms)))
            out[name] = (int(sh[0]), int(sh[1]), int(sh[2]), float(ms.value), int(sh[3]))
        return out

    def tuning_steps(self):
        """Level-step kernels of complex64 products: {"matrix_cores": bool,
        "ms_vector": t, "ms_matrix": t} (timed at build, 0 if not timed)."""
        m = ctypes.c_int()
        ms = np.zeros(2, np.float64)
        _check(lib().mlfma_tuning_steps(self._h, ctypes.byref(m), ms.ctypes.data))
        return {"matrix_cores": bool(m.value), "ms_vector": float(ms[0]), "ms_matrix": float(ms[1])}

    def tuning_levels(self, dtype=torch.complex64):
        """Vector level-step kernel shapes for four or more right-hand sides
        (mlfma_tuning_level): {level: {"agg_rb", "agg_pipe", "dis_rb",
        "dis_pipe", "agg_group"}} for the steps between level and level + 1."""
        dt = C128 if dtype == torch.complex128 else C64
        out = {}
        for lev in range(2, self.levels - 1):
            s = np.zeros(5, np.int32)
            _check(lib().mlfma_tuning_level(self._h, dt, lev, s.ctypes.data))
            out[lev] = {"agg_rb": int(s[0]), "agg_pipe": int(s[1]), "dis_rb": int(s[2]), "dis_pipe": int(s[3]),
                        "agg_group": int(s[4])}
        return out

    def profile(self, enable=True):
        _check(lib().mlfma_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        ms = np.zeros(8)
        calls = ctypes.c_longlong()
        _check(lib().mlfma_profile_read(self._h, ms.ctypes.data, ctypes.byref(calls)))
        return dict(zip(STAGES, ms.tolist())), calls.value

    def matvec(self, x, op="C", out=None, stream=None, part=PART_ALL):
        """y = A x on the GPU; x: complex128 or complex64 CUDA tensor of shape
        (2N,) or (2N, nrhs).  Returns y with the same shape and dtype.
        part selects the diagnostic split of mlfma_matvec_part (PART_NEAR,
        PART_FAR, PART_LEVEL + l); the default is the whole product."""
        if not (isinstance(x, torch.Tensor) and x.is_cuda):
            raise TypeError("x must be a CUDA tensor")
        if x.dtype == torch.complex128:
            dt = C128
        elif x.dtype == torch.complex64:
            dt = C64
        else:
            raise TypeError("x must be complex128 or complex64")
        squeeze = x.dim() == 1
        X = x[:, None] if squeeze else x
        if X.shape[0] != 2 * self.n_rwg:
            raise ValueError("x must have 2N = %d rows" % (2 * self.n_rwg))
        nrhs = X.shape[1]
        xt = X.t().contiguous()                         # column-major 2N x nrhs storage
        yt = torch.empty_like(xt) if out is None else out
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        with torch.cuda.device(self.device):
            if part == PART_ALL:
                _check(lib().mlfma_matvec_LK(self._h, _OPS.get(op, op), dt, nrhs, xt.data_ptr(), 2 * self.n_rwg,
                                             yt.data_ptr(), 2 * self.n_rwg, s.cuda_stream))
            else:
                _check(lib().mlfma_matvec_part(self._h, _OPS.get(op, op), dt, part, nrhs, xt.data_ptr(), 2 * self.n_rwg,
                                               yt.data_ptr(), 2 * self.n_rwg, s.cuda_stream))
        y = yt.t()
        return y[:, 0] if squeeze else y

    def matvec_raw(self, op, dtype, nrhs, x_ptr, ldx, y_ptr, ldy, stream_ptr):
        """Direct call of mlfma_matvec_LK on device pointers (column-major)."""
        _check(lib().mlfma_matvec_LK(self._h, _OPS.get(op, op), dtype, nrhs, x_ptr, ldx, y_ptr, ldy, stream_ptr))

    def matvec_noalloc_raw(self, op, dtype, nrhs, x_ptr, ldx, y_ptr, ldy, stream_ptr):
        """Direct call of mlfma_matvec_LK_noalloc (no allocation; the
        library's static scratch array) on device pointers (column-major)."""
        _check(lib().mlfma_matvec_LK_noalloc(self._h, _OPS.get(op, op), dtype, nrhs, x_ptr, ldx, y_ptr, ldy,
                                             stream_ptr))

    def sai_build(self, op="C", k_nearest=16):
        """mlfma_sai_build: SAI preconditioner of op's near field over
        patterns of the k_nearest nearest RWGs."""
        with torch.cuda.device(self.device):
            _check(lib().mlfma_sai_build(self._h, _OPS.get(op, op), k_nearest))
        return self

    def sai_apply(self, x, op="C", stream=None):
        """y = M x (mlfma_sai_apply); x: complex CUDA tensor (2N,) or (2N, nrhs)."""
        if x.dtype == torch.complex128:
            dt = C128
        elif x.dtype == torch.complex64:
            dt = C64
        else:
            raise TypeError("x must be complex128 or complex64")
        squeeze = x.dim() == 1
        X = x[:, None] if squeeze else x
        xt = X.t().contiguous()
        yt = torch.empty_like(xt)
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        with torch.cuda.device(self.device):
            _check(lib().mlfma_sai_apply(self._h, _OPS.get(op, op), dt, xt.shape[0], xt.data_ptr(), 2 * self.n_rwg,
                                         yt.data_ptr(), 2 * self.n_rwg, s.cuda_stream))
        y = yt.t()
        return y[:, 0] if squeeze else y

    def sai_info(self, op="C"):
        nnz, mp, ms, by = ctypes.c_longlong(), ctypes.c_int(), ctypes.c_double(), ctypes.c_ulonglong()
        _check(lib().mlfma_sai_info(self._h, _OPS.get(op, op), ctypes.byref(nnz), ctypes.byref(mp), ctypes.byref(ms),
                                    ctypes.byref(by)))
        return {"nnz": nnz.value, "max_pattern": mp.value, "build_ms": ms.value, "bytes": by.value}

    def gmres(self, b, op="C", x0=None, restart=30, max_iters=300, tol=1e-3, stream=None, precond=None):
        """Solve A x = b (mlfma_gmres_precond).  b: complex CUDA tensor (2N,)
        or (2N, nrhs); precond None or "sai" (right preconditioning with the
        SAI of op, built by sai_build).  Returns (x, Arnoldi steps, true
        relative residual per column)."""
        if b.dtype == torch.complex128:
            dt = C128
        elif b.dtype == torch.complex64:
            dt = C64
        else:
            raise TypeError("b must be complex128 or complex64")
        squeeze = b.dim() == 1
        B = b[:, None] if squeeze else b
        nrhs = B.shape[1]
        bt = B.t().contiguous()
        xt = torch.zeros_like(bt) if x0 is None else (x0[:, None] if squeeze else x0).t().contiguous()
        rel = np.zeros(nrhs)
        its = ctypes.c_int()
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        with torch.cuda.device(self.device):
            pc = {None: PRECOND_NONE, "sai": PRECOND_SAI}[precond]
            _check(lib().mlfma_gmres_precond(self._h, _OPS.get(op, op), dt, nrhs, bt.data_ptr(), 2 * self.n_rwg,
                                             xt.data_ptr(), 2 * self.n_rwg, restart, max_iters, tol, pc,
                                             ctypes.byref(its), rel.ctypes.data, s.cuda_stream))
        x = xt.t()
        return (x[:, 0] if squeeze else x), its.value, rel

    def capture(self, op, dtype, nrhs, x_ptr, ldx, y_ptr, ldy):
        """mlfma_graph_create: the whole product on fixed device pointers
        (column-major) as a replayable HIP graph."""
        return Graph(self, op, dtype, nrhs, x_ptr, ldx, y_ptr, ldy)

    def release(self):
        if getattr(self, "_h", None):
            lib().mlfma_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Graph:
    """A captured product (mlfma_graph_*); keeps its geometry alive."""

    def __init__(self, geom, op, dtype, nrhs, x_ptr, ldx, y_ptr, ldy):
        self.geom = geom
        g = ctypes.c_void_p()
        _check(lib().mlfma_graph_create(geom._h, _OPS.get(op, op), dtype, nrhs, x_ptr, ldx, y_ptr, ldy,
                                        ctypes.byref(g)))
        self._g = g

    def launch(self, stream_ptr):
        _check(lib().mlfma_graph_launch(self._g, stream_ptr))

    def close(self):
        if getattr(self, "_g", None):
            lib().mlfma_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server (mlfma_server_*): submit products for
    resident geometries from any thread, wait for tickets."""

    def __init__(self, streams=4, max_batch_rhs=16, hbm_budget_bytes=0, device=None, use_graphs=True):
        o = ServerOptions()
        _check(lib().mlfma_server_opts_default(ctypes.byref(o)))
        o.streams = streams
        o.max_batch_rhs = max_batch_rhs
        o.hbm_budget_bytes = hbm_budget_bytes
        o.use_graphs = 1 if use_graphs else 0
        o.device = torch.cuda.current_device() if device is None else int(device)
        self.device = o.device
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().mlfma_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._s = h
        self._keep = {}
        # wait() calls inside the library; close() lets them leave before it
        # destroys the server (a waiter returns within one wait slice)
        self._cv = threading.Condition()
        self._active = 0
        self._closing = False

    def submit(self, geom, x, y, op="C"):
        """Enqueue y = A x; x, y: column-major storage given as (nrhs, 2N)
        contiguous CUDA tensors (row r = right-hand side r).  Returns a ticket.
        The tensors are kept alive until the ticket is waited for.  The server
        uses x and y only after the work queued so far on torch's current
        stream, so an x computed there just before is read as computed."""
        dt = C128 if x.dtype == torch.complex128 else C64
        nrhs, n2 = x.shape
        t = ctypes.c_longlong()
        with torch.cuda.device(self.device):
            st = torch.cuda.current_stream().cuda_stream
        _check(lib().mlfma_server_submit(self._s, geom._h, _OPS.get(op, op), dt, nrhs, x.data_ptr(), n2,
                                         y.data_ptr(), n2, st, ctypes.byref(t)))
        self._keep[t.value] = (x, y)
        return t.value

    def wait(self, ticket, timeout=-1.0, _slice=0.05):
        """Block until the ticket is done; returns (latency_s, batch_rhs).
        Raises MlfmaError (MLFMA_ERR_STATE) on timeout or when the server is
        closed meanwhile."""
        lat = ctypes.c_double()
        br = ctypes.c_int()
        with self._cv:
            if self._closing or not self._s:
                raise MlfmaError(-5, "the server is closed")
            self._active += 1
        done = False
        try:
            t_end = None if timeout < 0 else time.monotonic() + timeout
            while True:
                left = _slice if t_end is None else min(_slice, max(0.0, t_end - time.monotonic()))
                rc = lib().mlfma_server_wait(self._s, ticket, left, ctypes.byref(lat), ctypes.byref(br))
                if rc == 0:
                    done = True
                    break
                msg = lib().mlfma_last_error().decode()
                if rc != -5 or "within the timeout" not in msg:
                    done = True
                    raise MlfmaError(rc, msg)
                if self._closing:
                    raise MlfmaError(-5, "the server was closed before the request finished")
                if t_end is not None and time.monotonic() >= t_end:
                    raise MlfmaError(-5, msg)
        finally:
            if done:
                self._keep.pop(ticket, None)
            with self._cv:
                self._active -= 1
                self._cv.notify_all()
        return lat.value, br.value

    def stats(self):
        out = np.zeros(5, np.int64)
        _check(lib().mlfma_server_stats(self._s, out.ctypes.data))
        return {"launches": int(out[0]), "requests": int(out[1]), "arena_bytes": int(out[2]), "queued": int(out[3]),
                "graph_captures": int(out[4])}

    def close(self):
        """Destroy the server: requests still queued or running fail, waiting
        threads return with MLFMA_ERR_STATE first."""
        cv = getattr(self, "_cv", None)
        if cv is None or not getattr(self, "_s", None):
            return
        with cv:
            if self._closing:
                return
            self._closing = True
            cv.wait_for(lambda: self._active == 0)
        lib().mlfma_server_destroy(self._s)
        self._s = None
        self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _csr(m, shape):
    """(ptr int64, col int32, val complex128 interleaved) host arrays of a
    scipy.sparse matrix or a (ptr, col, val) triple."""
    if hasattr(m, "tocsr"):
        m = m.tocsr()
        if m.shape != shape:
            raise ValueError("sparse matrix has shape %s, expected %s" % (m.shape, shape))
        ptr, col, val = m.indptr, m.indices, m.data
    else:
        ptr, col, val = m
    ptr = np.ascontiguousarray(ptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    val = np.ascontiguousarray(val, np.complex128)
    if len(ptr) != shape[0] + 1:
        raise ValueError("row pointer array must have %d entries" % (shape[0] + 1))
    return ptr, col, val


class Hybrid:
    """Reduced operator of the hybrid solver (eq. 52; mlfma_hybrid_*):
    y = (C - D_xl Q^-1 D_lx) x with the sparse couplings D_lx (n_hdg x 2N)
    and D_xl (2N x n_hdg) and the caller's solve with Q.

    solve(b, xq) is called with two (nrhs, n_hdg) CUDA tensor views of the
    operator's own buffers (complex128 or complex64 like the product) and
    must write xq = Q^-1 b on torch's current stream."""

    def __init__(self, geom, n_hdg, D_lx, D_xl, solve, max_rhs=1):
        self.geom = geom
        self.n_hdg = int(n_hdg)
        self.max_rhs = int(max_rhs)
        n2 = 2 * geom.n_rwg
        self._arrays = _csr(D_lx, (self.n_hdg, n2)) + _csr(D_xl, (n2, self.n_hdg))
        self._buf1 = torch.zeros((self.max_rhs, self.n_hdg), dtype=torch.complex128, device="cuda:%d" % geom.device)
        self._buf2 = torch.zeros_like(self._buf1)
        self._solve = solve

        def _cb(user, dtype, n, nrhs, b, ldb, xq, ldxq, stream):
            try:
                views = []
                for buf, ptr in ((self._buf1, b), (self._buf2, xq)):
                    if ptr != buf.data_ptr():
                        return 2
                    flat = buf.view(-1)
                    if dtype == C64:
                        flat = flat.view(torch.float64).view(torch.complex64)
                    views.append(flat[:nrhs * self.n_hdg].view(nrhs, self.n_hdg))
                self._solve(views[0], views[1])
                return 0
            except Exception:          # reported as a failed product
                import traceback
                traceback.print_exc()
                return 1

        self._cb = QSOLVE(_cb)
        lx, xl = self._arrays[:3], self._arrays[3:]
        h = ctypes.c_void_p()
        with torch.cuda.device(geom.device):
            _check(lib().mlfma_hybrid_create(geom._h, self.n_hdg, lx[0].ctypes.data, lx[1].ctypes.data,
                                             lx[2].ctypes.data, xl[0].ctypes.data, xl[1].ctypes.data,
                                             xl[2].ctypes.data, self._cb, None, self._buf1.data_ptr(),
                                             self._buf2.data_ptr(), self.n_hdg, self.max_rhs, ctypes.byref(h)))
        self._h = h

    def matvec(self, x):
        """y = (C - D_xl Q^-1 D_lx) x; x complex CUDA tensor (2N,) or (2N, nrhs)."""
        dt = C128 if x.dtype == torch.complex128 else C64
        squeeze = x.dim() == 1
        X = x[:, None] if squeeze else x
        nrhs = X.shape[1]
        xt = X.t().contiguous()
        yt = torch.empty_like(xt)
        n2 = 2 * self.geom.n_rwg
        with torch.cuda.device(self.geom.device):
            st = torch.cuda.current_stream().cuda_stream
            _check(lib().mlfma_hybrid_matvec(self._h, dt, nrhs, xt.data_ptr(), n2, yt.data_ptr(), n2, st))
        y = yt.t()
        return y[:, 0] if squeeze else y

    def gmres(self, b, x0=None, restart=30, max_iters=500, tol=1e-3, precond=None):
        """GMRES on the reduced system (mlfma_hybrid_gmres); returns (x, steps,
        true relative residual per column)."""
        dt = C128 if b.dtype == torch.complex128 else C64
        squeeze = b.dim() == 1
        B = b[:, None] if squeeze else b
        nrhs = B.shape[1]
        bt = B.t().contiguous()
        xt = torch.zeros_like(bt) if x0 is None else (x0[:, None] if squeeze else x0).t().contiguous().clone()
        it = ctypes.c_int()
        rel = np.zeros(nrhs, np.float64)
        n2 = 2 * self.geom.n_rwg
        pc = PRECOND_SAI if precond == "sai" else PRECOND_NONE
        with torch.cuda.device(self.geom.device):
            st = torch.cuda.current_stream().cuda_stream
            _check(lib().mlfma_hybrid_gmres(self._h, dt, nrhs, bt.data_ptr(), n2, xt.data_ptr(), n2, restart,
                                            max_iters, tol, pc, ctypes.byref(it), rel.ctypes.data, st))
        x = xt.t()
        return (x[:, 0] if squeeze else x), it.value, rel

    def close(self):
        if getattr(self, "_h", None):
            lib().mlfma_hybrid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def peak_probe(kind, device=None):
    """mlfma_peak_probe: measured HBM copy bandwidth (kind "hbm", GB/s), FP32
    matrix-core rate ("mfma_f32", TFLOP/s) or FP32 vector FMA rate
    ("valu_f32", TFLOP/s) of the device."""
    code = {"hbm": 0, "mfma_f32": 1, "valu_f32": 2}[kind]
    v = ctypes.c_double()
    dev = torch.cuda.current_device() if device is None else int(device)
    rc = lib().mlfma_peak_probe(code, dev, ctypes.byref(v))
    if rc != 0:
        raise MlfmaError(rc, "peak probe %s failed" % kind)
    return v.value


def matvec_batch(items, stream=None, fused=False):
    """mlfma_matvec_batch: items = [(geometry, x, op), ...] with x complex CUDA
    tensors (2N,) or (2N, nrhs); returns the products in the same order.
    Products of different geometries run concurrently.  fused: the lockstep
    form with shared translation launches (mlfma_matvec_batch_fused;
    distinct geometries, one dtype and one right-hand-side count)."""
    arr = (BatchItem * len(items))()
    keep, outs = [], []
    for i, (g, x, op) in enumerate(items):
        if x.dtype == torch.complex128:
            dt = C128
        elif x.dtype == torch.complex64:
            dt = C64
        else:
            raise TypeError("x must be complex128 or complex64")
        squeeze = x.dim() == 1
        X = x[:, None] if squeeze else x
        xt = X.t().contiguous()
        yt = torch.empty_like(xt)
        keep.append(xt)
        outs.append((yt, squeeze))
        arr[i] = BatchItem(g._h, _OPS.get(op, op), dt, X.shape[1], xt.data_ptr(), 2 * g.n_rwg, yt.data_ptr(),
                           2 * g.n_rwg)
    dev = items[0][0].device if items else 0
    s = torch.cuda.current_stream(dev) if stream is None else stream
    with torch.cuda.device(dev):
        fn = lib().mlfma_matvec_batch_fused if fused else lib().mlfma_matvec_batch
        _check(fn(ctypes.cast(arr, ctypes.c_void_p), len(items), s.cuda_stream))
    res = []
    for yt, squeeze in outs:
        y = yt.t()
        res.append(y[:, 0] if squeeze else y)
    return res


def translation_operator(k, L, X, khat):
    """T_L(khat, X) (host utility of the library)."""
    X = np.ascontiguousarray(X, np.float64)
    kh = np.ascontiguousarray(khat, np.float64)
    out = np.zeros(2 * len(kh))
    _check(lib().mlfma_translation_operator(k, L, X.ctypes.data, len(kh), kh.ctypes.data, out.ctypes.data))
    return out[0::2] + 1j * out[1::2]
