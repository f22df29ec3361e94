"""ctypes binding of libnat_bem.so (declared in include/nat_bem.h and
include/nat_serve.h).

Argument marshalling only: every function forwards torch tensors' device
pointers and the current HIP stream to the C entry point of the same name
and turns non-OK statuses into exceptions.  All computation happens in the
HIP kernels of the library; there is no fallback path, and loading fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import weakref
from pathlib import Path
from typing import Optional, Sequence

import numpy as np

LIB_PATH = Path(__file__).resolve().parent / "libnat_bem.so"

(NAT_OK, NAT_E_INVALID, NAT_E_BUDGET, NAT_E_NOCONV, NAT_E_HIP, NAT_E_INTERNAL, NAT_E_PENDING,
 NAT_E_CANCELLED) = range(8)
NAT_REQ_MCBEM, NAT_REQ_DENSE = 0, 1
NAT_PREC_FP64, NAT_PREC_FP32 = 0, 1
NAT_NEUMANN_PER_VERTEX, NAT_NEUMANN_PER_TRIANGLE = 0, 1


class NatError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_str(status)}: {message}")
        self.status = status


NAT_MC_NO_GRAPH = 1
NAT_MC_ASSEMBLED = 2
NAT_MC_MATRIX_FREE = 4
NAT_MC_EXACT_DISK = 8
NAT_MC_ORDERED_SUM = 16
NAT_MC_FP64_PHASE = 32
NAT_MC_POISSON = 64
NAT_JUMP_HALF = 0
NAT_JUMP_POLYHEDRAL = 1
NAT_FIELD_SHELL = 0
NAT_FIELD_FFAT_GRID = 1
NAT_TUNE_FORCE = 1
TUNE_BUCKETS = 10


class nat_mc_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("layout", C.c_int32), ("eps_scale", C.c_double),
                ("gmres_tol", C.c_double), ("gmres_max_iter", C.c_int32), ("flags", C.c_int32),
                ("jump", C.c_int32), ("n_streams", C.c_int32)]


class nat_mc_job(C.Structure):
    _fields_ = [("mesh", C.c_void_p), ("v_n", C.c_void_p), ("n_modes", C.c_int32),
                ("n_queries", C.c_int32), ("k", C.c_void_p), ("q_tri", C.c_void_p),
                ("q_bary", C.c_void_p), ("n_samples", C.c_int32), ("reserved", C.c_int32),
                ("seed", C.c_uint64), ("p_out", C.c_void_p), ("p_samples", C.c_void_p)]


class nat_field_job(C.Structure):
    _fields_ = [("mesh", C.c_void_p), ("v_n", C.c_void_p), ("n_modes", C.c_int32),
                ("n_points", C.c_int32), ("k", C.c_void_p), ("p_samples", C.c_void_p),
                ("n_samples", C.c_int32), ("reserved", C.c_int32), ("seed", C.c_uint64),
                ("points", C.c_void_p), ("p_out", C.c_void_p), ("abs_out", C.c_void_p)]


class nat_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("flops", C.c_double)]


class nat_solve_report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("rel_resid", C.c_double),
                ("eps", C.c_double), ("area", C.c_double), ("t_sample_ms", C.c_double),
                ("t_rhs_ms", C.c_double), ("t_solve_ms", C.c_double), ("t_eval_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class nat_server_opts(C.Structure):
    _fields_ = [("n_slots", C.c_int32), ("max_batch", C.c_int32), ("hbm_budget", C.c_size_t),
                ("mc", nat_mc_opts), ("dense_tol", C.c_double), ("dense_max_iter", C.c_int32),
                ("dense_burton_miller", C.c_int32)]


class nat_request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("layout", C.c_int32), ("mesh", C.c_void_p),
                ("n_modes", C.c_int32), ("n_queries", C.c_int32), ("k", C.c_void_p),
                ("v_n", C.c_void_p), ("q_tri", C.c_void_p), ("q_bary", C.c_void_p),
                ("n_samples", C.c_int32), ("reserved", C.c_int32), ("seed", C.c_uint64),
                ("p_out", C.c_void_p), ("report", C.c_void_p)]


class nat_request_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("batch_size", C.c_int32), ("slot", C.c_int32),
                ("max_iters", C.c_int32), ("batch_id", C.c_int64), ("queue_ms", C.c_double),
                ("run_ms", C.c_double), ("latency_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class nat_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("cancelled", C.c_int64),
                ("batches", C.c_int64), ("max_batch_seen", C.c_int64), ("max_concurrent", C.c_int32),
                ("reserved", C.c_int32), ("peak_bytes", C.c_size_t), ("budget", C.c_size_t)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


_P = C.c_void_p
_SIGS = {
    "nat_ctx_create": ([C.c_int32, C.c_size_t, C.POINTER(_P)], C.c_int),
    "nat_ctx_destroy": ([_P], None),
    "nat_ctx_bytes_in_use": ([_P], C.c_size_t),
    "nat_mesh_create": ([_P, _P, C.c_int32, _P, C.c_int32, C.POINTER(_P)], C.c_int),
    "nat_mesh_destroy": ([_P], None),
    "nat_mesh_validate": ([_P, C.c_int32, _P, C.c_int32], C.c_int),
    "nat_mesh_geometry": ([_P, C.c_int32, _P, C.c_int32, _P, _P, _P], C.c_int),
    "nat_mesh_free_terms": ([_P, C.c_int32, _P, C.c_int32, _P, _P], C.c_int),
    "nat_mesh_info": ([_P, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "nat_mesh_vertex_queries": ([_P, _P, _P], C.c_int),
    "nat_mc_opts_default": ([C.POINTER(nat_mc_opts)], None),
    "nat_mcbem_samples": ([_P, C.c_int32, C.c_uint64, _P, _P, _P], C.c_int),
    "nat_mcbem_poisson_samples": ([_P, C.c_int32, C.c_uint64, _P, _P, C.POINTER(C.c_int32), _P], C.c_int),
    "nat_mcbem_estimate": ([_P, _P, C.c_int32, _P, _P, _P, C.c_int32, C.c_int32, C.c_uint64,
                            C.POINTER(nat_mc_opts), _P, _P, _P, _P], C.c_int),
    "nat_mcbem_estimate_noalloc": ([_P, _P, C.c_int32, _P, _P, _P, C.c_int32, C.c_int32, C.c_uint64,
                                    C.POINTER(nat_mc_opts), _P, _P, _P, _P], C.c_int),
    "nat_mcbem_estimate_batch": ([_P, _P, C.c_int32, C.POINTER(nat_mc_opts), _P, _P], C.c_int),
    "nat_mcbem_field": ([_P, _P, C.c_int32, _P, _P, C.c_int32, C.c_uint64, _P, C.c_int32,
                         C.POINTER(nat_mc_opts), _P, _P, _P], C.c_int),
    "nat_mcbem_field_batch": ([_P, _P, C.c_int32, C.POINTER(nat_mc_opts), _P], C.c_int),
    "nat_field_points": ([_P, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_uint64,
                          _P, _P, _P], C.c_int),
    "nat_bem_assemble": ([_P, C.c_double, C.c_int32, C.POINTER(_P), _P], C.c_int),
    "nat_bem_solve": ([_P, _P, C.c_int32, C.c_int32, C.c_double, C.c_int32, _P, _P, _P], C.c_int),
    "nat_bem_op_matrices": ([_P, _P, _P, _P], C.c_int),
    "nat_bem_op_destroy": ([_P], None),
    "nat_profile_enable": ([_P, C.c_int32], C.c_int),
    "nat_profile_read": ([_P, _P, C.c_int32], C.c_int32),
    "nat_autotune": ([_P, C.c_char_p, C.c_int32, _P], C.c_int),
    "nat_tune_get": ([_P, _P, _P, C.POINTER(C.c_int32)], C.c_int),
    "nat_tune_set": ([_P, _P, _P], C.c_int),
    "nat_tune_get_form": ([_P, _P, _P, _P], C.c_int),
    "nat_tune_set_form": ([_P, _P], C.c_int),
    "nat_server_opts_default": ([C.POINTER(nat_server_opts)], None),
    "nat_server_create": ([_P, C.POINTER(nat_server_opts), C.POINTER(_P)], C.c_int),
    "nat_server_submit": ([_P, C.POINTER(nat_request), C.POINTER(C.c_uint64)], C.c_int),
    "nat_server_wait": ([_P, C.c_uint64, C.c_double, C.POINTER(nat_request_result)], C.c_int),
    "nat_server_cancel": ([_P, C.c_uint64], C.c_int),
    "nat_server_stats_read": ([_P, C.POINTER(nat_server_stats)], C.c_int),
    "nat_server_destroy": ([_P], None),
    "nat_status_str": ([C.c_int], C.c_char_p),
    "nat_last_error": ([C.c_char_p, C.c_size_t], C.c_size_t),
    "nat_nf_create": ([_P, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_uint64, C.POINTER(_P)], C.c_int),
    "nat_nf_destroy": ([_P], None),
    "nat_nf_info": ([_P, C.POINTER(C.c_int32), C.POINTER(C.c_int64)], C.c_int),
    "nat_nf_set_params": ([_P, _P, C.c_int64], C.c_int),
    "nat_nf_get_params": ([_P, _P, C.c_int64], C.c_int),
    "nat_nf_get_grads": ([_P, _P, C.c_int64], C.c_int),
    "nat_nf_loss_grad": ([_P, _P, _P, C.c_int32, C.POINTER(C.c_double), _P], C.c_int),
    "nat_nf_train_step": ([_P, _P, _P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double), _P], C.c_int),
    "nat_nf_infer": ([_P, _P, C.c_int32, _P, _P], C.c_int),
}

_lib = None


def lib():
    """Load libnat_bem.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2506_06190_amd/build.py "
                              "(there is no CPU fallback)")
        L = C.CDLL(str(LIB_PATH))
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def status_str(s: int) -> str:
    return lib().nat_status_str(s).decode()


def last_error() -> str:
    buf = C.create_string_buffer(1024)
    lib().nat_last_error(buf, len(buf))
    return buf.value.decode()


def _check(st: int, allow=()):
    if st != NAT_OK and st not in allow:
        raise NatError(st, last_error())
    return st


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dptr(t, dtype=None, shape=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


# ------------------------------------------------------- host-only helpers
def nat_mesh_validate(vertices, tris):
    """Returns (status, message); host only."""
    v = np.ascontiguousarray(vertices, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    st = lib().nat_mesh_validate(v.ctypes.data_as(_P), len(v), t.ctypes.data_as(_P), len(t))
    return st, (last_error() if st != NAT_OK else "")


def nat_mesh_geometry(vertices, tris):
    v = np.ascontiguousarray(vertices, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    area = np.empty(len(t))
    normal = np.empty((len(t), 3))
    cdf = np.empty(len(t))
    _check(lib().nat_mesh_geometry(v.ctypes.data_as(_P), len(v), t.ctypes.data_as(_P), len(t),
                                   area.ctypes.data_as(_P), normal.ctypes.data_as(_P),
                                   cdf.ctypes.data_as(_P)))
    return area, normal, cdf


def nat_mesh_free_terms(vertices, tris):
    """(c_vert [V], c_edge [T, 3]): the free terms used by NAT_JUMP_POLYHEDRAL."""
    v = np.ascontiguousarray(vertices, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    cv = np.empty(len(v))
    ce = np.empty((len(t), 3))
    _check(lib().nat_mesh_free_terms(v.ctypes.data_as(_P), len(v), t.ctypes.data_as(_P), len(t),
                                     cv.ctypes.data_as(_P), ce.ctypes.data_as(_P)))
    return cv, ce


# ---------------------------------------------------------------- handles
class Context:
    """Handle of nat_ctx_create.  Closing it first closes every mesh,
    operator, server and neural field made from it that is still open (the
    C library requires them destroyed before their context)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = C.c_void_p()
        _check(lib().nat_ctx_create(device, hbm_budget_bytes, C.byref(h)))
        self.handle = h
        self.device = device
        self._children = []  # weak references, in creation order

    def _adopt(self, obj):
        self._children.append(weakref.ref(obj))

    def bytes_in_use(self) -> int:
        return int(lib().nat_ctx_bytes_in_use(self.handle))

    def close(self):
        if self.handle:
            live = [c for c in (r() for r in self._children) if c is not None]
            # dependents (servers, operators, fields) before the meshes they use
            for c in sorted(live, key=lambda c: isinstance(c, Mesh)):
                try:
                    c.close()
                except Exception:
                    pass
            self._children.clear()
            lib().nat_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    def __init__(self, ctx: Context, vertices: np.ndarray, tris: np.ndarray):
        v = np.ascontiguousarray(vertices, dtype=np.float64)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        h = C.c_void_p()
        _check(lib().nat_mesh_create(ctx.handle, v.ctypes.data_as(_P), len(v),
                                     t.ctypes.data_as(_P), len(t), C.byref(h)))
        self.ctx = ctx
        self.handle = h
        self.n_vertices = len(v)
        self.n_tris = len(t)
        ctx._adopt(self)

    def info(self):
        a, nv, nt = C.c_double(), C.c_int32(), C.c_int32()
        _check(lib().nat_mesh_info(self.handle, C.byref(a), C.byref(nv), C.byref(nt)))
        return a.value, nv.value, nt.value

    def vertex_queries(self):
        tri = np.empty(self.n_vertices, dtype=np.int32)
        bary = np.empty((self.n_vertices, 2), dtype=np.float64)
        _check(lib().nat_mesh_vertex_queries(self.handle, tri.ctypes.data_as(_P),
                                             bary.ctypes.data_as(_P)))
        return tri, bary

    def close(self):
        if self.handle:
            lib().nat_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BemOp:
    def __init__(self, handle, mesh: Mesh, k: float):
        self.handle = handle
        self.mesh = mesh
        self.k = k
        self.n = mesh.n_tris
        mesh.ctx._adopt(self)

    def close(self):
        if self.handle:
            lib().nat_bem_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ entry points
def nat_profile_enable(ctx: Context, enable: bool = True):
    _check(lib().nat_profile_enable(ctx.handle, int(bool(enable))))


def nat_profile_read(ctx: Context):
    """{kernel name: {launches, total_ms, flops, avg_ms}}"""
    buf = (nat_kernel_stat * 16)()
    n = lib().nat_profile_read(ctx.handle, C.cast(buf, _P), 16)
    out = {}
    for i in range(n):
        b = buf[i]
        out[b.name.decode()] = {"launches": b.launches, "total_ms": b.total_ms, "flops": b.flops,
                                "avg_ms": b.total_ms / max(b.launches, 1)}
    return out


def nat_autotune(ctx: Context, cache_path=None, force: bool = False, stream=None):
    """Fill the context's tiling table (from the cache or by a sweep); returns it."""
    path = None if cache_path is None else str(cache_path).encode()
    _check(lib().nat_autotune(ctx.handle, path, NAT_TUNE_FORCE if force else 0, _stream(stream)))
    return nat_tune_get(ctx)


def nat_tune_get(ctx: Context):
    """{"items_a": [10 ints], "items_b": [10 ints], "tuned": bool}"""
    a = np.zeros(TUNE_BUCKETS, dtype=np.int32)
    b = np.zeros(TUNE_BUCKETS, dtype=np.int32)
    t = C.c_int32()
    _check(lib().nat_tune_get(ctx.handle, a.ctypes.data_as(_P), b.ctypes.data_as(_P), C.byref(t)))
    return {"items_a": a.tolist(), "items_b": b.tolist(), "tuned": bool(t.value)}


def nat_tune_set(ctx: Context, items_a, items_b):
    a = np.ascontiguousarray(items_a, dtype=np.int32)
    b = np.ascontiguousarray(items_b, dtype=np.int32)
    if a.shape != (TUNE_BUCKETS,) or b.shape != (TUNE_BUCKETS,):
        raise ValueError(f"tables must have {TUNE_BUCKETS} entries")
    _check(lib().nat_tune_set(ctx.handle, a.ctypes.data_as(_P), b.ctypes.data_as(_P)))


def nat_tune_get_form(ctx: Context, with_rates: bool = False):
    """Per bucket of N: 1 if the GMRES matvec uses the assembled operator;
    with_rates adds the sweep's measured matvec rates (pair-modes/s)."""
    a = np.zeros(TUNE_BUCKETS, dtype=np.int32)
    rf = np.zeros(TUNE_BUCKETS)
    ra = np.zeros(TUNE_BUCKETS)
    _check(lib().nat_tune_get_form(ctx.handle, a.ctypes.data_as(_P), rf.ctypes.data_as(_P),
                                   ra.ctypes.data_as(_P)))
    if with_rates:
        return {"assembled": a.tolist(), "rate_matrix_free": rf.tolist(), "rate_assembled": ra.tolist()}
    return a.tolist()


def nat_tune_set_form(ctx: Context, assembled):
    a = np.ascontiguousarray(assembled, dtype=np.int32)
    if a.shape != (TUNE_BUCKETS,):
        raise ValueError(f"table must have {TUNE_BUCKETS} entries")
    _check(lib().nat_tune_set_form(ctx.handle, a.ctypes.data_as(_P)))


def nat_mc_opts_default() -> nat_mc_opts:
    o = nat_mc_opts()
    lib().nat_mc_opts_default(C.byref(o))
    return o


def nat_mcbem_samples(mesh: Mesh, n_samples: int, seed: int, tri, bary, stream=None):
    import torch
    _check(lib().nat_mcbem_samples(mesh.handle, n_samples, C.c_uint64(seed),
                                   _dptr(tri, torch.int32, (n_samples,), "tri"),
                                   _dptr(bary, torch.float64, (n_samples, 2), "bary"),
                                   _stream(stream)))


def nat_mcbem_poisson_samples(mesh: Mesh, n_samples: int, seed: int, tri=None, bary=None, stream=None,
                              device="cuda"):
    """Poisson-disk sample records: (tri [N] int32, bary [N, 2] float64, accepted count)."""
    import torch
    if tri is None:
        tri = torch.empty(n_samples, dtype=torch.int32, device=device)
    if bary is None:
        bary = torch.empty((n_samples, 2), dtype=torch.float64, device=device)
    n = C.c_int32(0)
    _check(lib().nat_mcbem_poisson_samples(mesh.handle, int(n_samples), C.c_uint64(seed),
                                           _dptr(tri, torch.int32, (n_samples,), "tri"),
                                           _dptr(bary, torch.float64, (n_samples, 2), "bary"),
                                           C.byref(n), _stream(stream)))
    return tri, bary, int(n.value)


def nat_mcbem_estimate(mesh: Mesh, v_n, k: Sequence[float], q_tri, q_bary, n_samples: int,
                       seed: int, opts: Optional[nat_mc_opts] = None, p_out=None,
                       p_samples=None, stream=None, allow_noconv: bool = False):
    """Returns (p_out [n_modes, Q] complex128, list of per-mode report dicts)."""
    import torch
    if opts is None:
        opts = nat_mc_opts_default()
    k = np.ascontiguousarray(np.atleast_1d(k), dtype=np.float64)
    M = len(k)
    ng = mesh.n_tris if opts.layout == NAT_NEUMANN_PER_TRIANGLE else mesh.n_vertices
    Q = int(q_tri.shape[0])
    dev = v_n.device
    if p_out is None:
        p_out = torch.empty((M, Q), dtype=torch.complex128, device=dev)
    reps = (nat_solve_report * M)()
    st = lib().nat_mcbem_estimate(
        mesh.handle, _dptr(v_n, torch.complex128, (M, ng), "v_n"), M, k.ctypes.data_as(_P),
        _dptr(q_tri, torch.int32, (Q,), "q_tri"), _dptr(q_bary, torch.float64, (Q, 2), "q_bary"),
        Q, n_samples, C.c_uint64(seed), C.byref(opts),
        _dptr(p_out, torch.complex128, (M, Q), "p_out"),
        _dptr(p_samples, torch.complex128, (M, n_samples), "p_samples") if p_samples is not None else None,
        C.cast(reps, _P), _stream(stream))
    _check(st, allow=(NAT_E_NOCONV,) if allow_noconv else ())
    return p_out, [r.as_dict() for r in reps]


def nat_mcbem_estimate_noalloc(mesh: Mesh, v_n, k: Sequence[float], q_tri, q_bary, n_samples: int,
                               seed: int, opts: Optional[nat_mc_opts] = None, p_out=None,
                               p_samples=None, stream=None, allow_noconv: bool = False):
    """nat_mcbem_estimate without allocation inside the call: p_out (and
    p_samples) must be given as device tensors by the caller."""
    import torch
    if opts is None:
        opts = nat_mc_opts_default()
    if p_out is None:
        raise ValueError("nat_mcbem_estimate_noalloc: p_out must be allocated by the caller")
    k = np.ascontiguousarray(np.atleast_1d(k), dtype=np.float64)
    M = len(k)
    ng = mesh.n_tris if opts.layout == NAT_NEUMANN_PER_TRIANGLE else mesh.n_vertices
    Q = int(q_tri.shape[0])
    reps = (nat_solve_report * M)()
    st = lib().nat_mcbem_estimate_noalloc(
        mesh.handle, _dptr(v_n, torch.complex128, (M, ng), "v_n"), M, k.ctypes.data_as(_P),
        _dptr(q_tri, torch.int32, (Q,), "q_tri"), _dptr(q_bary, torch.float64, (Q, 2), "q_bary"),
        Q, n_samples, C.c_uint64(seed), C.byref(opts),
        _dptr(p_out, torch.complex128, (M, Q), "p_out"),
        _dptr(p_samples, torch.complex128, (M, n_samples), "p_samples") if p_samples is not None else None,
        C.cast(reps, _P), _stream(stream))
    _check(st, allow=(NAT_E_NOCONV,) if allow_noconv else ())
    return p_out, [r.as_dict() for r in reps]


def nat_mcbem_field(mesh: Mesh, v_n, k: Sequence[float], p_samples, n_samples: int, seed: int,
                    points, opts: Optional[nat_mc_opts] = None, p_out=None, abs_out=None,
                    want_abs: bool = False, stream=None):
    """Exterior field at points [P, 3] (device float64) from an estimate's
    p_samples [n_modes, n_samples].  Returns (p_out [n_modes, P] complex128,
    abs_out [n_modes, P] float64 or None)."""
    import torch
    if opts is None:
        opts = nat_mc_opts_default()
    k = np.ascontiguousarray(np.atleast_1d(k), dtype=np.float64)
    M = len(k)
    ng = mesh.n_tris if opts.layout == NAT_NEUMANN_PER_TRIANGLE else mesh.n_vertices
    P = int(points.shape[0])
    dev = v_n.device
    if p_out is None:
        p_out = torch.empty((M, P), dtype=torch.complex128, device=dev)
    if abs_out is None and want_abs:
        abs_out = torch.empty((M, P), dtype=torch.float64, device=dev)
    st = lib().nat_mcbem_field(
        mesh.handle, _dptr(v_n, torch.complex128, (M, ng), "v_n"), M, k.ctypes.data_as(_P),
        _dptr(p_samples, torch.complex128, (M, n_samples), "p_samples"), n_samples, C.c_uint64(seed),
        _dptr(points, torch.float64, (P, 3), "points"), P, C.byref(opts),
        _dptr(p_out, torch.complex128, (M, P), "p_out"),
        _dptr(abs_out, torch.float64, (M, P), "abs_out") if abs_out is not None else None,
        _stream(stream))
    _check(st)
    return p_out, abs_out


class FieldJob:
    """One field of nat_mcbem_field_batch (device tensors, host k); the
    Neumann layout is the batch's (nat_mc_opts.layout)."""

    def __init__(self, mesh: Mesh, v_n, k, p_samples, n_samples: int, seed: int, points, p_out=None,
                 abs_out=None, want_abs: bool = False):
        import torch
        self.mesh = mesh
        self.k = np.ascontiguousarray(np.atleast_1d(k), dtype=np.float64)
        self.n_modes = len(self.k)
        self.v_n, self.p_samples, self.points = v_n, p_samples, points
        self.n_samples, self.seed = int(n_samples), int(seed)
        self.P = int(points.shape[0])
        if p_out is None:
            p_out = torch.empty((self.n_modes, self.P), dtype=torch.complex128, device=v_n.device)
        if abs_out is None and want_abs:
            abs_out = torch.empty((self.n_modes, self.P), dtype=torch.float64, device=v_n.device)
        self.p_out, self.abs_out = p_out, abs_out

    def record(self, layout: int) -> nat_field_job:
        import torch
        ng = self.mesh.n_tris if layout == NAT_NEUMANN_PER_TRIANGLE else self.mesh.n_vertices
        j = nat_field_job()
        j.mesh = self.mesh.handle.value
        j.v_n = _dptr(self.v_n, torch.complex128, (self.n_modes, ng), "v_n").value
        j.n_modes = self.n_modes
        j.n_points = self.P
        j.k = self.k.ctypes.data
        j.p_samples = _dptr(self.p_samples, torch.complex128, (self.n_modes, self.n_samples), "p_samples").value
        j.n_samples = self.n_samples
        j.seed = self.seed
        j.points = _dptr(self.points, torch.float64, (self.P, 3), "points").value
        j.p_out = _dptr(self.p_out, torch.complex128, (self.n_modes, self.P), "p_out").value
        j.abs_out = (_dptr(self.abs_out, torch.float64, (self.n_modes, self.P), "abs_out").value
                     if self.abs_out is not None else None)
        return j


def nat_mcbem_field_batch(ctx: Context, jobs, opts: Optional[nat_mc_opts] = None, stream=None):
    """Runs the field jobs (list of FieldJob) in one batch."""
    if opts is None:
        opts = nat_mc_opts_default()
    recs = (nat_field_job * len(jobs))(*[j.record(opts.layout) for j in jobs])
    _check(lib().nat_mcbem_field_batch(ctx.handle, C.cast(recs, _P), len(jobs), C.byref(opts), _stream(stream)))
    return jobs


def nat_field_points(mesh: Mesh, kind: int, n_a: int, n_b: int = 1, r_lo: float = 1.5,
                     r_hi: float = 3.0, seed: int = 0, points=None, coords=None, stream=None,
                     device="cuda"):
    """Shell (NAT_FIELD_SHELL, n_a points) or FFAT grid (NAT_FIELD_FFAT_GRID,
    n_a x n_b) field points: returns (points [n, 3], coords [n, 3] = (r, theta, phi))."""
    import torch
    n = n_a if kind == NAT_FIELD_SHELL else n_a * n_b
    if points is None:
        points = torch.empty((n, 3), dtype=torch.float64, device=device)
    if coords is None:
        coords = torch.empty((n, 3), dtype=torch.float64, device=device)
    _check(lib().nat_field_points(mesh.handle, int(kind), int(n_a), int(n_b), float(r_lo), float(r_hi),
                                  C.c_uint64(seed), _dptr(points, torch.float64, (n, 3), "points"),
                                  _dptr(coords, torch.float64, (n, 3), "coords"), _stream(stream)))
    return points, coords


class McJob:
    """One problem of nat_mcbem_estimate_batch (device tensors, host k).  The
    Neumann layout must be the batch's (nat_mc_opts.layout): the C job record
    carries none, and v_n is read with the batch's layout."""

    def __init__(self, mesh: Mesh, v_n, k, q_tri, q_bary, n_samples: int, seed: int,
                 p_out=None, p_samples=None, layout: int = NAT_NEUMANN_PER_VERTEX):
        import torch
        self.mesh = mesh
        self.k = np.ascontiguousarray(np.atleast_1d(k), dtype=np.float64)
        self.n_modes = len(self.k)
        self.layout = int(layout)
        ng = mesh.n_tris if layout == NAT_NEUMANN_PER_TRIANGLE else mesh.n_vertices
        self.Q = int(q_tri.shape[0])
        self.v_n, self.q_tri, self.q_bary = v_n, q_tri, q_bary
        self.n_samples, self.seed = int(n_samples), int(seed)
        _dptr(v_n, torch.complex128, (self.n_modes, ng), "v_n")
        _dptr(q_tri, torch.int32, (self.Q,), "q_tri")
        _dptr(q_bary, torch.float64, (self.Q, 2), "q_bary")
        if p_out is None:
            p_out = torch.empty((self.n_modes, self.Q), dtype=torch.complex128, device=v_n.device)
        self.p_out = p_out
        self.p_samples = p_samples

    def record(self, layout: int) -> nat_mc_job:
        import torch
        if int(layout) != self.layout:
            raise ValueError(f"job layout {self.layout} differs from the batch layout {layout}")
        ng = self.mesh.n_tris if layout == NAT_NEUMANN_PER_TRIANGLE else self.mesh.n_vertices
        j = nat_mc_job()
        j.mesh = self.mesh.handle.value
        j.v_n = _dptr(self.v_n, torch.complex128, (self.n_modes, ng), "v_n").value
        j.n_modes = self.n_modes
        j.n_queries = self.Q
        j.k = self.k.ctypes.data
        j.q_tri = self.q_tri.data_ptr()
        j.q_bary = self.q_bary.data_ptr()
        j.n_samples = self.n_samples
        j.seed = self.seed
        j.p_out = _dptr(self.p_out, torch.complex128, (self.n_modes, self.Q), "p_out").value
        j.p_samples = (_dptr(self.p_samples, torch.complex128, (self.n_modes, self.n_samples),
                             "p_samples").value if self.p_samples is not None else None)
        return j


def nat_mcbem_estimate_batch(ctx: Context, jobs, opts: Optional[nat_mc_opts] = None, stream=None,
                             allow_noconv: bool = False):
    """Runs the jobs (list of McJob) in one batch; returns per-job lists of report dicts."""
    if opts is None:
        opts = nat_mc_opts_default()
    recs = (nat_mc_job * len(jobs))(*[j.record(opts.layout) for j in jobs])
    n_sys = sum(j.n_modes for j in jobs)
    reps = (nat_solve_report * n_sys)()
    st = lib().nat_mcbem_estimate_batch(ctx.handle, C.cast(recs, _P), len(jobs), C.byref(opts),
                                        C.cast(reps, _P), _stream(stream))
    _check(st, allow=(NAT_E_NOCONV,) if allow_noconv else ())
    out, q = [], 0
    for j in jobs:
        out.append([reps[q + m].as_dict() for m in range(j.n_modes)])
        q += j.n_modes
    return out


def nat_bem_assemble(mesh: Mesh, k: float, burton_miller: bool = True, stream=None) -> BemOp:
    h = C.c_void_p()
    _check(lib().nat_bem_assemble(mesh.handle, float(k), int(bool(burton_miller)), C.byref(h),
                                  _stream(stream)))
    return BemOp(h, mesh, k)


def nat_bem_solve(op: BemOp, v_n, layout: int = NAT_NEUMANN_PER_VERTEX, tol: float = 1e-10,
                  max_iter: int = 500, p_out=None, stream=None, allow_noconv: bool = False):
    import torch
    M = int(v_n.shape[0])
    ng = op.mesh.n_tris if layout == NAT_NEUMANN_PER_TRIANGLE else op.mesh.n_vertices
    if p_out is None:
        p_out = torch.empty((M, op.n), dtype=torch.complex128, device=v_n.device)
    reps = (nat_solve_report * M)()
    st = lib().nat_bem_solve(op.handle, _dptr(v_n, torch.complex128, (M, ng), "v_n"), M, layout,
                             float(tol), int(max_iter), _dptr(p_out, torch.complex128, (M, op.n), "p_out"),
                             C.cast(reps, _P), _stream(stream))
    _check(st, allow=(NAT_E_NOCONV,) if allow_noconv else ())
    return p_out, [r.as_dict() for r in reps]


def nat_bem_op_matrices(op: BemOp, stream=None):
    import torch
    A = torch.empty((op.n, op.n), dtype=torch.complex128, device=f"cuda:{op.mesh.ctx.device}")
    B = torch.empty_like(A)
    _check(lib().nat_bem_op_matrices(op.handle, _dptr(A), _dptr(B), _stream(stream)))
    return A, B


# ------------------------------------------------------------- served form
def nat_server_opts_default() -> nat_server_opts:
    o = nat_server_opts()
    lib().nat_server_opts_default(C.byref(o))
    return o


class Request:
    """One served request: device tensors, host k, and the output tensor.

    kind NAT_REQ_MCBEM: p_out [n_modes, Q] at the query points;
    kind NAT_REQ_DENSE: p_out [n_modes, n_tris] at the centroids."""

    def __init__(self, kind: int, mesh: Mesh, v_n, k, q_tri=None, q_bary=None, n_samples: int = 0,
                 seed: int = 0, layout: int = NAT_NEUMANN_PER_VERTEX, p_out=None):
        import torch
        self.kind, self.mesh, self.layout = int(kind), mesh, int(layout)
        self.k = np.ascontiguousarray(np.atleast_1d(k), dtype=np.float64)
        self.n_modes = len(self.k)
        ng = mesh.n_tris if layout == NAT_NEUMANN_PER_TRIANGLE else mesh.n_vertices
        _dptr(v_n, torch.complex128, (self.n_modes, ng), "v_n")
        self.v_n, self.q_tri, self.q_bary = v_n, q_tri, q_bary
        self.n_samples, self.seed = int(n_samples), int(seed)
        if kind == NAT_REQ_MCBEM:
            self.Q = int(q_tri.shape[0])
            _dptr(q_tri, torch.int32, (self.Q,), "q_tri")
            _dptr(q_bary, torch.float64, (self.Q, 2), "q_bary")
            shape = (self.n_modes, self.Q)
        else:
            self.Q = 0
            shape = (self.n_modes, mesh.n_tris)
        if p_out is None:
            p_out = torch.empty(shape, dtype=torch.complex128, device=v_n.device)
        _dptr(p_out, torch.complex128, shape, "p_out")
        self.p_out = p_out
        self.reports = (nat_solve_report * self.n_modes)()

    def record(self) -> nat_request:
        r = nat_request()
        r.kind, r.layout, r.mesh = self.kind, self.layout, self.mesh.handle.value
        r.n_modes, r.n_queries = self.n_modes, self.Q
        r.k = self.k.ctypes.data
        r.v_n = self.v_n.data_ptr()
        if self.kind == NAT_REQ_MCBEM:
            r.q_tri = self.q_tri.data_ptr()
            r.q_bary = self.q_bary.data_ptr()
        r.n_samples, r.seed = self.n_samples, self.seed
        r.p_out = self.p_out.data_ptr()
        r.report = C.cast(self.reports, _P).value
        return r


class Server:
    """Handle of nat_server_create; keeps each submitted Request alive until
    its result has been collected."""

    def __init__(self, ctx: Context, opts: Optional[nat_server_opts] = None):
        if opts is None:
            opts = nat_server_opts_default()
        h = C.c_void_p()
        _check(lib().nat_server_create(ctx.handle, C.byref(opts), C.byref(h)))
        self.ctx, self.handle, self.opts = ctx, h, opts
        self._live = {}
        ctx._adopt(self)

    def close(self):
        if self.handle:
            lib().nat_server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nat_server_create(ctx: Context, opts: Optional[nat_server_opts] = None) -> Server:
    return Server(ctx, opts)


def nat_server_submit(srv: Server, req: Request) -> int:
    """Queue req (device work is stream-ordered on the server's own streams:
    the caller synchronises its producers first); returns the ticket."""
    t = C.c_uint64()
    rec = req.record()
    _check(lib().nat_server_submit(srv.handle, C.byref(rec), C.byref(t)))
    srv._live[t.value] = req
    return t.value


def nat_server_wait(srv: Server, ticket: int, timeout_ms: float = -1.0):
    """(status, result dict, per-mode report dicts); status NAT_E_PENDING
    (result None) if the request has not ended within timeout_ms."""
    res = nat_request_result()
    st = lib().nat_server_wait(srv.handle, C.c_uint64(ticket), float(timeout_ms), C.byref(res))
    if st == NAT_E_PENDING:
        return st, None, None
    req = srv._live.pop(ticket, None)
    if req is None:
        _check(st)
    reps = [r.as_dict() for r in req.reports] if st in (NAT_OK, NAT_E_NOCONV) else None
    return st, res.as_dict(), reps


def nat_server_cancel(srv: Server, ticket: int) -> int:
    return _check(lib().nat_server_cancel(srv.handle, C.c_uint64(ticket)))


def nat_server_stats_read(srv: Server) -> dict:
    s = nat_server_stats()
    _check(lib().nat_server_stats_read(srv.handle, C.byref(s)))
    return s.as_dict()


def nat_server_destroy(srv: Server):
    srv.close()


# ------------------------------------------------------------ neural field
class NeuralField:
    """The neural acoustic transfer field of include/nat_neural.h: inputs are
    float32 device rows (theta, phi, r, v_0 .. v_{n_v-1}, f), targets float32
    device rows [B, n_out]."""

    def __init__(self, ctx: Context, n_v: int, n_out: int, r_lo: float, r_hi: float, seed: int = 0):
        self.ctx = ctx
        self.n_v, self.n_out = int(n_v), int(n_out)
        self.r_lo, self.r_hi = float(r_lo), float(r_hi)
        h = _P()
        _check(lib().nat_nf_create(ctx.handle, self.n_v, self.n_out, float(r_lo), float(r_hi),
                                   C.c_uint64(seed), C.byref(h)))
        self.handle = h
        ctx._adopt(self)
        d = C.c_int32()
        n = C.c_int64()
        _check(lib().nat_nf_info(h, C.byref(d), C.byref(n)))
        self.input_dim, self.n_params = d.value, n.value

    def _host(self, fn, what):
        out = np.empty(self.n_params, dtype=np.float32)
        _check(fn(self.handle, out.ctypes.data_as(_P), self.n_params))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().nat_nf_set_params(self.handle, p.ctypes.data_as(_P), int(p.size)))

    def get_params(self):
        return self._host(lib().nat_nf_get_params, "params")

    def get_grads(self):
        return self._host(lib().nat_nf_get_grads, "grads")

    def _rows(self, inputs, targets=None):
        import torch
        B = int(inputs.shape[0]) if inputs.dim() == 2 else -1
        pi = _dptr(inputs, torch.float32, (B, 3 + self.n_v + 1), "inputs")
        pt = None
        if targets is not None:
            pt = _dptr(targets, torch.float32, (B, self.n_out), "targets")
        return B, pi, pt

    def loss_grad(self, inputs, targets, stream=None) -> float:
        B, pi, pt = self._rows(inputs, targets)
        loss = C.c_double()
        _check(lib().nat_nf_loss_grad(self.handle, pi, pt, B, C.byref(loss), _stream(stream)))
        return loss.value

    def train_step(self, inputs, targets, step: int, total_steps: int, want_loss: bool = True, stream=None):
        B, pi, pt = self._rows(inputs, targets)
        loss = C.c_double()
        _check(lib().nat_nf_train_step(self.handle, pi, pt, B, int(step), int(total_steps),
                                       C.byref(loss) if want_loss else None, _stream(stream)))
        return loss.value if want_loss else None

    def infer(self, inputs, out=None, stream=None):
        import torch
        B, pi, _ = self._rows(inputs)
        if out is None:
            out = torch.empty((B, self.n_out), dtype=torch.float32, device=inputs.device)
        _check(lib().nat_nf_infer(self.handle, pi, B, _dptr(out, torch.float32, (B, self.n_out), "out"),
                                  _stream(stream)))
        return out

    def save(self, path):
        """Writes the field's sizes, training shell and parameters to a .npz
        file (the Adam moments are not saved: a field loaded from it starts
        them at zero, as after set_params)."""
        np.savez(path, format=np.int64(1), n_v=np.int64(self.n_v), n_out=np.int64(self.n_out),
                 r_lo=np.float64(self.r_lo), r_hi=np.float64(self.r_hi), params=self.get_params())

    @classmethod
    def load(cls, ctx: Context, path):
        """A field made from a file written by save()."""
        with np.load(path, allow_pickle=False) as z:
            if int(z["format"]) != 1:
                raise ValueError(f"{path}: unknown neural-field file format {int(z['format'])}")
            nf = cls(ctx, int(z["n_v"]), int(z["n_out"]), float(z["r_lo"]), float(z["r_hi"]))
            nf.set_params(z["params"])
        return nf

    def close(self):
        if getattr(self, "handle", None):
            lib().nat_nf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
