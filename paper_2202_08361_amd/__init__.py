"""MI355X (gfx950) implementation of the parallel one-sided Jacobi SVD hot path
of V. Novakovic, arXiv:2202.08361: batched branch-free 2x2 Hermitian EVD,
scaled dot-products, scaled Gram matrices and column-pair rotations, as HIP
kernels behind the C ABI of ``include/jsvd.h``.

This package is a thin ctypes binding over ``libjsvd.so``: it marshals torch
tensors (device memory) and the current HIP stream into the C calls and does
no arithmetic of the method itself.  Importing it does not load the library;
the first call does, and raises if the library is not built (there is no CPU
fallback).

Matrices are column-major: an ``m x n`` matrix is a float64 CUDA tensor of
shape ``(m, n)`` with ``stride(0) == 1`` (see :func:`fortran_empty`), or a
float32 one for the single precision variant (``State(..., fp32=True)``,
:func:`gesvj` on float32 input).  Complex matrices are split into real and
imaginary tensors.
"""
from __future__ import annotations

import ctypes as _ct
import os as _os

__all__ = [
    "lib", "JsvdError", "fortran_empty", "to_device_fortran", "evd2_batched", "State", "gesvj",
    "gesvj_batched", "Server", "split", "merge", "EVD_SCALED", "EVD_SINFORM", "NO_PERMUTE", "PERMUTE", "COMPENSATED", "NO_GS",
    "dot_scaled_batched", "evd2_batched_f32", "nrmf_batched",
]

_HERE = _os.path.dirname(_os.path.abspath(__file__))
LIB_PATH = _os.path.join(_HERE, "libjsvd.so")

OK, NOT_CONVERGED, EINVAL, ENONFINITE, EZERO, ENOMEM, EDEVICE, EAGAIN, ENOTFOUND = 0, 1, -1, -2, -3, -4, -5, -6, -7
EVD_SCALED, EVD_SINFORM = 1, 2
NO_PERMUTE = 1
COMPENSATED = 2
NO_GS = 4
PERMUTE = 8

_lib = None


class JsvdError(RuntimeError):
    def __init__(self, status, what=""):
        msg = lib().jsvd_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} ({status})")
        self.status = status


class _Info(_ct.Structure):
    _fields_ = [("steps", _ct.c_int64), ("sweeps", _ct.c_int64), ("T", _ct.c_int64),
                ("last_t", _ct.c_int64), ("swaps", _ct.c_int64), ("s", _ct.c_int32),
                ("rescaled", _ct.c_int32), ("Mt", _ct.c_double), ("converged", _ct.c_int32),
                ("status", _ct.c_int32), ("last_sweep_T", _ct.c_int64), ("last_sweep_swaps", _ct.c_int64),
                ("gs", _ct.c_int64), ("last_sweep_gs", _ct.c_int64), ("loop_sweeps", _ct.c_int64),
                ("loop_redos", _ct.c_int64), ("skipped_pairs", _ct.c_int64), ("local_sweeps", _ct.c_int64)]


class ServeConfig(_ct.Structure):
    _fields_ = [("hbm_budget_bytes", _ct.c_size_t), ("max_slots", _ct.c_int),
                ("max_sweeps", _ct.c_int), ("max_queue", _ct.c_int), ("flags", _ct.c_uint),
                ("max_large", _ct.c_int)]


class Request(_ct.Structure):
    _fields_ = [("m", _ct.c_int), ("n", _ct.c_int), ("is_complex", _ct.c_int),
                ("G_re", _ct.c_void_p), ("G_im", _ct.c_void_p), ("ldg", _ct.c_size_t),
                ("V_re", _ct.c_void_p), ("V_im", _ct.c_void_p), ("ldv", _ct.c_size_t),
                ("sv_e", _ct.c_void_p), ("sv_f", _ct.c_void_p), ("tag", _ct.c_uint64)]


class ServeStats(_ct.Structure):
    _fields_ = [("submitted", _ct.c_uint64), ("completed", _ct.c_uint64), ("rejected", _ct.c_uint64),
                ("p50_ns", _ct.c_double), ("p99_ns", _ct.c_double), ("p50_queue_ns", _ct.c_double),
                ("p99_queue_ns", _ct.c_double), ("svds_per_s", _ct.c_double),
                ("queue_depth", _ct.c_int), ("active", _ct.c_int), ("hbm_in_use", _ct.c_size_t),
                ("p50_service_ns", _ct.c_double), ("p99_service_ns", _ct.c_double),
                ("persistent_sweeps", _ct.c_uint64), ("persistent_redos", _ct.c_uint64)]


def lib():
    """Load libjsvd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not _os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(the HIP library is required, there is no CPU fallback)")
        L = _ct.CDLL(LIB_PATH)
        vp, sz, i, u, d = _ct.c_void_p, _ct.c_size_t, _ct.c_int, _ct.c_uint, _ct.c_double
        L.jsvd_version.restype = i
        L.jsvd_strerror.restype = _ct.c_char_p
        L.jsvd_strerror.argtypes = [i]
        L.jsvd_evd2_batched.restype = i
        L.jsvd_evd2_batched.argtypes = [sz, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, u, vp]
        L.jsvd_evd2_batched_f32.restype = i
        L.jsvd_evd2_batched_f32.argtypes = [sz, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, u, vp]
        L.jsvd_evd2_stream_ceiling.restype = i
        L.jsvd_evd2_stream_ceiling.argtypes = [sz, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.jsvd_state_create.restype = i
        L.jsvd_state_create.argtypes = [i, i, i, _ct.POINTER(vp)]
        L.jsvd_state_create_f32.restype = i
        L.jsvd_state_create_f32.argtypes = [i, i, i, _ct.POINTER(vp)]
        L.jsvd_state_load_f32.restype = i
        L.jsvd_state_load_f32.argtypes = [vp, vp, vp, sz, vp]
        L.jsvd_state_save_f32.restype = i
        L.jsvd_state_save_f32.argtypes = [vp, vp, vp, sz, vp, vp, sz, vp, vp, _ct.POINTER(_ct.c_int32),
                                          _ct.POINTER(d), _ct.POINTER(_ct.c_int64), vp]
        L.jsvd_state_restore_f32.restype = i
        L.jsvd_state_restore_f32.argtypes = [vp, vp, vp, sz, vp, vp, sz, _ct.c_int32, d, _ct.c_int64, vp]
        L.jsvd_state_finalize_f32.restype = i
        L.jsvd_state_finalize_f32.argtypes = [vp, vp, vp, sz, vp, vp, sz, vp, vp, vp, vp]
        L.jsvd_nrmf_batched.restype = i
        L.jsvd_nrmf_batched.argtypes = [i, i, vp, vp, sz, i, vp, vp, vp, vp, vp]
        L.jsvd_gesvj_f32.restype = i
        L.jsvd_gesvj_f32.argtypes = [i, i, vp, vp, sz, vp, vp, sz, vp, vp, vp, i, _ct.POINTER(i), u, vp]
        L.jsvd_state_destroy.restype = None
        L.jsvd_state_destroy.argtypes = [vp]
        L.jsvd_state_load.restype = i
        L.jsvd_state_load.argtypes = [vp, vp, vp, sz, vp]
        L.jsvd_step.restype = i
        L.jsvd_step.argtypes = [vp, vp]
        L.jsvd_sweep.restype = i
        L.jsvd_sweep.argtypes = [vp, vp]
        L.jsvd_state_iterate.restype = i
        L.jsvd_state_iterate.argtypes = [vp, vp]
        L.jsvd_state_set_loop_wait.restype = i
        L.jsvd_state_set_loop_wait.argtypes = [vp, d]
        L.jsvd_state_set_loop_local.restype = i
        L.jsvd_state_set_loop_local.argtypes = [vp, i]
        L.jsvd_state_query.restype = i
        L.jsvd_state_query.argtypes = [vp, _ct.POINTER(_Info), vp]
        L.jsvd_state_save.restype = i
        L.jsvd_state_save.argtypes = [vp, vp, vp, sz, vp, vp, sz, vp, vp, _ct.POINTER(_ct.c_int32),
                                      _ct.POINTER(d), _ct.POINTER(_ct.c_int64), vp]
        L.jsvd_state_restore.restype = i
        L.jsvd_state_restore.argtypes = [vp, vp, vp, sz, vp, vp, sz, _ct.c_int32, d, _ct.c_int64, vp]
        L.jsvd_state_finalize.restype = i
        L.jsvd_state_finalize.argtypes = [vp, vp, vp, sz, vp, vp, sz, vp, vp, vp, vp]
        L.jsvd_state_set_launch.restype = i
        L.jsvd_state_set_launch.argtypes = [vp, i]
        L.jsvd_state_set_flags.restype = i
        L.jsvd_state_set_flags.argtypes = [vp, u]
        L.jsvd_dot_scaled_batched.restype = i
        L.jsvd_dot_scaled_batched.argtypes = [i, i, vp, vp, vp, vp, sz, vp, vp, vp, vp, vp, vp, u, vp]
        L.jsvd_gesvj.restype = i
        L.jsvd_gesvj.argtypes = [i, i, vp, vp, sz, vp, vp, sz, vp, vp, vp, i, _ct.POINTER(i), u, vp]
        L.jsvd_gesvj_batched.restype = i
        L.jsvd_gesvj_batched.argtypes = [i, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i, vp, vp, vp, u, vp]
        L.jsvd_gesvj_batched_noalloc.restype = i
        L.jsvd_gesvj_batched_noalloc.argtypes = [i, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i, vp, vp, vp, u,
                                                 vp]
        L.jsvd_batched_tune.restype = i
        L.jsvd_batched_tune.argtypes = [i, vp, vp, vp, u, vp]
        L.jsvd_batched_set_launch.restype = i
        L.jsvd_batched_set_launch.argtypes = [i]
        L.jsvd_batched_launch_of.restype = i
        L.jsvd_batched_launch_of.argtypes = [i, i, i, u]
        L.jsvd_batched_set_schedule.restype = i
        L.jsvd_batched_set_schedule.argtypes = [i, i, i]
        L.jsvd_batched_set_tuning.restype = i
        L.jsvd_batched_set_tuning.argtypes = [u]
        L.jsvd_batched_schedule_of.restype = i
        L.jsvd_batched_schedule_of.argtypes = [i, i, i, u, _ct.POINTER(i), _ct.POINTER(i), _ct.POINTER(i)]
        L.jsvd_serve_create.restype = i
        L.jsvd_serve_create.argtypes = [_ct.POINTER(ServeConfig), _ct.POINTER(vp)]
        L.jsvd_serve_submit.restype = i
        L.jsvd_serve_submit.argtypes = [vp, _ct.POINTER(Request), _ct.POINTER(_ct.c_uint64)]
        L.jsvd_serve_poll.restype = i
        L.jsvd_serve_poll.argtypes = [vp, _ct.c_uint64, _ct.POINTER(i), _ct.POINTER(i), _ct.POINTER(i)]
        L.jsvd_serve_wait.restype = i
        L.jsvd_serve_wait.argtypes = [vp, _ct.c_uint64, _ct.POINTER(i), _ct.POINTER(i)]
        L.jsvd_serve_stats_get.restype = i
        L.jsvd_serve_stats_get.argtypes = [vp, _ct.POINTER(ServeStats)]
        L.jsvd_serve_load.restype = i
        L.jsvd_serve_load.argtypes = [vp, _ct.POINTER(i), _ct.POINTER(i), _ct.POINTER(sz)]
        L.jsvd_serve_destroy.restype = i
        L.jsvd_serve_destroy.argtypes = [vp]
        L.jsvd_split.restype = i
        L.jsvd_split.argtypes = [i, i, vp, sz, vp, vp, sz, vp]
        L.jsvd_merge.restype = i
        L.jsvd_merge.argtypes = [i, i, vp, vp, sz, vp, sz, vp]
        _lib = L
    return _lib


def _check(status, what, allow=(OK,)):
    if status not in allow:
        raise JsvdError(status, what)
    return status


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return _ct.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else _ct.c_void_p(t.data_ptr())


def _vec(t, n, name):
    torch = _torch()
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() >= n):
        raise ValueError(f"{name}: expected a contiguous float64 CUDA tensor of >= {n} elements")
    return t


def _mat(t, m, n, name, dtype=None):
    """Column-major check: shape (m, n), stride(0) == 1, dtype (default
    float64); returns the leading dimension."""
    torch = _torch()
    dtype = torch.float64 if dtype is None else dtype
    if not (t.is_cuda and t.dtype == dtype):
        raise ValueError(f"{name}: expected a {dtype} CUDA tensor")
    if tuple(t.shape) != (m, n):
        raise ValueError(f"{name}: expected shape {(m, n)}, got {tuple(t.shape)}")
    if m > 1 and t.stride(0) != 1:
        raise ValueError(f"{name}: must be column-major (stride(0) == 1); use fortran_empty")
    if n > 1 and t.stride(1) < m:
        raise ValueError(f"{name}: leading dimension {t.stride(1)} < {m}")
    return t.stride(1) if n > 1 else max(m, 1)


def fortran_empty(m, n, device="cuda", ld=None, dtype=None):
    """An uninitialised column-major (m, n) tensor (float64 unless dtype) with
    leading dimension ld >= m."""
    torch = _torch()
    ld = m if ld is None else ld
    dtype = torch.float64 if dtype is None else dtype
    return torch.empty((n, ld), dtype=dtype, device=device).t()[:m]


def to_device_fortran(a, device="cuda", dtype=None):
    """Copy a host array (numpy / torch, any order) into a column-major device
    tensor (float64 unless dtype; the values are converted on the host)."""
    torch = _torch()
    dtype = torch.float64 if dtype is None else dtype
    a = torch.as_tensor(a).to(dtype)
    m, n = a.shape
    out = fortran_empty(m, n, device, dtype=dtype)
    out.copy_(a)
    return out


# ---------------------------------------------------------------------------- EVD
def evd2_batched(a11, a22, a21_re, a21_im=None, flags=0, out=None, with_lambda=True, with_zp=True,
                 stream=None):
    """Batched 2x2 EVD (Listing 1) over float64 CUDA vectors.  Returns a dict of
    tensors: cos, ctan_re, ctan_im (complex only), lambda1, lambda2, zp."""
    torch = _torch()
    r = a11.numel()
    for t, nm in ((a11, "a11"), (a22, "a22"), (a21_re, "a21_re"), (a21_im, "a21_im")):
        _vec(t, r, nm)
    dev = a11.device
    if out is None:
        out = dict(cos=torch.empty(r, dtype=torch.float64, device=dev),
                   ctan_re=torch.empty(r, dtype=torch.float64, device=dev))
        if a21_im is not None:
            out["ctan_im"] = torch.empty(r, dtype=torch.float64, device=dev)
        if with_lambda:
            out["lambda1"] = torch.empty(r, dtype=torch.float64, device=dev)
            out["lambda2"] = torch.empty(r, dtype=torch.float64, device=dev)
        if with_zp:
            out["zp"] = torch.empty(r, dtype=torch.int32, device=dev)
    st = lib().jsvd_evd2_batched(r, _ptr(a11), _ptr(a22), _ptr(a21_re), _ptr(a21_im), _ptr(out["cos"]),
                                 _ptr(out["ctan_re"]), _ptr(out.get("ctan_im")), _ptr(out.get("lambda1")),
                                 _ptr(out.get("lambda2")), _ptr(out.get("zp")), flags, _stream(stream))
    _check(st, "jsvd_evd2_batched")
    return out


def evd2_stream_ceiling(a11, a22, a21_re, a21_im, out, stream=None):
    """jsvd_evd2_stream_ceiling: the batched EVD's streams moved without its
    arithmetic, into the output tensors of an evd2_batched call (with lambda
    and zp).  A measurement aid; the outputs carry no meaning."""
    r = a11.numel()
    _check(lib().jsvd_evd2_stream_ceiling(r, _ptr(a11), _ptr(a22), _ptr(a21_re), _ptr(a21_im), _ptr(out["cos"]),
                                          _ptr(out["ctan_re"]), _ptr(out.get("ctan_im")), _ptr(out["lambda1"]),
                                          _ptr(out["lambda2"]), _ptr(out["zp"]), _stream(stream)),
           "jsvd_evd2_stream_ceiling")


def dot_scaled_batched(Q_re, P_re, eq, fq, ep, fp, Q_im=None, P_im=None, flags=0, stream=None):
    """Batched scaled dot-products (jsvd_dot_scaled_batched): for every column j
    of the m x npairs column-major tensors, z_j = (q_j 2^-eq_j)^* (p_j 2^-ep_j)
    / (fq_j fp_j).  Returns (z_re, z_im) (z_im None for real data)."""
    torch = _torch()
    m, npairs = Q_re.shape
    ld = _mat(Q_re, m, npairs, "Q_re")
    for t, nm in ((P_re, "P_re"), (Q_im, "Q_im"), (P_im, "P_im")):
        if t is not None and _mat(t, m, npairs, nm) != ld:
            raise ValueError(f"{nm}: leading dimension differs from Q_re's")
    for t, nm in ((eq, "eq"), (fq, "fq"), (ep, "ep"), (fp, "fp")):
        _vec(t, npairs, nm)
    z_re = torch.empty(npairs, dtype=torch.float64, device=Q_re.device)
    z_im = torch.empty(npairs, dtype=torch.float64, device=Q_re.device) if Q_im is not None else None
    _check(lib().jsvd_dot_scaled_batched(npairs, m, _ptr(Q_re), _ptr(Q_im), _ptr(P_re), _ptr(P_im), ld,
                                         _ptr(eq), _ptr(fq), _ptr(ep), _ptr(fp), _ptr(z_re), _ptr(z_im),
                                         flags, _stream(stream)), "jsvd_dot_scaled_batched")
    return z_re, z_im


def nrmf_batched(X_re, X_im=None, lanes=1024, stream=None):
    """Widened-exponent Frobenius norms of the columns of an (m, ncols)
    column-major float64 CUDA tensor (Alg. rnF, jsvd_nrmf_batched).  Returns
    (e2, f2, e, f): ||x_j||^2 = 2^e2 f2, ||x_j|| = 2^e f, float64 tensors."""
    torch = _torch()
    m, ncols = X_re.shape
    ld = _mat(X_re, m, ncols, "X_re")
    if X_im is not None and _mat(X_im, m, ncols, "X_im") != ld:
        raise ValueError("X_re and X_im need the same leading dimension")
    out = [torch.empty(ncols, dtype=torch.float64, device=X_re.device) for _ in range(4)]
    _check(lib().jsvd_nrmf_batched(ncols, m, _ptr(X_re), _ptr(X_im), ld, lanes, *[_ptr(o) for o in out],
                                   _stream(stream)), "jsvd_nrmf_batched")
    return tuple(out)


def evd2_batched_f32(a11, a22, a21_re, a21_im=None, flags=0, out=None, with_lambda=True, with_zp=True,
                     stream=None):
    """Single precision batched 2x2 EVD over float32 CUDA vectors (same outputs
    as evd2_batched, float32)."""
    torch = _torch()
    r = a11.numel()
    for t, nm in ((a11, "a11"), (a22, "a22"), (a21_re, "a21_re"), (a21_im, "a21_im")):
        if t is not None and not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() >= r):
            raise ValueError(f"{nm}: expected a contiguous float32 CUDA tensor of {r} elements")
    dev = a11.device
    if out is None:
        out = dict(cos=torch.empty(r, dtype=torch.float32, device=dev),
                   ctan_re=torch.empty(r, dtype=torch.float32, device=dev))
        if a21_im is not None:
            out["ctan_im"] = torch.empty(r, dtype=torch.float32, device=dev)
        if with_lambda:
            out["lambda1"] = torch.empty(r, dtype=torch.float32, device=dev)
            out["lambda2"] = torch.empty(r, dtype=torch.float32, device=dev)
        if with_zp:
            out["zp"] = torch.empty(r, dtype=torch.int32, device=dev)
    st = lib().jsvd_evd2_batched_f32(r, _ptr(a11), _ptr(a22), _ptr(a21_re), _ptr(a21_im), _ptr(out["cos"]),
                                     _ptr(out["ctan_re"]), _ptr(out.get("ctan_im")), _ptr(out.get("lambda1")),
                                     _ptr(out.get("lambda2")), _ptr(out.get("zp")), flags, _stream(stream))
    _check(st, "jsvd_evd2_batched_f32")
    return out


# ---------------------------------------------------------------------------- state
class State:
    """Device-resident SVD state (jsvd_state_*): the hot path one step at a
    time; fp32=True makes a single precision state (float32 tensors, the
    jsvd_state_*_f32 calls)."""

    def __init__(self, m, n, cplx=False, fp32=False):
        torch = _torch()
        self.m, self.n, self.cplx, self.fp32 = m, n, bool(cplx), bool(fp32)
        self.dtype = torch.float32 if fp32 else torch.float64
        self._sfx = "_f32" if fp32 else ""
        h = _ct.c_void_p()
        create = lib().jsvd_state_create_f32 if fp32 else lib().jsvd_state_create
        _check(create(m, n, int(cplx), _ct.byref(h)), "jsvd_state_create" + self._sfx)
        self._h = h

    def _fn(self, name):
        return getattr(lib(), name + self._sfx)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.jsvd_state_destroy(self._h)
            self._h = None

    def close(self):
        self.__del__()

    def load(self, G_re, G_im=None, stream=None):
        ld = _mat(G_re, self.m, self.n, "G_re", self.dtype)
        if G_im is not None and _mat(G_im, self.m, self.n, "G_im", self.dtype) != ld:
            raise ValueError("G_re and G_im need the same leading dimension")
        return _check(self._fn("jsvd_state_load")(self._h, _ptr(G_re), _ptr(G_im), ld, _stream(stream)),
                      "jsvd_state_load" + self._sfx, allow=(OK, ENONFINITE, EZERO))

    def set_launch(self, threads):
        _check(lib().jsvd_state_set_launch(self._h, threads), "jsvd_state_set_launch")

    def set_flags(self, flags):
        _check(lib().jsvd_state_set_flags(self._h, flags), "jsvd_state_set_flags")

    def step(self, stream=None):
        _check(lib().jsvd_step(self._h, _stream(stream)), "jsvd_step")

    def sweep(self, stream=None):
        _check(lib().jsvd_sweep(self._h, _stream(stream)), "jsvd_sweep")

    def iterate(self, stream=None):
        """Sweeps until the state stops (jsvd_state_iterate; synchronises)."""
        _check(lib().jsvd_state_iterate(self._h, _stream(stream)), "jsvd_state_iterate")

    def set_loop_wait(self, seconds):
        """Wait budget of a persistent sweep's workgroup for one column
        (jsvd_state_set_loop_wait; 0 turns persistent sweeps off)."""
        _check(lib().jsvd_state_set_loop_wait(self._h, float(seconds)), "jsvd_state_set_loop_wait")

    def set_loop_local(self, allow):
        """Allow (True, the default) or forbid the L2-local mode of persistent
        sweeps (jsvd_state_set_loop_local)."""
        _check(lib().jsvd_state_set_loop_local(self._h, 1 if allow else 0), "jsvd_state_set_loop_local")

    def query(self, stream=None):
        info = _Info()
        _check(lib().jsvd_state_query(self._h, _ct.byref(info), _stream(stream)), "jsvd_state_query")
        return {f: getattr(info, f) for f, _ in _Info._fields_}

    def save(self, stream=None):
        torch = _torch()
        dt = self.dtype
        Gr = fortran_empty(self.m, self.n, dtype=dt)
        Gi = fortran_empty(self.m, self.n, dtype=dt) if self.cplx else None
        Vr = fortran_empty(self.n, self.n, dtype=dt)
        Vi = fortran_empty(self.n, self.n, dtype=dt) if self.cplx else None
        e = torch.empty(self.n, dtype=dt, device="cuda")
        f = torch.empty(self.n, dtype=dt, device="cuda")
        s, Mt, k = _ct.c_int32(), _ct.c_double(), _ct.c_int64()
        _check(self._fn("jsvd_state_save")(self._h, _ptr(Gr), _ptr(Gi), self.m, _ptr(Vr), _ptr(Vi), self.n,
                                           _ptr(e), _ptr(f), _ct.byref(s), _ct.byref(Mt), _ct.byref(k),
                                           _stream(stream)), "jsvd_state_save" + self._sfx)
        return dict(G_re=Gr, G_im=Gi, V_re=Vr, V_im=Vi, e=e, f=f, s=s.value, Mt=Mt.value, k=k.value)

    def restore(self, G_re, G_im, V_re, V_im, s, Mt, k, stream=None):
        ldg = _mat(G_re, self.m, self.n, "G_re", self.dtype)
        ldv = _mat(V_re, self.n, self.n, "V_re", self.dtype)
        _check(self._fn("jsvd_state_restore")(self._h, _ptr(G_re), _ptr(G_im), ldg, _ptr(V_re), _ptr(V_im), ldv,
                                              int(s), float(Mt), int(k), _stream(stream)),
               "jsvd_state_restore" + self._sfx)

    def finalize(self, stream=None):
        torch = _torch()
        dt = self.dtype
        U_re = fortran_empty(self.m, self.n, dtype=dt)
        U_im = fortran_empty(self.m, self.n, dtype=dt) if self.cplx else None
        V_re = fortran_empty(self.n, self.n, dtype=dt)
        V_im = fortran_empty(self.n, self.n, dtype=dt) if self.cplx else None
        sv_e = torch.empty(self.n, dtype=dt, device="cuda")
        sv_f = torch.empty(self.n, dtype=dt, device="cuda")
        sv = torch.empty(self.n, dtype=dt, device="cuda")
        _check(self._fn("jsvd_state_finalize")(self._h, _ptr(U_re), _ptr(U_im), self.m, _ptr(V_re), _ptr(V_im),
                                               self.n, _ptr(sv_e), _ptr(sv_f), _ptr(sv), _stream(stream)),
               "jsvd_state_finalize" + self._sfx)
        return dict(U_re=U_re, U_im=U_im, V_re=V_re, V_im=V_im, sv_e=sv_e, sv_f=sv_f, sv=sv)


def gesvj(G_re, G_im=None, max_sweeps=0, flags=0, overwrite=False, stream=None):
    """The whole SVD G = U diag(sigma) V^*.  Returns a dict with U (in place of a
    copy of G unless overwrite), V, sv_e, sv_f, sv, status, sweeps.  float32
    input runs the single precision variant (jsvd_gesvj_f32)."""
    torch = _torch()
    m, n = G_re.shape
    dt = G_re.dtype
    if dt not in (torch.float64, torch.float32):
        raise ValueError("G_re: expected a float64 or float32 CUDA tensor")
    name = "jsvd_gesvj_f32" if dt == torch.float32 else "jsvd_gesvj"
    if not overwrite:
        g = fortran_empty(m, n, dtype=dt)
        g.copy_(G_re)
        G_re = g
        if G_im is not None:
            g = fortran_empty(m, n, dtype=dt)
            g.copy_(G_im)
            G_im = g
    ldg = _mat(G_re, m, n, "G_re", dt)
    if G_im is not None and _mat(G_im, m, n, "G_im", dt) != ldg:
        raise ValueError("G_re and G_im need the same leading dimension")
    V_re = fortran_empty(n, n, dtype=dt)
    V_im = fortran_empty(n, n, dtype=dt) if G_im is not None else None
    sv_e = torch.empty(n, dtype=dt, device="cuda")
    sv_f = torch.empty(n, dtype=dt, device="cuda")
    sv = torch.empty(n, dtype=dt, device="cuda")
    sw = _ct.c_int()
    st = getattr(lib(), name)(m, n, _ptr(G_re), _ptr(G_im), ldg, _ptr(V_re), _ptr(V_im), n, _ptr(sv_e),
                              _ptr(sv_f), _ptr(sv), max_sweeps, _ct.byref(sw), flags, _stream(stream))
    _check(st, name, allow=(OK, NOT_CONVERGED, ENONFINITE, EZERO))
    return dict(status=st, sweeps=sw.value, U_re=G_re, U_im=G_im, V_re=V_re, V_im=V_im, sv_e=sv_e,
                sv_f=sv_f, sv=sv)


def gesvj_batched(mats, max_sweeps=0, flags=0, stream=None, noalloc=False):
    """Many SVDs in one call.  ``mats`` is a list of (G_re, G_im|None) column-major
    device tensors, overwritten by U.  Returns a list of dicts like :func:`gesvj`.
    noalloc: the library allocates no device memory for the call
    (jsvd_gesvj_batched_noalloc: at most 8192 matrices, each at most 512 x 512)."""
    torch = _torch()
    cnt = len(mats)
    I = _ct.c_int * cnt
    P = _ct.c_void_p * cnt
    Z = _ct.c_size_t * cnt
    m_a, n_a, c_a = I(), I(), I()
    gr, gi, vr, vi, se, sf = P(), P(), P(), P(), P(), P()
    lg, lv = Z(), Z()
    res = []
    for idx, (Gr, Gi) in enumerate(mats):
        m, n = Gr.shape
        ld = _mat(Gr, m, n, "G_re")
        if Gi is not None and _mat(Gi, m, n, "G_im") != ld:
            raise ValueError("G_re and G_im need the same leading dimension")
        Vr = fortran_empty(n, n)
        Vi = fortran_empty(n, n) if Gi is not None else None
        e = torch.empty(n, dtype=torch.float64, device="cuda")
        f = torch.empty(n, dtype=torch.float64, device="cuda")
        m_a[idx], n_a[idx], c_a[idx] = m, n, int(Gi is not None)
        gr[idx], gi[idx] = Gr.data_ptr(), (Gi.data_ptr() if Gi is not None else None)
        vr[idx], vi[idx] = Vr.data_ptr(), (Vi.data_ptr() if Vi is not None else None)
        se[idx], sf[idx] = e.data_ptr(), f.data_ptr()
        lg[idx], lv[idx] = ld, n
        res.append(dict(U_re=Gr, U_im=Gi, V_re=Vr, V_im=Vi, sv_e=e, sv_f=f))
    sweeps, status, trans = I(), I(), (_ct.c_int64 * cnt)()
    fn = lib().jsvd_gesvj_batched_noalloc if noalloc else lib().jsvd_gesvj_batched
    st = fn(cnt, m_a, n_a, c_a, gr, gi, lg, vr, vi, lv, se, sf, max_sweeps, sweeps, status, trans, flags,
            _stream(stream))
    _check(st, "jsvd_gesvj_batched_noalloc" if noalloc else "jsvd_gesvj_batched",
           allow=(OK, NOT_CONVERGED, ENONFINITE, EZERO))
    for idx in range(cnt):
        res[idx]["status"] = status[idx]
        res[idx]["sweeps"] = sweeps[idx]
        res[idx]["transformations"] = trans[idx]
    return res


def batched_tune(shapes, flags=0, stream=None):
    """Measure the batched launch shape (threads per matrix) of the classes of
    these (m, n, is_complex) shapes (jsvd_batched_tune)."""
    cnt = len(shapes)
    I = _ct.c_int * max(cnt, 1)
    m_a, n_a, c_a = I(), I(), I()
    for idx, (m, n, c) in enumerate(shapes):
        m_a[idx], n_a[idx], c_a[idx] = m, n, int(bool(c))
    _check(lib().jsvd_batched_tune(cnt, m_a, n_a, c_a, flags, _stream(stream)), "jsvd_batched_tune")


def batched_set_launch(threads_per_matrix):
    """Force the batched threads per matrix (128, 256, 512; 0 = measured)."""
    _check(lib().jsvd_batched_set_launch(threads_per_matrix), "jsvd_batched_set_launch")


def batched_launch_of(m, n, cplx=False, flags=0):
    """Threads per matrix a batched call would use now for an m x n matrix
    (0: not a batched shape)."""
    r = lib().jsvd_batched_launch_of(m, n, int(bool(cplx)), flags)
    if r < 0:
        _check(r, "jsvd_batched_launch_of")
    return r


TUNE_DENSE = 1
TUNE_WGS = 2


def batched_set_schedule(threads_per_matrix, dense=0, workgroups_per_cu=0):
    """Force the batched schedule of every class (threads 0 = measured)."""
    _check(lib().jsvd_batched_set_schedule(threads_per_matrix, int(dense), workgroups_per_cu),
           "jsvd_batched_set_schedule")


def batched_set_tuning(candidates=TUNE_DENSE | TUNE_WGS):
    """The candidate schedules the batched tuner tries (and forget the measured ones)."""
    _check(lib().jsvd_batched_set_tuning(candidates), "jsvd_batched_set_tuning")


def batched_schedule_of(m, n, cplx=False, flags=0):
    """(threads per matrix, dense, workgroups per CU) a batched call would use
    now for an m x n matrix (threads 0: not a batched shape)."""
    t, d, w = _ct.c_int(), _ct.c_int(), _ct.c_int()
    _check(lib().jsvd_batched_schedule_of(m, n, int(bool(cplx)), flags, _ct.byref(t), _ct.byref(d), _ct.byref(w)),
           "jsvd_batched_schedule_of")
    return t.value, d.value, w.value


# ---------------------------------------------------------------------------- serving
class Server:
    """Continuous-batching SVD server (jsvd_serve_*)."""

    def __init__(self, hbm_budget_bytes=8 << 30, max_slots=64, max_sweeps=0, max_queue=0, flags=0, max_large=0):
        cfg = ServeConfig(hbm_budget_bytes, max_slots, max_sweeps, max_queue, flags, max_large)
        h = _ct.c_void_p()
        _check(lib().jsvd_serve_create(_ct.byref(cfg), _ct.byref(h)), "jsvd_serve_create")
        self._h = h
        self._keep = {}

    def submit(self, G_re, G_im=None, tag=0):
        """Submit G (overwritten by U); returns a ticket, or None when the queue
        is full.  The server's streams do not order after the caller's, so
        the caller's current stream is waited for first: G must be complete."""
        torch = _torch()
        torch.cuda.current_stream().synchronize()
        m, n = G_re.shape
        ld = _mat(G_re, m, n, "G_re")
        Vr = fortran_empty(n, n)
        Vi = fortran_empty(n, n) if G_im is not None else None
        e = torch.empty(n, dtype=torch.float64, device="cuda")
        f = torch.empty(n, dtype=torch.float64, device="cuda")
        req = Request(m, n, int(G_im is not None), G_re.data_ptr(), G_im.data_ptr() if G_im is not None else None,
                      ld, Vr.data_ptr(), Vi.data_ptr() if Vi is not None else None, n, e.data_ptr(), f.data_ptr(),
                      tag)
        t = _ct.c_uint64()
        st = lib().jsvd_serve_submit(self._h, _ct.byref(req), _ct.byref(t))
        if st == EAGAIN:
            return None
        _check(st, "jsvd_serve_submit")
        self._keep[t.value] = dict(U_re=G_re, U_im=G_im, V_re=Vr, V_im=Vi, sv_e=e, sv_f=f)
        return t.value

    def poll(self, ticket):
        d, s, w = _ct.c_int(), _ct.c_int(), _ct.c_int()
        _check(lib().jsvd_serve_poll(self._h, ticket, _ct.byref(d), _ct.byref(s), _ct.byref(w)), "jsvd_serve_poll")
        return bool(d.value), s.value, w.value

    def wait(self, ticket):
        s, w = _ct.c_int(), _ct.c_int()
        _check(lib().jsvd_serve_wait(self._h, ticket, _ct.byref(s), _ct.byref(w)), "jsvd_serve_wait")
        out = self._keep.pop(ticket)
        out["status"], out["sweeps"] = s.value, w.value
        return out

    def stats(self):
        st = ServeStats()
        _check(lib().jsvd_serve_stats_get(self._h, _ct.byref(st)), "jsvd_serve_stats_get")
        return {f: getattr(st, f) for f, _ in ServeStats._fields_}

    def load(self):
        """(queue_depth, active, hbm_in_use) now, without the latency
        percentiles of stats() (jsvd_serve_load)."""
        q, a, h = _ct.c_int(), _ct.c_int(), _ct.c_size_t()
        _check(lib().jsvd_serve_load(self._h, _ct.byref(q), _ct.byref(a), _ct.byref(h)), "jsvd_serve_load")
        return q.value, a.value, h.value

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().jsvd_serve_destroy(self._h), "jsvd_serve_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------- layout
def split(Z, stream=None):
    """Interleaved complex (m, n) column-major complex128 tensor -> (re, im) split."""
    torch = _torch()
    m, n = Z.shape
    Zr = torch.view_as_real(Z)              # (m, n, 2)
    if Zr.stride(0) != 2:
        raise ValueError("Z must be column-major")
    ldz = Zr.stride(1)
    Xr, Xi = fortran_empty(m, n), fortran_empty(m, n)
    _check(lib().jsvd_split(m, n, _ct.c_void_p(Z.data_ptr()), ldz, _ptr(Xr), _ptr(Xi), m, _stream(stream)),
           "jsvd_split")
    return Xr, Xi


def merge(Xr, Xi, stream=None):
    torch = _torch()
    m, n = Xr.shape
    ld = _mat(Xr, m, n, "X_re")
    Z = torch.empty((n, m), dtype=torch.complex128, device="cuda").t()
    _check(lib().jsvd_merge(m, n, _ptr(Xr), _ptr(Xi), ld, _ct.c_void_p(Z.data_ptr()), 2 * m, _stream(stream)),
           "jsvd_merge")
    return Z
