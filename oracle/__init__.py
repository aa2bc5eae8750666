"""CPU oracle of the parallel one-sided Jacobi SVD hot path (arXiv:2202.08361).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The product path (the HIP library and its
binding) never imports it, and it imports nothing from the product.

A thin ctypes layer over ``liboracle.so`` (plain C, see ``oracle.h``); every
array argument is a numpy float64 array, matrices column-major (Fortran
order), complex data split into real and imaginary arrays.
"""
import ctypes as _ct
import os as _os

import numpy as _np

_HERE = _os.path.dirname(_os.path.abspath(__file__))
_LIB_PATH = _os.path.join(_HERE, "liboracle.so")
_lib = None

OK, NOT_CONVERGED, EINVAL, ENONFINITE, EZERO = 0, 1, -1, -2, -3
EVD_SCALED, EVD_SINFORM = 1, 2
NO_PERMUTE = 1      # the default: U, not U P (named for explicitness)
COMPENSATED = 2
NO_GS = 4
PERMUTE = 8         # apply the EVD's sorting permutation P during the iteration
LANES = 1024

_dp = _ct.POINTER(_ct.c_double)
_fp = _ct.POINTER(_ct.c_float)
_ip = _ct.POINTER(_ct.c_int32)


def lib():
    """Load (building on first use if absent) the oracle library."""
    global _lib
    if _lib is None:
        if not _os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = _ct.CDLL(_LIB_PATH)
        d, i, sz = _ct.c_double, _ct.c_int, _ct.c_size_t
        L.ora_evd2_cplx.restype = i
        L.ora_evd2_cplx.argtypes = [d, d, d, d, _dp, _dp, _dp, _dp, _dp, _ct.c_uint]
        L.ora_evd2_real.restype = i
        L.ora_evd2_real.argtypes = [d, d, d, _dp, _dp, _dp, _dp, _ct.c_uint]
        L.ora_evd2_batch.restype = None
        L.ora_evd2_batch.argtypes = [sz, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _ip, _ct.c_uint, i]
        f = _ct.c_float
        L.ora_sevd2_cplx.restype = i
        L.ora_sevd2_cplx.argtypes = [f, f, f, f, _fp, _fp, _fp, _fp, _fp, _ct.c_uint]
        L.ora_sevd2_real.restype = i
        L.ora_sevd2_real.argtypes = [f, f, f, _fp, _fp, _fp, _fp, _ct.c_uint]
        L.ora_sevd2_batch.restype = None
        L.ora_sevd2_batch.argtypes = [sz, _fp, _fp, _fp, _fp, _fp, _fp, _fp, _fp, _fp, _ip, _ct.c_uint, i]
        L.ora_omp_max_threads.restype = i
        L.ora_set_step_threads.restype = None
        L.ora_set_step_threads.argtypes = [i]
        L.ora_set_exact.restype = None
        L.ora_set_exact.argtypes = [i]
        L.ora_get_exact.restype = i
        L.ora_get_exact.argtypes = []
        L.ora_colnorm_exact.restype = None
        L.ora_colnorm_exact.argtypes = [i, _dp, _dp, _dp, _dp]
        L.ora_dpscl_exact.restype = None
        L.ora_dpscl_exact.argtypes = [i, _dp, _dp, _dp, _dp, d, d, d, d, _dp, _dp]
        L.ora_hypot.restype = d
        L.ora_hypot.argtypes = [d, d]
        L.ora_getexp.restype = i
        L.ora_getexp.argtypes = [d]
        L.ora_lg_bound_m.restype = i
        L.ora_lg_bound_m.argtypes = [i, i]
        L.ora_s_round.restype = i
        L.ora_s_round.argtypes = [d, i]
        L.ora_s_square.restype = i
        L.ora_s_square.argtypes = [d, i, i]
        L.ora_rr_pair.restype = i
        L.ora_rr_pair.argtypes = [i, _ct.c_long, i, _ct.POINTER(i), _ct.POINTER(i)]
        L.ora_rr_steps.restype = i
        L.ora_rr_steps.argtypes = [i]
        L.ora_colnorm.restype = None
        L.ora_colnorm.argtypes = [i, _dp, _dp, _dp, _dp]
        L.ora_dpscl.restype = None
        L.ora_dpscl.argtypes = [i, _dp, _dp, _dp, _dp, d, d, d, d, _dp, _dp]
        L.ora_mul_rd.restype = d
        L.ora_mul_rd.argtypes = [d, d]
        L.ora_2sum.restype = None
        L.ora_2sum.argtypes = [d, d, _dp, _dp]
        L.ora_dpscl_cs.restype = None
        L.ora_dpscl_cs.argtypes = [i, _dp, _dp, _dp, _dp, d, d, d, d, _dp, _dp]
        L.ora_gram.restype = None
        L.ora_gram.argtypes = [d, d, d, d, d, d, _dp, _dp, _dp, _dp]
        L.ora_rot.restype = d
        L.ora_rot.argtypes = [i, _dp, _dp, _dp, _dp, d, d, d, i]
        L.ora_init_ext.restype = i
        L.ora_init_ext.argtypes = [i, i, _dp, _dp, sz, _dp, _dp, sz, _dp, _dp, _ct.POINTER(i), _dp]
        L.ora_step_ext.restype = None
        L.ora_step_ext.argtypes = [i, i, _dp, _dp, sz, _dp, _dp, sz, _dp, _dp, _ct.POINTER(i), _dp,
                                   _ct.c_long, _ct.POINTER(_ct.c_long), _ct.POINTER(_ct.c_long),
                                   _ct.POINTER(_ct.c_long), _ct.POINTER(i), _ct.c_uint]
        L.ora_nrmf.restype = i
        L.ora_nrmf.argtypes = [i, _dp, _dp, i, _dp, _dp, _dp, _dp]
        L.ora_nrmf_lanes.restype = i
        L.ora_nrmf_lanes.argtypes = [i, _dp, _dp, i, _dp, _dp]
        L.ora_gs_case.restype = i
        L.ora_gs_case.argtypes = [d, d, d, d, d]
        L.ora_gs.restype = d
        L.ora_gs.argtypes = [i, _dp, _dp, _dp, _dp, d, d, d, d, d, d]
        L.ora_finalize_ext.restype = None
        L.ora_finalize_ext.argtypes = [i, i, _dp, _dp, sz, _dp, _dp, sz, _dp, _dp, i, _dp, _dp]
        L.ora_gesvj.restype = i
        L.ora_gesvj.argtypes = [i, i, _dp, _dp, sz, _dp, _dp, sz, _dp, _dp, i,
                                _ct.POINTER(i), _ct.POINTER(_ct.c_long), _ct.c_uint]
        f = _ct.c_float
        L.ora_s_hypot.restype = f
        L.ora_s_hypot.argtypes = [f, f]
        L.ora_s_lg_bound_m.restype = i
        L.ora_s_lg_bound_m.argtypes = [i, i]
        L.ora_s_s_round.restype = i
        L.ora_s_s_round.argtypes = [f, i]
        L.ora_s_s_square.restype = i
        L.ora_s_s_square.argtypes = [f, i, i]
        L.ora_s_colnorm.restype = None
        L.ora_s_colnorm.argtypes = [i, _fp, _fp, _fp, _fp]
        L.ora_s_dpscl.restype = None
        L.ora_s_dpscl.argtypes = [i, _fp, _fp, _fp, _fp, f, f, f, f, _fp, _fp]
        L.ora_s_rot.restype = f
        L.ora_s_rot.argtypes = [i, _fp, _fp, _fp, _fp, f, f, f, i]
        L.ora_sgesvj.restype = i
        L.ora_sgesvj.argtypes = [i, i, _fp, _fp, sz, _fp, _fp, sz, _fp, _fp, i,
                                 _ct.POINTER(i), _ct.POINTER(_ct.c_long), _ct.c_uint]
        L.ora_s_init_ext.restype = i
        L.ora_s_init_ext.argtypes = [i, i, _fp, _fp, sz, _fp, _fp, sz, _fp, _fp, _ct.POINTER(i), _fp]
        L.ora_s_step_ext.restype = None
        L.ora_s_step_ext.argtypes = [i, i, _fp, _fp, sz, _fp, _fp, sz, _fp, _fp, _ct.POINTER(i), _fp,
                                     _ct.c_long, _ct.POINTER(_ct.c_long), _ct.POINTER(_ct.c_long),
                                     _ct.POINTER(_ct.c_long), _ct.POINTER(i), _ct.c_uint]
        L.ora_s_gs_case.restype = i
        L.ora_s_gs_case.argtypes = [f, f, f, f, f]
        L.ora_s_gs.restype = f
        L.ora_s_gs.argtypes = [i, _fp, _fp, _fp, _fp, f, f, f, f, f, f]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == _np.float64 and (a.flags.f_contiguous or a.flags.c_contiguous)
    return a.ctypes.data_as(_dp)


def _pi(a):
    if a is None:
        return None
    assert a.dtype == _np.int32
    return a.ctypes.data_as(_ip)


# ---------------------------------------------------------------- EVD
def evd2(a11, a22, a21r, a21i=None, flags=0):
    """Scalar EVD (Listing 1 / Alg. d8jac2).  Returns a dict of the outputs."""
    L = lib()
    c, C, S, l1, l2 = (_ct.c_double() for _ in range(5))
    if a21i is None:
        z = L.ora_evd2_real(a11, a22, a21r, c, C, l1, l2, flags)
        S.value = 0.0
    else:
        z = L.ora_evd2_cplx(a11, a22, a21r, a21i, c, C, S, l1, l2, flags)
    return dict(cos=c.value, ctan_re=C.value, ctan_im=S.value, l1=l1.value, l2=l2.value, zp=z)


def evd2_batch(a11, a22, a21r, a21i=None, flags=0, nthreads=0):
    """Batched EVD over numpy SoA arrays; returns (cos, ctan_re, ctan_im|None, l1, l2, zp)."""
    r = a11.shape[0]
    out = [_np.empty(r) for _ in range(5)]
    zp = _np.empty(r, dtype=_np.int32)
    cti = out[2] if a21i is not None else None
    lib().ora_evd2_batch(r, _p(a11), _p(a22), _p(a21r), _p(a21i), _p(out[0]), _p(out[1]), _p(cti),
                         _p(out[3]), _p(out[4]), _pi(zp), flags, nthreads)
    return out[0], out[1], cti, out[3], out[4], zp


def _pf(a):
    if a is None:
        return None
    assert a.dtype == _np.float32 and (a.flags.f_contiguous or a.flags.c_contiguous)
    return a.ctypes.data_as(_fp)


def sevd2(a11, a22, a21r, a21i=None, flags=0):
    """Single precision scalar EVD; inputs are rounded to float32 first.
    Returns a dict of float32 outputs."""
    L = lib()
    c, C, S, l1, l2 = (_ct.c_float() for _ in range(5))
    a11, a22, a21r = (_np.float32(x) for x in (a11, a22, a21r))
    if a21i is None:
        z = L.ora_sevd2_real(a11, a22, a21r, c, C, l1, l2, flags)
        S.value = 0.0
    else:
        z = L.ora_sevd2_cplx(a11, a22, a21r, _np.float32(a21i), c, C, S, l1, l2, flags)
    f32 = _np.float32
    return dict(cos=f32(c.value), ctan_re=f32(C.value), ctan_im=f32(S.value), l1=f32(l1.value), l2=f32(l2.value),
                zp=z)


def sevd2_batch(a11, a22, a21r, a21i=None, flags=0, nthreads=0):
    """Single precision batched EVD over float32 SoA arrays."""
    a11, a22, a21r = (_np.ascontiguousarray(x, dtype=_np.float32) for x in (a11, a22, a21r))
    a21i = None if a21i is None else _np.ascontiguousarray(a21i, dtype=_np.float32)
    r = a11.shape[0]
    out = [_np.empty(r, dtype=_np.float32) for _ in range(5)]
    zp = _np.empty(r, dtype=_np.int32)
    cti = out[2] if a21i is not None else None
    lib().ora_sevd2_batch(r, _pf(a11), _pf(a22), _pf(a21r), _pf(a21i), _pf(out[0]), _pf(out[1]), _pf(cti),
                          _pf(out[3]), _pf(out[4]), _pi(zp), flags, nthreads)
    return out[0], out[1], cti, out[3], out[4], zp


def omp_max_threads():
    return lib().ora_omp_max_threads()


def set_step_threads(nthreads):
    """Threads of the oracle step's loops over pairs (1: sequential, the
    default; results do not depend on it)."""
    lib().ora_set_step_threads(int(nthreads))


# ---------------------------------------------------------------- helpers
def hypot(x, y):
    return lib().ora_hypot(x, y)


def lg_bound_m(m, cplx):
    return lib().ora_lg_bound_m(m, int(cplx))


def s_round(Mt, cplx):
    return lib().ora_s_round(Mt, int(cplx))


def s_square(Mt, m, cplx):
    return lib().ora_s_square(Mt, m, int(cplx))


def rr_steps(n):
    return lib().ora_rr_steps(n)


def rr_pair(n, k, l):
    p, q = _ct.c_int(), _ct.c_int()
    ok = lib().ora_rr_pair(n, k, l, p, q)
    return bool(ok), p.value, q.value


def colnorm(xr, xi=None):
    e, f = _ct.c_double(), _ct.c_double()
    xr = _np.ascontiguousarray(xr, dtype=_np.float64)
    xi = None if xi is None else _np.ascontiguousarray(xi, dtype=_np.float64)
    lib().ora_colnorm(xr.shape[0], _p(xr), _p(xi), e, f)
    return e.value, f.value


def dpscl(qr, qi, pr, pi, eq, fq, ep, fp):
    zr, zi = _ct.c_double(), _ct.c_double()
    qr, pr = (_np.ascontiguousarray(a, dtype=_np.float64) for a in (qr, pr))
    qi = None if qi is None else _np.ascontiguousarray(qi, dtype=_np.float64)
    pi = None if pi is None else _np.ascontiguousarray(pi, dtype=_np.float64)
    lib().ora_dpscl(qr.shape[0], _p(qr), _p(qi), _p(pr), _p(pi), eq, fq, ep, fp, zr, zi)
    return zr.value, zi.value


def colnorm_exact(xr, xi=None):
    """The exact mode's column norm: binary128 sum of squares, sqrt, rounded once."""
    e, f = _ct.c_double(), _ct.c_double()
    xr = _np.ascontiguousarray(xr, dtype=_np.float64)
    xi = None if xi is None else _np.ascontiguousarray(xi, dtype=_np.float64)
    lib().ora_colnorm_exact(xr.shape[0], _p(xr), _p(xi), e, f)
    return e.value, f.value


def dpscl_exact(qr, qi, pr, pi, eq, fq, ep, fp):
    """The exact mode's scaled dot-product: binary128 sum rounded once, then / fl(fq fp)."""
    zr, zi = _ct.c_double(), _ct.c_double()
    qr, pr = (_np.ascontiguousarray(a, dtype=_np.float64) for a in (qr, pr))
    qi = None if qi is None else _np.ascontiguousarray(qi, dtype=_np.float64)
    pi = None if pi is None else _np.ascontiguousarray(pi, dtype=_np.float64)
    lib().ora_dpscl_exact(qr.shape[0], _p(qr), _p(qi), _p(pr), _p(pi), eq, fq, ep, fp, zr, zi)
    return zr.value, zi.value


class exact_mode:
    """Context manager: the iteration (State, gesvj) uses the exact mode's
    norms and dot-products inside the block."""

    def __enter__(self):
        self._old = lib().ora_get_exact()
        lib().ora_set_exact(1)
        return self

    def __exit__(self, *exc):
        lib().ora_set_exact(self._old)
        return False


def mul_rd(a, b):
    """RD(a b), the product rounded toward -infinity (Sect. SM2.2, item G.)."""
    return lib().ora_mul_rd(a, b)


def two_sum(a, b):
    """eq. (d2sum): (s, t) with s = fl(a + b) and a + b = s + t."""
    s, t = _ct.c_double(), _ct.c_double()
    lib().ora_2sum(a, b, s, t)
    return s.value, t.value


def dpscl_cs(qr, qi, pr, pi, eq, fq, ep, fp):
    """Alg. zdpsclcs / ddpsclcs: the compensated scaled dot-product."""
    zr, zi = _ct.c_double(), _ct.c_double()
    qr, pr = (_np.ascontiguousarray(a, dtype=_np.float64) for a in (qr, pr))
    qi = None if qi is None else _np.ascontiguousarray(qi, dtype=_np.float64)
    pi = None if pi is None else _np.ascontiguousarray(pi, dtype=_np.float64)
    lib().ora_dpscl_cs(qr.shape[0], _p(qr), _p(qi), _p(pr), _p(pi), eq, fq, ep, fp, zr, zi)
    return zr.value, zi.value


def gram(zr, zi, e1, f1, e2, f2):
    o = [_ct.c_double() for _ in range(4)]
    lib().ora_gram(zr, zi, e1, f1, e2, f2, *o)
    return tuple(x.value for x in o)


def rot(xpr, xpi, xqr, xqi, c, C, S, swap):
    """In-place rotation of a column pair; returns the max-norm."""
    return lib().ora_rot(xpr.shape[0], _p(xpr), _p(xpi), _p(xqr), _p(xqi), c, C, S, int(swap))


def gs_case(e1, f1, e2, f2, ups):
    """eq. (GScond): 1 if ||g_p|| > 2^eta_hat ups ||g_q||, 2 if the reverse, else 0."""
    return lib().ora_gs_case(e1, f1, e2, f2, ups)


def gs(xr, xi, yr, yi, ex, fx, ey, fy, wr, wi):
    """eq. (GS) in place on y (x unchanged); returns the max-norm of the new y."""
    return lib().ora_gs(yr.shape[0], _p(xr), _p(xi), _p(yr), _p(yi), ex, fx, ey, fy, wr, wi)


def s_gs_case(e1, f1, e2, f2, ups):
    return lib().ora_s_gs_case(e1, f1, e2, f2, ups)


def s_gs(xr, xi, yr, yi, ex, fx, ey, fy, wr, wi):
    return lib().ora_s_gs(yr.shape[0], _pf(xr), _pf(xi), _pf(yr), _pf(yi), ex, fx, ey, fy, wr, wi)


# ---------------------------------------------------------------- SVD
class State:
    """Oracle SVD state on host numpy arrays (column-major)."""

    def __init__(self, G_re, G_im=None, permute=False, compensated=False, nogs=False):
        self.permute = bool(permute)
        self.compensated = bool(compensated)
        self.nogs = bool(nogs)
        self.m, self.n = G_re.shape
        self.cplx = G_im is not None
        self.Gr = _np.array(G_re, dtype=_np.float64, order="F", copy=True)
        self.Gi = _np.array(G_im, dtype=_np.float64, order="F", copy=True) if self.cplx else None
        self.Vr = _np.zeros((self.n, self.n), order="F")
        self.Vi = _np.zeros((self.n, self.n), order="F") if self.cplx else None
        self.e = _np.full(self.n, -_np.inf)
        self.f = _np.ones(self.n)
        self.s = 0
        self.Mt = 0.0
        self.k = 0
        self.last_t = 0
        self.last_sw = 0
        self.last_gs = 0
        self.rescaled = 0

    def _args(self):
        return (self.m, self.n, _p(self.Gr), _p(self.Gi), self.m, _p(self.Vr), _p(self.Vi), self.n,
                _p(self.e), _p(self.f))

    def init(self):
        s, Mt = _ct.c_int(), _ct.c_double()
        st = lib().ora_init_ext(*self._args(), s, Mt)
        self.s, self.Mt, self.k = s.value, Mt.value, 0
        return st

    def step(self):
        s, Mt = _ct.c_int(self.s), _ct.c_double(self.Mt)
        t, sw, gs_, r = _ct.c_long(), _ct.c_long(), _ct.c_long(), _ct.c_int()
        flags = ((PERMUTE if self.permute else 0) | (COMPENSATED if self.compensated else 0) |
                 (NO_GS if self.nogs else 0))
        lib().ora_step_ext(*self._args(), s, Mt, self.k, t, sw, gs_, r, flags)
        self.s, self.Mt, self.last_t, self.last_sw = s.value, Mt.value, t.value, sw.value
        self.last_gs = gs_.value
        self.rescaled += r.value
        self.k += 1
        return t.value

    def finalize(self):
        sv_e, sv_f = _np.empty(self.n), _np.empty(self.n)
        lib().ora_finalize_ext(*self._args(), self.s, _p(sv_e), _p(sv_f))
        return sv_e, sv_f


def gesvj(G_re, G_im=None, max_sweeps=128, flags=0):
    """The whole SVD.  Returns dict(status, U_re, U_im, V_re, V_im, sv_e, sv_f, sweeps, steps)."""
    m, n = G_re.shape
    Gr = _np.array(G_re, dtype=_np.float64, order="F", copy=True)
    Gi = _np.array(G_im, dtype=_np.float64, order="F", copy=True) if G_im is not None else None
    Vr = _np.zeros((n, n), order="F")
    Vi = _np.zeros((n, n), order="F") if G_im is not None else None
    sv_e, sv_f = _np.empty(n), _np.empty(n)
    sw, stp = _ct.c_int(), _ct.c_long()
    st = lib().ora_gesvj(m, n, _p(Gr), _p(Gi), m, _p(Vr), _p(Vi), n, _p(sv_e), _p(sv_f),
                         max_sweeps, sw, stp, flags)
    return dict(status=st, U_re=Gr, U_im=Gi, V_re=Vr, V_im=Vi, sv_e=sv_e, sv_f=sv_f,
                sweeps=sw.value, steps=stp.value)


# ---- single precision SVD ----
def s_colnorm(xr, xi=None):
    e, f = _ct.c_float(), _ct.c_float()
    xr = _np.ascontiguousarray(xr, dtype=_np.float32)
    xi = None if xi is None else _np.ascontiguousarray(xi, dtype=_np.float32)
    lib().ora_s_colnorm(xr.shape[0], _pf(xr), _pf(xi), e, f)
    return _np.float32(e.value), _np.float32(f.value)


def s_dpscl(qr, qi, pr, pi, eq, fq, ep, fp):
    zr, zi = _ct.c_float(), _ct.c_float()
    qr, pr = (_np.ascontiguousarray(a, dtype=_np.float32) for a in (qr, pr))
    qi = None if qi is None else _np.ascontiguousarray(qi, dtype=_np.float32)
    pi = None if pi is None else _np.ascontiguousarray(pi, dtype=_np.float32)
    lib().ora_s_dpscl(qr.shape[0], _pf(qr), _pf(qi), _pf(pr), _pf(pi), eq, fq, ep, fp, zr, zi)
    return _np.float32(zr.value), _np.float32(zi.value)


def s_lg_bound_m(m, cplx):
    return lib().ora_s_lg_bound_m(m, int(cplx))


def s_s_round(Mt, cplx):
    return lib().ora_s_s_round(Mt, int(cplx))


def s_s_square(Mt, m, cplx):
    return lib().ora_s_s_square(Mt, m, int(cplx))


class SState:
    """Single precision oracle SVD state on host float32 arrays (column-major)."""

    def __init__(self, G_re, G_im=None, permute=False, nogs=False):
        self.permute = bool(permute)
        self.nogs = bool(nogs)
        self.m, self.n = G_re.shape
        self.cplx = G_im is not None
        self.Gr = _np.array(G_re, dtype=_np.float32, order="F", copy=True)
        self.Gi = _np.array(G_im, dtype=_np.float32, order="F", copy=True) if self.cplx else None
        self.Vr = _np.zeros((self.n, self.n), dtype=_np.float32, order="F")
        self.Vi = _np.zeros((self.n, self.n), dtype=_np.float32, order="F") if self.cplx else None
        self.e = _np.full(self.n, -_np.inf, dtype=_np.float32)
        self.f = _np.ones(self.n, dtype=_np.float32)
        self.s = 0
        self.Mt = _np.float32(0)
        self.k = 0
        self.last_t = 0
        self.last_sw = 0
        self.last_gs = 0
        self.rescaled = 0

    def _args(self):
        return (self.m, self.n, _pf(self.Gr), _pf(self.Gi), self.m, _pf(self.Vr), _pf(self.Vi), self.n,
                _pf(self.e), _pf(self.f))

    def init(self):
        s, Mt = _ct.c_int(), _ct.c_float()
        st = lib().ora_s_init_ext(*self._args(), s, Mt)
        self.s, self.Mt, self.k = s.value, _np.float32(Mt.value), 0
        return st

    def step(self):
        s, Mt = _ct.c_int(self.s), _ct.c_float(self.Mt)
        t, sw, gs_, r = _ct.c_long(), _ct.c_long(), _ct.c_long(), _ct.c_int()
        flags = (PERMUTE if self.permute else 0) | (NO_GS if self.nogs else 0)
        lib().ora_s_step_ext(*self._args(), s, Mt, self.k, t, sw, gs_, r, flags)
        self.s, self.Mt, self.last_t, self.last_sw = s.value, _np.float32(Mt.value), t.value, sw.value
        self.last_gs = gs_.value
        self.rescaled += r.value
        self.k += 1
        return t.value


def sgesvj(G_re, G_im=None, max_sweeps=128, flags=0):
    """The single precision SVD.  Returns dict(status, U_re, U_im, V_re, V_im, sv_e, sv_f, sweeps, steps)
    with float32 arrays."""
    m, n = G_re.shape
    Gr = _np.array(G_re, dtype=_np.float32, order="F", copy=True)
    Gi = _np.array(G_im, dtype=_np.float32, order="F", copy=True) if G_im is not None else None
    Vr = _np.zeros((n, n), dtype=_np.float32, order="F")
    Vi = _np.zeros((n, n), dtype=_np.float32, order="F") if G_im is not None else None
    sv_e, sv_f = _np.empty(n, dtype=_np.float32), _np.empty(n, dtype=_np.float32)
    sw, stp = _ct.c_int(), _ct.c_long()
    st = lib().ora_sgesvj(m, n, _pf(Gr), _pf(Gi), m, _pf(Vr), _pf(Vi), n, _pf(sv_e), _pf(sv_f),
                          max_sweeps, sw, stp, flags)
    return dict(status=st, U_re=Gr, U_im=Gi, V_re=Vr, V_im=Vi, sv_e=sv_e, sv_f=sv_f,
                sweeps=sw.value, steps=stp.value)


def sv_values(sv_e, sv_f):
    """sigma_j = 2^e_j f_j as float64 (may overflow or underflow)."""
    return _np.ldexp(sv_f, _np.where(_np.isinf(sv_e), -2000, sv_e).astype(_np.int64))


# ---------------------------------------------------------------- Alg. rnF
def nrmf(xr, xi=None, lanes=1024):
    """Alg. rnF with `lanes` lanes: dict(e2, f2, e, f) with ||x||^2 = 2^e2 f2 and
    ||x|| = 2^e f (integral e as floats, -inf for a zero array)."""
    xr = _np.ascontiguousarray(xr, dtype=_np.float64)
    xi = None if xi is None else _np.ascontiguousarray(xi, dtype=_np.float64)
    o = [_ct.c_double() for _ in range(4)]
    st = lib().ora_nrmf(xr.shape[0], _p(xr), _p(xi), lanes, *o)
    if st != OK:
        raise ValueError("ora_nrmf: invalid arguments")
    return dict(e2=o[0].value, f2=o[1].value, e=o[2].value, f=o[3].value)


def nrmf_lanes(xr, xi=None, lanes=1024):
    """The unsorted lane partial sums (e, f) of ||x||^2 of Alg. rnF."""
    xr = _np.ascontiguousarray(xr, dtype=_np.float64)
    xi = None if xi is None else _np.ascontiguousarray(xi, dtype=_np.float64)
    le, lf = _np.empty(lanes), _np.empty(lanes)
    if lib().ora_nrmf_lanes(xr.shape[0], _p(xr), _p(xi), lanes, _p(le), _p(lf)) != OK:
        raise ValueError("ora_nrmf_lanes: invalid arguments")
    return le, lf
