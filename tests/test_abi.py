"""The C-ABI library loads and exports every function include/jsvd.h declares
(no device call is made: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jsvd.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char\s*\*)\s*(jsvd_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def _lib():
    import paper_2202_08361_amd as J
    if not os.path.exists(J.LIB_PATH):
        from paper_2202_08361_amd import build
        build.build()
    return ctypes.CDLL(J.LIB_PATH)


def test_header_parses():
    names = _declared()
    for must in ("jsvd_evd2_batched", "jsvd_step", "jsvd_gesvj", "jsvd_gesvj_batched", "jsvd_serve_create",
                 "jsvd_serve_submit", "jsvd_serve_wait", "jsvd_serve_stats_get", "jsvd_state_create"):
        assert must in names
    assert len(names) >= 23


def test_exports_every_declared_symbol():
    L = _lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_host_only_calls():
    """Calls that touch no device: version, error strings, argument validation."""
    import paper_2202_08361_amd as J
    L = J.lib()
    assert L.jsvd_version() == (0 << 16) | 1
    assert L.jsvd_strerror(0) == b"ok"
    assert L.jsvd_strerror(-3) == b"input is the zero matrix"
    h = ctypes.c_void_p()
    assert L.jsvd_state_create(3, 5, 0, ctypes.byref(h)) == J.EINVAL      # m < n
    assert L.jsvd_state_create(5, 0, 0, ctypes.byref(h)) == J.EINVAL      # n < 1
    assert L.jsvd_state_create((1 << 24) + 1, 5, 1, ctypes.byref(h)) == J.EINVAL  # beyond 2^24 rows
    assert L.jsvd_evd2_batched(10, None, None, None, None, None, None, None, None, None, None, 0, None) == J.EINVAL
    assert L.jsvd_gesvj(3, 4, None, None, 3, None, None, 4, None, None, None, 0, None, 0, None) == J.EINVAL
    assert L.jsvd_state_create_f32(3, 5, 0, ctypes.byref(h)) == J.EINVAL  # m < n
    assert L.jsvd_state_create_f32((1 << 24) + 1, 5, 0, ctypes.byref(h)) == J.EINVAL
    assert L.jsvd_gesvj_f32(3, 4, None, None, 3, None, None, 4, None, None, None, 0, None, 0, None) == J.EINVAL
    # the compensated dot-products are double precision only (rejected before any device call)
    p = ctypes.c_void_p(256)
    assert L.jsvd_gesvj_f32(8, 4, p, None, 8, p, None, 4, p, p, None, 0, None, J.COMPENSATED, None) == J.EINVAL
    # the persistent sweep's settings need a state
    L.jsvd_state_set_loop_local.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.jsvd_state_set_loop_wait.argtypes = [ctypes.c_void_p, ctypes.c_double]
    assert L.jsvd_state_set_loop_local(None, 1) == J.EINVAL
    assert L.jsvd_state_set_loop_wait(None, 0.25) == J.EINVAL


def test_no_oracle_in_product():
    """The product package never imports or links the oracle."""
    pkg = os.path.join(ROOT, "paper_2202_08361_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "liboracle" not in txt, f
