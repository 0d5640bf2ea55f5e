"""Host-side checks that need no GPU: the library loads and exports the header's symbols."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "montexp.h")
LIB = os.path.join(ROOT, "paper_2410_18129_amd", "libmontexp.so")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", src)) - {"if", "sizeof"})


def test_header_declares_the_boundary():
    fns = header_functions()
    for f in ("mont_ctx_init", "mont_ctx_query", "mont_ctx_export", "mont_ctx_destroy", "mont_mul_batch",
              "mont_sqr_batch", "modexp_batch", "mont_last_error"):
        assert f in fns


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmontexp.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    for f in header_functions():
        assert hasattr(L, f), f
    from paper_2410_18129_amd import montexp
    assert set(montexp.EXPORTS) == set(header_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmontexp.so not built")
def test_host_side_argument_errors_without_gpu():
    """Argument checks return MX_EINVAL before touching a device."""
    from paper_2410_18129_amd import montexp as mx
    L = mx.lib()
    h = ctypes.c_void_p()
    import numpy as np
    even = np.array([[4]], dtype=np.uint64)
    assert L.mont_ctx_init(ctypes.byref(h), even.ctypes.data_as(ctypes.c_void_p), 64, 1, None) == mx.MX_EINVAL
    assert b"even" in L.mont_last_error()
    one = np.array([[1]], dtype=np.uint64)
    assert L.mont_ctx_init(ctypes.byref(h), one.ctypes.data_as(ctypes.c_void_p), 64, 1, None) == mx.MX_EINVAL
    odd = np.array([[7]], dtype=np.uint64)
    assert L.mont_ctx_init(ctypes.byref(h), odd.ctypes.data_as(ctypes.c_void_p), 96, 1, None) == mx.MX_EINVAL
    assert b"size class" in L.mont_last_error()
    assert L.mont_ctx_init(ctypes.byref(h), odd.ctypes.data_as(ctypes.c_void_p), 64, 0, None) == mx.MX_EINVAL
    assert L.mont_mul_batch(None, None, None, None, None, 1, 0, None) == mx.MX_EINVAL
    assert L.modexp_batch(None, None, None, None, 8, 5, None, 1, 0, None) == mx.MX_EINVAL
    assert L.rsa_crt_batch(None, None, None, None, None, None, None, 0, None, 1, 0, None) == mx.MX_EINVAL
    # raw products: methods, sizes and the workspace are checked before any launch
    nb = ctypes.c_size_t()
    assert L.mp_mul_ws_bytes(4108, 64, 0, ctypes.byref(nb)) == mx.MX_OK and nb.value > 0
    assert L.mp_mul_ws_bytes(4257, 64, 0, ctypes.byref(nb)) == mx.MX_EUNSUPPORTED
    assert L.mp_mul_ws_bytes(4108, 64, 3, ctypes.byref(nb)) == mx.MX_EINVAL
    assert L.mp_mul_batch(None, None, None, 4108, 1, 0, None, 0, None) == mx.MX_EINVAL
    assert L.mp_mul_batch(None, None, None, 4108, 0, 0, None, 0, None) == mx.MX_OK  # n = 0


def test_header_constants_match_the_binding():
    """Status codes and flags have the same values in include/montexp.h and the Python binding."""
    from paper_2410_18129_amd import montexp
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    vals = dict((k, int(v)) for k, v in re.findall(r"\b(MX_[A-Z0-9_]+)\s*=\s*(\d+)", src))
    for name in ("MX_OK", "MX_EINVAL", "MX_ENOMEM", "MX_EDEVICE", "MX_EUNSUPPORTED", "MX_REDC_TRUNC",
                 "MX_REDC_PLAIN", "MX_IMPL_BLOCK", "MX_MUL_KARATSUBA", "MX_ONE_LANE", "MX_REDC_CIOS", "MX_TWO_LANES",
                 "MX_REDC_KARATSUBA", "MX_MUL_KARATSUBA2", "MX_CHECK_INPUTS", "MX_FOUR_LANES"):
        assert vals[name] == getattr(montexp, name), name
    flags = [vals[k] for k in ("MX_REDC_PLAIN", "MX_IMPL_BLOCK", "MX_MUL_KARATSUBA", "MX_ONE_LANE", "MX_REDC_CIOS",
                               "MX_TWO_LANES", "MX_REDC_KARATSUBA", "MX_MUL_KARATSUBA2", "MX_CHECK_INPUTS",
                               "MX_FOUR_LANES")]
    assert all(f & (f - 1) == 0 for f in flags) and len(set(flags)) == len(flags)


def test_work_counts_match_the_model():
    """The bench's product counts per operation equal the oracle model's (all three reductions)."""
    from oracle import montred_model as m
    from paper_2410_18129_amd import counts
    for n in (3, 37, 74):
        c = m.counts(n)
        assert counts.op_products(n, trunc=True) == {"mul": c["mul_trunc"], "sqr": c["sqr_trunc"]}
        assert counts.op_products(n, trunc=False) == {"mul": c["mul_plain"], "sqr": c["sqr_plain"]}
        assert counts.op_products(n, cios=True) == {"mul": c["mul_cios"], "sqr": c["sqr_cios"]}
