"""CPU checks of the C ABI library: it loads, exports every declared entry
point, and rejects bad arguments before touching the device."""
import ctypes as C
import os

import pytest

from paper_2010_03817_amd import spec as S


def test_library_exports_every_declared_symbol():
    if not os.path.exists(S.LIB_PATH):
        pytest.fail("libspec.so not built (python -m paper_2010_03817_amd.build)")
    names = S.declared_symbols()
    assert "spec_create" in names and "spec_intersect_dev" in names and "spec_reflect" in names
    lib = C.CDLL(S.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_argument_errors():
    L = S.lib()
    assert L.spec_status_str(S.OK).decode() == "ok"
    assert "interior" in L.spec_status_str(S.NOT_INTERIOR).decode()
    h = C.c_void_p()
    one = (C.c_int * 1)(3)
    kind = (C.c_int * 1)(S.DENSE)
    A = (C.c_double * 9)()
    # n < 1 and NULL handle are argument errors, checked before any device call
    assert L.spec_create(0, 1, one, kind, A, C.byref(h)) == S.EINVAL
    assert L.spec_create(1, 1, one, kind, A, None) == S.EINVAL
    bad = (C.c_int * 1)(7)
    assert L.spec_create(1, 1, one, bad, A, C.byref(h)) == S.EINVAL
    assert L.spec_destroy(None) == S.EINVAL
    assert L.spec_intersect(None, 1, None, None, None, None, None) == S.EINVAL
    # host walk and host training: NULL handle / arrays are argument errors
    p = S.WalkParams(tau=1.0)
    st = S.WalkStats()
    assert L.spec_walk_run(None, S.BILLIARD, 4, None, 10, 1, C.byref(p), None, None, C.byref(st)) == S.EINVAL
    tp = S.MlpTrainParams()
    ts = S.MlpTrainStats()
    assert L.spec_mlp_train(None, 10, None, None, None, None, C.byref(tp), C.byref(ts)) == S.EINVAL
    o = S.Options()
    assert L.spec_options_default(C.byref(o)) == S.OK
    assert o.kmax == 80 and o.tol == 1e-8 and o.refine_ratio == 1e3 and o.tol_loose == 1e-3
    assert o.certify == 0 and o.escalate_ratio == 1e-3 and o.refresh_period == 16
    assert C.sizeof(S.Options) == 56  # the struct of include/spec.h (8 fields and padding)
    d = C.c_double()
    assert L.spec_diag_assembly_rows(None, C.byref(d)) == S.EINVAL
    assert L.spec_set_options(None, C.byref(o)) == S.EINVAL
    assert L.spec_walk_state(None, 0) == S.EINVAL


def test_non_symmetric_block_rejected():
    L = S.lib()
    h = C.c_void_p()
    one = (C.c_int * 1)(2)
    kind = (C.c_int * 1)(S.DENSE)
    # n = 1: A0 = I, A1 = [[0, 1], [0, 0]] (not symmetric)
    A = (C.c_double * 8)(1, 0, 0, 1, 0, 1, 0, 0)
    assert L.spec_create(1, 1, one, kind, A, C.byref(h)) == S.EINVAL
