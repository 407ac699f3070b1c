"""CPU checks of the C ABI: the library loads and exports every function
that include/sisdc.h declares (no compute call: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sisdc.h")
LIB = os.path.join(ROOT, "paper_2504_18526_amd", "libsisdc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\*?\s*([a-z_][a-z_0-9]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_boundary():
    names = declared_functions()
    for n in ("sisdc_create", "sisdc_sweep", "sisdc_step", "mlsdc_vcycle", "helmholtz_solve"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsisdc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsisdc.so not built")
def test_binding_lists_match_header():
    from paper_2504_18526_amd import sisdc as S
    assert sorted(S.EXPORTS) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsisdc.so not built")
def test_invalid_arguments_rejected_without_gpu_work():
    from paper_2504_18526_amd import sisdc as S
    lib = S.lib()
    bad = S.make_problem(4, (2, 2, 2), (0, 0, 0), (1, 1, 1), S.EQ_CONVDIFF)
    meth = S.make_method([4], [3])
    h = ctypes.c_void_p()
    rc = lib.sisdc_create(ctypes.byref(bad), ctypes.byref(meth), None, ctypes.byref(h))
    assert rc == S.EINVAL
    assert b"dim" in lib.sisdc_last_error()
    good = S.make_problem(2, (2, 2), (0, 0), (1, 1), S.EQ_CONVDIFF)
    badm = S.make_method([9], [3])
    rc = lib.sisdc_create(ctypes.byref(good), ctypes.byref(badm), None, ctypes.byref(h))
    assert rc == S.EINVAL
