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


def header_enums():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return {k: int(v) for k, v in re.findall(r"\b(SISDC_[A-Z0-9_]+)\s*=\s*(-?\d+)", text)}


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsisdc.so not built")
def test_binding_constants_match_header_enums():
    from paper_2504_18526_amd import sisdc as S
    enums = header_enums()
    checked = 0
    for name, value in enums.items():
        short = name[len("SISDC_"):]
        if hasattr(S, short):
            assert getattr(S, short) == value, name
            checked += 1
    for short in ("OP_QUAD", "PROJ_L2", "NODES_LOBATTO", "NONINCREMENTAL", "IMEX_EULER", "CG_PERSISTENT_COOPERATIVE"):
        assert "SISDC_" + short in enums and getattr(S, short) == enums["SISDC_" + short]
    assert checked > 20


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """The ctypes mirrors of sisdc_problem / sisdc_method / sisdc_stats have
    the sizes and field offsets that gcc gives the header's structs."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    from paper_2504_18526_amd import sisdc as S
    structs = {"sisdc_problem": S.Problem, "sisdc_method": S.Method, "sisdc_stats": S.Stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sisdc.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        cname, field, value = line.split()
        py = structs[cname]
        if field == "size":
            assert ctypes.sizeof(py) == int(value), cname
        else:
            assert getattr(py, field).offset == int(value), (cname, field)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsisdc.so not built")
def test_method_options_validated_without_gpu_work():
    from paper_2504_18526_amd import sisdc as S
    lib = S.lib()
    h = ctypes.c_void_p()
    prob = S.make_problem(2, (3, 4), (0, 0), (1, 1), S.EQ_CONVDIFF, nu=0.01)
    cases = [
        (S.make_method([4, 2], [3, 1], nodes=S.NODES_LOBATTO), b"Lobatto"),
        (S.make_method([4, 2], [3, 2], h_coarsen=[0, 1]), b"even"),
        (S.make_method([4, 2], [3, 2], h_coarsen=[1, 0]), b"h_coarsen[0]"),
        (S.make_method([4], [3], projection=7), b"projection"),
        (S.make_method([4], [3], formulation=5), b"formulation"),
        (S.make_method([4], [3], integrator=9), b"integrator"),
    ]
    for meth, msg in cases:
        rc = lib.sisdc_create(ctypes.byref(prob), ctypes.byref(meth), None, ctypes.byref(h))
        assert rc == S.EINVAL, msg
        assert msg in lib.sisdc_last_error(), (msg, lib.sisdc_last_error())
