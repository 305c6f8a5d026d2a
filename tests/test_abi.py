"""The C-ABI library loads and exports every function include/gba.h declares
(no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

from paper_2509_26581_amd import gba

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gba.h")


def _ensure_built():
    if not os.path.exists(gba.LIB_PATH):
        from paper_2509_26581_amd import build
        build.build()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(gba_[a-z_]+)\s*\(", text))
    return sorted(n for n in names if n not in ("gba_alloc_fn", "gba_free_fn"))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ["gba_create", "gba_add_cameras", "gba_add_points", "gba_add_edges",
                     "gba_set_robust_kernel", "gba_solve", "gba_get_cost",
                     "gba_get_cameras", "gba_get_points", "gba_destroy"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    _ensure_built()
    lib = ctypes.CDLL(gba.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(gba.exported_symbols()) == _declared_functions()


def test_binding_loads_and_default_options():
    _ensure_built()
    gba.load()
    o = gba.gba_default_options()
    assert o.initial_lambda == 1e-4 and o.min_diag == 1e-6 and o.max_diag == 1e32
    assert o.pcg_max_iters == 100 and o.pcg_tol == 1e-6 and o.pcg_tol_relative == 1
    assert o.precond == gba.GBA_PRECOND_BLOCK_JACOBI


def test_struct_layouts_match_the_header(tmp_path):
    """ctypes field offsets equal those the C compiler gives for gba.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"gba_options": gba.gba_options, "gba_report": gba.gba_report,
               "gba_trial": gba.gba_trial, "gba_problem": gba.gba_problem,
               "gba_result": gba.gba_result, "gba_server_config": gba.gba_server_config,
               "gba_serving_stats": gba.gba_serving_stats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gba.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            cf = "lambda" if fname == "lambda_" else fname
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {cf}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.strip().splitlines():
        cname, field, val = line.split()
        py = structs[cname]
        got = ctypes.sizeof(py) if field == "sizeof" else getattr(py, field).offset
        assert got == int(val), (cname, field, got, val)


def test_missing_library_fails_loudly(tmp_path):
    saved = gba._lib
    try:
        gba._lib = None
        with pytest.raises(gba.GbaError):
            gba.load(str(tmp_path / "absent.so"))
    finally:
        gba._lib = saved


def test_create_without_a_gpu_returns_an_error_code():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    _ensure_built()
    with pytest.raises(gba.GbaError) as ei:
        gba.gba_create(gba.GBA_FP64, 0)
    assert ei.value.status == -6


def test_server_default_config_and_create_without_a_gpu():
    _ensure_built()
    c = gba.gba_server_default_config()
    assert c.precision == gba.GBA_MIXED_FP32
    assert c.max_slots == 64 and c.hbm_budget_bytes == 4 << 30
    assert c.loss == gba.GBA_LOSS_HUBER and c.delta == 1.0
    assert c.options.pcg_max_iters == 100
    import torch
    if torch.cuda.is_available():
        return
    with pytest.raises(gba.GbaError) as ei:
        gba.gba_server_create(c)
    assert ei.value.status == -6
