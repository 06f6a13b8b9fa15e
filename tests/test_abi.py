"""The C-ABI library loads and exports every entry point declared in include/hsf.h
(no compute calls: no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hsf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hsf_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for name in ["hsf_create", "hsf_evaluate", "hsf_invert", "hsf_step", "hsf_set_fields"]:
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_1204_2088_amd import hsf
    path = hsf.library_path()
    if not os.path.exists(path):
        pytest.fail(f"{path} not built (run python -m paper_1204_2088_amd.build)")
    lib = ctypes.CDLL(path)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(declared_symbols()) == sorted(hsf.EXPORTED)


def test_binding_loads_without_gpu_calls():
    from paper_1204_2088_amd import hsf
    lib = hsf.load()
    assert lib.hsf_total_sites(None) == -1
    assert lib.hsf_num_species(None) == -1
    assert lib.hsf_last_error(None) == b"null context"


def test_create_rejects_bad_parameters_without_gpu():
    """Parameter validation happens before any device call."""
    from paper_1204_2088_amd import hsf, workloads as W
    lib = hsf.load()
    wl = W.melt16_a4b4()
    p = hsf.params_from_workload(wl)
    p.tau = 0.4  # must exceed 1/2
    h = ctypes.c_void_p()
    assert lib.hsf_create(ctypes.byref(p), 1, ctypes.byref(h)) == hsf.HSF_EINVAL
    p = hsf.params_from_workload(wl)
    p.n_beads = 0
    assert lib.hsf_create(ctypes.byref(p), 1, ctypes.byref(h)) == hsf.HSF_EINVAL
    arr = (hsf.Params * 2)(hsf.params_from_workload(wl), hsf.params_from_workload(wl, precision="fp32"))
    assert lib.hsf_create(arr, 2, ctypes.byref(h)) == hsf.HSF_EINVAL
    assert lib.hsf_create(arr, 0, ctypes.byref(h)) == hsf.HSF_EINVAL
    # a box above the 32-bit site limit (1291^3 > 2^31 - 1), and one whose edge product
    # overflows 32 bits outright
    for L in ((1291, 1291, 1291), (65536, 65536, 2)):
        p = hsf.params_from_workload(wl)
        p.Lx, p.Ly, p.Lz = L
        assert lib.hsf_create(ctypes.byref(p), 1, ctypes.byref(h)) == hsf.HSF_EINVAL, L
        assert not h.value
    p = hsf.params_from_workload(wl)
    p.Lx = 0
    assert lib.hsf_create(ctypes.byref(p), 1, ctypes.byref(h)) == hsf.HSF_EINVAL


def test_param_structs_match_header(tmp_path):
    """The ctypes structures of the binding have the sizes and field offsets of the
    C declarations (compiled from include/hsf.h with the host C compiler)."""
    import ctypes
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no host C compiler")
    from paper_1204_2088_amd import hsf
    structs = {"hsf_params": hsf.Params, "hsf_invert_stats": hsf.InvertStats, "hsf_cn_stats": hsf.CnStats,
               "hsf_step_record": hsf.StepRecord}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hsf.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([gcc, "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln.strip():
            parts = ln.split()
            got[tuple(parts[:-1])] = int(parts[-1])
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
