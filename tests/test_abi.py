"""CPU-side checks of the C ABI: the library loads, exports every function
that include/spoch.h declares, and rejects invalid arguments before it
touches a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "spoch.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ch_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def binding():
    from paper_2412_18008_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libspoch.so not built")
    binding.lib()
    return binding


def test_exports_every_declared_symbol(binding):
    names = declared_functions()
    assert set(names) == set(binding.EXPORTED)
    L = C.CDLL(binding.LIB_PATH)
    for f in names:
        assert hasattr(L, f), f


def test_version(binding):
    assert binding.version().startswith("spoch-gfx950")


def test_null_and_invalid_arguments(binding):
    L = binding.lib()
    h = C.c_void_p()
    assert L.ch_build(None, None, C.byref(h)) == binding.CH_E_INVALID
    assert "NULL" in L.ch_last_error().decode()
    off = np.zeros(2, np.uint64)
    g = binding.Graph(1, 0, off.ctypes.data, None, None, None)
    assert L.ch_build(C.byref(g), None, None) == binding.CH_E_INVALID
    p = binding.Params(0, 0, 0, 0, 3, None, 0, 0, 0, 0, None)  # group 3 is not allowed
    assert L.ch_build(C.byref(g), C.byref(p), C.byref(h)) == binding.CH_E_INVALID
    p = binding.Params(7, 0, 0, 0, 0, None, 0, 0, 0, 0, None)  # unknown search mode
    assert L.ch_build(C.byref(g), C.byref(p), C.byref(h)) == binding.CH_E_UNSUPPORTED
    p = binding.Params(0, 0, 0, 0, 0, None, 9, 0, 0, 0, None)  # unknown search kernel
    assert L.ch_build(C.byref(g), C.byref(p), C.byref(h)) == binding.CH_E_INVALID
    p = binding.Params(0, 0, 0, 0, 0, None, 0, 0, 0, 1, None)  # learned without weights
    assert L.ch_build(C.byref(g), C.byref(p), C.byref(h)) == binding.CH_E_INVALID
    p = binding.Params(7, 0, 0, 0, 0, None, 0, 0, 0, 0, None)
    assert L.ch_build(C.byref(g), C.byref(p), C.byref(h)) == binding.CH_E_UNSUPPORTED
    p = binding.Params(tiebreak=2)  # unknown tie-break
    assert L.ch_build(C.byref(g), C.byref(p), C.byref(h)) == binding.CH_E_INVALID
    p = binding.Params(ls_step=33)  # bucket shift above 32
    assert L.ch_build(C.byref(g), C.byref(p), C.byref(h)) == binding.CH_E_INVALID
    assert "ls_step" in L.ch_last_error().decode()
    lab = np.zeros(1, np.uint32)
    gl = binding.Graph(1, 0, off.ctypes.data, None, None, lab.ctypes.data)
    p = binding.Params(tiebreak=binding.CH_TIE_RAW_ID)  # raw ids and labels together
    assert L.ch_build(C.byref(gl), C.byref(p), C.byref(h)) == binding.CH_E_INVALID
    assert "RAW_ID" in L.ch_last_error().decode()
    assert L.ch_build_batch(C.byref(gl), 1, C.byref(p), C.byref(h)) == binding.CH_E_INVALID
    g = binding.Graph(0xFFFFFFFF, 0, off.ctypes.data, None, None, None)
    assert L.ch_build(C.byref(g), None, C.byref(h)) == binding.CH_E_INVALID
    assert L.ch_query_batch(None, None, None, 0, None, 0, None) == binding.CH_E_INVALID
    assert L.ch_get_summary(None, None) == binding.CH_E_INVALID
    L.ch_free(None)


def test_struct_layouts_match_header(binding, tmp_path):
    """ctypes mirrors of the ABI structs have the sizes and field offsets
    that a C compiler gives the header's definitions."""
    import subprocess

    structs = {"ch_graph_t": binding.Graph, "ch_params_t": binding.Params,
               "ch_query_stats_t": binding.QueryStats,
               "ch_summary_t": binding.Summary, "ch_round_stats_t": binding.RoundStats,
               "ch_mlp_train_params_t": binding.MlpTrainParams}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "spoch.h"', 'int main(void){']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().split("\n") if l)
    for cname, py in structs.items():
        assert int(out[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_header_constants_match_binding(binding):
    """Every plain numeric #define of the header that the binding mirrors
    has the same value there."""
    import re

    text = open(os.path.join(ROOT, "include", "spoch.h")).read()
    found = 0
    for name, val in re.findall(r"^#define\s+(CH_\w+)\s+(0x[0-9A-Fa-f]+|\d+)u?\b", text, re.M):
        if hasattr(binding, name):
            assert getattr(binding, name) == int(val, 0), name
            found += 1
    for name in ("CH_F_TAIL_STEPWISE", "CH_F_KEEP_ORDER", "CH_LS_TABLE", "CH_LS_TAIL",
                 "CH_F_STATS", "CH_DENSE_TAIL_OFF"):
        assert hasattr(binding, name), name
    assert found >= 10
