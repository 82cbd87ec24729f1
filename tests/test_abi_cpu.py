"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2110_07131_amd import rkmips

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    with open(os.path.join(ROOT, "include", "rkmips.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rk_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert header_functions() == sorted(rkmips.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = rkmips.lib()
    for name in header_functions():
        assert hasattr(lib, name), name


STRUCTS = (("rk_build_opts", rkmips.BuildOpts), ("rk_stats", rkmips.Stats),
           ("rk_server_opts", rkmips.ServerOpts), ("rk_completion", rkmips.Completion))


def test_struct_layouts_match_the_c_compiler(tmp_path):
    # sizeof/offsetof as gcc lays out the header's structs vs the ctypes mirror
    lines = []
    for cname, py in STRUCTS:
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"rkmips.h\"\n"
                   "int main(void){" + "".join(lines) + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    for cname, py in STRUCTS:
        assert int(out[cname]) == ctypes.sizeof(py)
        for f, _ in py._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(py, f).offset, f


def test_default_opts():
    o = rkmips.build_opts()
    assert (o.precision, o.lb_items, o.block_size, o.device, o.cand_cap, o.auto_rebuild) == (0, 0, 0, 0, 0, 0)
    assert o.margin_rel == 0.0


@pytest.mark.parametrize("kw,args", [
    ({}, dict(n=-1)), ({}, dict(d=0)), ({}, dict(d=513)), ({}, dict(k_max=0)),
    ({}, dict(k_max=129)), ({"precision": 7}, {}), ({"lb_items": -2}, {}),
    ({"margin_rel": -1.0}, {}), ({"margin_rel": float("nan")}, {}), ({"cand_cap": -1}, {}),
])
def test_build_rejects_bad_arguments_before_device(kw, args):
    L = rkmips.lib()
    n, m, d, k_max = args.get("n", 4), args.get("m", 3), args.get("d", 2), args.get("k_max", 2)
    Q = np.ones((4, 2), np.float32)
    P = np.ones((3, 2), np.float32)
    o = rkmips.build_opts()
    for key, v in kw.items():
        setattr(o, key, v)
    h = ctypes.c_void_p()
    st = L.rk_build_index(Q.ctypes.data, n, P.ctypes.data, m, d, k_max, ctypes.byref(o), ctypes.byref(h))
    assert st == rkmips.RK_E_INVAL
    assert h.value is None
    assert len(L.rk_last_error()) > 0


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf, 2.0 ** 40, -3.0e12])
def test_build_rejects_bad_values(bad):
    L = rkmips.lib()
    Q = np.ones((4, 2), np.float32)
    Q[2, 1] = bad
    P = np.ones((3, 2), np.float32)
    h = ctypes.c_void_p()
    st = L.rk_build_index(Q.ctypes.data, 4, P.ctypes.data, 3, 2, 2, None, ctypes.byref(h))
    assert st == rkmips.RK_E_INVAL and h.value is None


def test_null_pointers_rejected():
    L = rkmips.lib()
    h = ctypes.c_void_p()
    assert L.rk_build_index(None, 4, None, 3, 2, 2, None, ctypes.byref(h)) == rkmips.RK_E_INVAL
    assert L.rk_build_index(None, 0, None, 0, 2, 2, None, None) == rkmips.RK_E_INVAL
    cnt = ctypes.c_int64()
    assert L.rk_reverse_kmips(None, None, 1, None, 0, ctypes.byref(cnt)) == rkmips.RK_E_INVAL
    assert L.rk_index_stats(None, None) == rkmips.RK_E_INVAL
    assert L.rk_index_export(None, 0, None, 0) == rkmips.RK_E_INVAL
    assert L.rk_index_rebuild(None, 3) == rkmips.RK_E_INVAL
    L.rk_index_free(None)


def test_footprint_model():
    n, m, d, kmax = 100_000, 20_000, 50, 25
    fp32 = rkmips.index_footprint(n, m, d, kmax)
    bf16 = rkmips.index_footprint(n, m, d, kmax, precision="bf16")
    # dominant arrays: users tiled + row-major (2 n d 4), items tiled + row-major
    # (2 m d 4), bound tables L64 + L32 (kmax n 12)
    core = 2 * n * d * 4 + 2 * m * d * 4 + kmax * n * 12
    assert core < fp32 < 1.25 * core
    assert bf16 - fp32 >= (n + m) * 64 * 2  # bf16 copies, d padded to 64
    assert rkmips.index_footprint(-1, 1, 1, 1) == -1
