"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/gf.h declares, validates arguments on the host, and refuses to run
without a GPU (no compute call is made here)."""
import ctypes as C
import os
import re

import pytest

import paper_1209_4008_amd as gf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "gf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gf_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound():
    names = declared_symbols()
    assert len(names) >= 20
    L = gf.lib()
    for n in names:
        assert hasattr(L, n), n
        assert n in gf.SIGNATURES, f"{n} has no binding"
    assert set(gf.SIGNATURES) == set(names)


def test_version_and_host_selftest():
    assert b"gfx950" in gf.lib().gf_version()
    assert gf.lib().gf_selftest_host() == gf.OK


def test_geometry_validation_and_sizes():
    g = gf.Geom.make((8, 8, 8, 8), gf.FP64, gf.R18)
    assert gf.check_geom(g) == gf.OK
    assert gf.field_bytes(g) == 4 * 8 ** 4 * 18 * 8
    assert gf.field_bytes(gf.Geom.make((32, 32, 32, 32), gf.FP32, gf.R12)) == 4 * 32 ** 4 * 12 * 4
    assert gf.field_bytes(gf.Geom.make((48,) * 4, gf.FP64, gf.R12)) == 4 * 48 ** 4 * 12 * 8
    # V/2 is padded to whole tiles of 2048 sites: 6x4x2x10 has 240 sites per
    # parity, 10x8x10x14 5600 (two tiles and a ragged third)
    assert gf.field_bytes(gf.Geom.make((6, 4, 2, 10), gf.FP32, gf.R18)) == 8 * 2048 * 18 * 4
    assert gf.field_bytes(gf.Geom.make((2, 2, 2, 2), gf.FP64, gf.R12)) == 8 * 2048 * 12 * 8
    assert gf.field_bytes(gf.Geom.make((10, 8, 10, 14), gf.FP64, gf.R12)) == 8 * 6144 * 12 * 8
    # the largest accepted volume, 2^30 sites: sizes computed without overflow
    big = gf.Geom.make((256, 256, 128, 128), gf.FP64, gf.R18)
    assert gf.check_geom(big) == gf.OK
    assert gf.field_bytes(big) == 4 * 2 ** 30 * 18 * 8
    assert gf.check_geom(gf.Geom.make((256, 256, 128, 130))) == gf.ERR_ARG
    for bad in [gf.Geom.make((7, 8, 8, 8)), gf.Geom.make((8, 8, 8, 0)),
                gf.Geom.make((8, 8, 8, 8), 5, gf.R18), gf.Geom.make((8, 8, 8, 8), gf.FP32, 10),
                gf.Geom.make((2048, 2048, 2048, 2))]:
        assert gf.check_geom(bad) == gf.ERR_ARG
        assert gf.field_bytes(bad) == 0
    assert gf.lib().gf_check_geom(None) == gf.ERR_ARG
    # gauge-transformation field: FP32 rows 0 and 1 (6 complex) per padded site
    assert gf.gauge_bytes(gf.Geom.make((6, 4, 2, 10), gf.FP32, gf.R12)) == 2 * 2048 * 6 * 8
    assert gf.gauge_bytes(gf.Geom.make((32,) * 4, gf.FP32, gf.R18)) == 32 ** 4 * 6 * 8
    assert gf.gauge_bytes(gf.Geom.make((7, 8, 8, 8))) == 0


def test_calls_without_context_are_rejected_on_host():
    g = gf.Geom.make((4, 4, 4, 4))
    L = gf.lib()
    assert L.gf_sweep(None, None, C.byref(g), 0, 0, 1.5) == gf.ERR_ARG
    assert L.gf_measure(None, None, C.byref(g), 0, None, None) == gf.ERR_ARG
    assert L.gf_destroy(None) == gf.ERR_ARG


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    st = gf.lib().gf_create(0, None, C.byref(h))
    assert st == gf.ERR_DEVICE
    assert b"no GPU" in gf.lib().gf_last_error(None)
    with pytest.raises(gf.GFError):
        gf.Context()


def test_struct_layouts_match_the_header(tmp_path):
    """the ctypes structures of the binding have the sizes and field offsets
    that a C compiler gives the structs of include/gf.h"""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"gf_geom": gf.Geom, "gf_fix_params": gf.FixParams, "gf_fix_result": gf.FixResult,
               "gf_check_record": gf.CheckRecord}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gf.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        cname, field, value = line.split()
        py = structs[cname]
        got = C.sizeof(py) if field == "size" else getattr(py, field).offset
        assert got == int(value), (cname, field, got, value)
        seen += 1
    assert seen == sum(len(p._fields_) + 1 for p in structs.values())
