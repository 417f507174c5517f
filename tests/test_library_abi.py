"""The C-ABI library loads and exports every entry point include/bbc.h declares;
argument validation rejects bad calls before any GPU work (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bbc.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:bbc_status|const char\s*\*)\s*(bbc_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_2504_19163_amd import bbc
    if not os.path.exists(bbc.LIB_PATH):
        from paper_2504_19163_amd import build_lib
        build_lib.build()
    return bbc.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(L, n), n
    from paper_2504_19163_amd import bbc
    assert sorted(bbc.EXPORTS) == sorted(names)


def test_null_arguments_are_rejected(L):
    from paper_2504_19163_amd import bbc
    h = C.c_void_p()
    assert L.bbc_build_bounds(None, None, None, None, C.byref(h)) == bbc.EINVAL
    assert L.bbc_build_bounds(None, None, None, None, None) == bbc.EINVAL
    assert L.bbc_query_irradiance(None, None, 0, 1, 0, None, None, None) == bbc.EINVAL
    assert L.bbc_bounds_info(None, None) == bbc.EINVAL
    assert L.bbc_free_bounds(None) == bbc.OK
    assert "null" in bbc.last_error()


def test_bad_parameters_are_rejected(L):
    import numpy as np
    from paper_2504_19163_amd import bbc, scenes
    sc = scenes.flat_mirror()
    s = bbc.Scene()
    s.chain = 0
    s.memory = bbc.MEM_HOST
    s.n_tri = 1
    pos = np.ascontiguousarray(sc["pos"])
    nrm = np.ascontiguousarray(sc["nrm"])
    s.pos = pos.ctypes.data
    s.nrm = nrm.ctypes.data
    s.eta = 1.0
    for k in ("q0", "f1", "f2"):
        getattr(s, k)[:] = [float(x) for x in sc[k]]
    e = bbc.Emitters()
    e.memory = bbc.MEM_HOST
    e.n = 1
    epos = np.ascontiguousarray(sc["epos"])
    eI = np.ascontiguousarray(sc["eI"])
    e.pos = epos.ctypes.data
    e.I0 = eI.ctypes.data
    h = C.c_void_p()
    good = bbc.default_params()
    for bad in [dict(max_depth=15), dict(grid_res=0), dict(init_pieces=300), dict(alpha=0.5), dict(flags=64)]:
        p = bbc.SubdivParams(**dict(good, **bad))
        assert L.bbc_build_bounds(C.byref(s), C.byref(e), C.byref(p), None, C.byref(h)) == bbc.EINVAL, bad
    p = bbc.SubdivParams(**good)
    s.f2[:] = list(s.f1)  # degenerate receiver
    assert L.bbc_build_bounds(C.byref(s), C.byref(e), C.byref(p), None, C.byref(h)) == bbc.EINVAL
    s.f2[:] = [float(x) for x in sc["f2"]]
    s.chain = 2  # two reflections without a second surface
    assert L.bbc_build_bounds(C.byref(s), C.byref(e), C.byref(p), None, C.byref(h)) == bbc.EINVAL
    s.chain = 7  # no such chain
    assert L.bbc_build_bounds(C.byref(s), C.byref(e), C.byref(p), None, C.byref(h)) == bbc.EINVAL
    s.chain = 1  # area lights are for the single reflection only
    edges = np.zeros((6, 1), np.float32)
    e.edges = edges.ctypes.data
    assert L.bbc_build_bounds(C.byref(s), C.byref(e), C.byref(p), None, C.byref(h)) == bbc.EINVAL
    assert "area lights" in bbc.last_error()


def test_struct_layout_matches_header(tmp_path):
    """The binding's ctypes structures have the header's sizes and field
    offsets (compiled with the system C compiler against include/bbc.h)."""
    import shutil
    import subprocess
    from paper_2504_19163_amd import bbc
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"bbc_scene": bbc.Scene, "bbc_emitters": bbc.Emitters, "bbc_subdiv_params": bbc.SubdivParams}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-o", str(exe), str(src)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        name, field, val = line.split()
        got[(name, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
