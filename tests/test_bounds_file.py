"""Bound files (bbc_bounds_save / bbc_bounds_load): argument checks and the
loader's validation of damaged files, all decided on the host before any
device call, so these run without a GPU.  The round trip through a real build
is in test_gpu_bounds_file.py."""
import ctypes as C
import os
import struct

import numpy as np
import pytest

HEADER_BYTES = 344  # magic, version, size, 3 i32 + f32, 8 i64, 9 f32 + pad, 8 params, 44 build counters


@pytest.fixture(scope="module")
def L():
    from paper_2504_19163_amd import bbc
    if not os.path.exists(bbc.LIB_PATH):
        from paper_2504_19163_amd import build_lib
        build_lib.build()
    return bbc.lib()


def _fnv(data):
    h = 1469598103934665603
    for b in data:
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def _file(toff=(0, 0), coff=(0, 0, 0), magic=b"BBCBOUND", version=2, grid_res=1, max_cell=0, extra_section=False,
          leaf=None, entry=None, cover=0):
    """A well-formed file of one mirror triangle, one point light, one tuple
    without leaves and a 1x1 receiver grid (built by hand, not by the library).
    leaf = (tuple, code) adds one leaf, entry = tuple one grid entry; the cell
    offsets end with the (empty) cover-all slice, whose length the header's
    cover counter gives (cover)."""
    nl, ne = int(leaf is not None), int(entry is not None)
    if leaf is not None:
        toff = (0, 1)
    if entry is not None:
        coff, max_cell = (0, 1, 1), 1
    hdr = magic + struct.pack("<II", version, HEADER_BYTES)
    hdr += struct.pack("<iiif", 0, 0, 32, 1.0)  # chain R, no edges, 32 floats per record, eta
    hdr += struct.pack("<8q", 1, 0, 1, 1, 1, nl, ne, max_cell)  # triangles, emitters, tuples, leaves, entries
    hdr += struct.pack("<9fI", 0, 0, 0, 1, 0, 0, 0, 1, 0, 0)
    hdr += struct.pack("<iffiiiif", 8, 1e-4, 2.0, grid_res, 100, 4, 0, 0.5)
    hdr += bytes(11 * 4) + struct.pack("<I", cover) + bytes(32 * 4)  # build counters, n_cover the 12th
    assert len(hdr) == HEADER_BYTES
    secs = [np.zeros(9, np.float32), np.zeros(9, np.float32), np.array([0, 0, 1], np.float32),
            np.ones(1, np.float32), np.zeros(32, np.float32), np.array([0, 1, 0, 1], np.float32),
            np.array(toff, np.uint32), np.array([leaf[0]] if nl else [], np.uint32),
            np.array([leaf[1]] if nl else [], np.uint32), np.zeros((nl, 4), np.float32),
            np.zeros((nl, 2), np.float32), np.array(coff, np.uint32), np.array([entry] if ne else [], np.uint32),
            np.zeros(ne, np.float32)]
    if extra_section:
        secs.append(np.zeros(1, np.uint32))
    body = hdr
    for a in secs:
        b = a.tobytes()
        body += struct.pack("<Q", len(b)) + b
    return body + struct.pack("<Q", _fnv(body))


def _load(L, path):
    h = C.c_void_p()
    st = L.bbc_bounds_load(os.fsencode(str(path)), None, C.byref(h))
    assert not h.value or st == 0
    return st


def test_null_arguments(L, tmp_path):
    from paper_2504_19163_amd import bbc
    h = C.c_void_p(1)
    assert L.bbc_bounds_load(None, None, C.byref(h)) == bbc.EINVAL and not h.value
    assert L.bbc_bounds_load(b"x", None, None) == bbc.EINVAL
    assert L.bbc_bounds_save(None, os.fsencode(str(tmp_path / "a"))) == bbc.EINVAL
    assert _load(L, tmp_path / "missing.bbc") == bbc.EINVAL
    assert "open" in bbc.last_error()


def test_wellformed_file_passes_host_validation(L, tmp_path):
    """A sound file gets past every host check; without a GPU the first device
    call then fails (EDEVICE), with one it loads (OK)."""
    from paper_2504_19163_amd import bbc
    p = tmp_path / "ok.bbc"
    for kw in ({}, {"leaf": (0, 2 << 28 | 3 << 14 | 1), "entry": 0}):
        p.write_bytes(_file(**kw))
        st = _load(L, p)
        assert st in (bbc.OK, bbc.EDEVICE), (kw, bbc.last_error())


@pytest.mark.parametrize("case,needle", [
    ("magic", "magic"), ("version", "version"), ("truncated", "file size"), ("flip", "checksum"),
    ("toff", "tuple offsets"), ("coff", "cell offsets"), ("max_cell", "fullest cell"), ("grid_res", "file size"),
    ("trailing", "file size"), ("empty", "truncated"), ("leaves_claimed", "file size"), ("leaf_tuple", "leaf tuple"), ("leaf_code", "leaf code"),
    ("entry", "grid entry"), ("cover", "cover-all"),
])
def test_damaged_files_are_rejected(L, tmp_path, case, needle):
    from paper_2504_19163_amd import bbc
    data = {
        "magic": lambda: _file(magic=b"BBCBOUNX"),
        "version": lambda: _file(version=1),
        "truncated": lambda: _file()[:-20],
        "flip": lambda: (lambda d: d[:400] + bytes([d[400] ^ 1]) + d[401:])(_file()),
        "toff": lambda: _file(toff=(0, 3)),
        "coff": lambda: _file(coff=(0, 2, 2)),
        "cover": lambda: _file(cover=1),
        "max_cell": lambda: _file(max_cell=1),
        "grid_res": lambda: _file(grid_res=2),
        "trailing": lambda: _file(extra_section=True),
        "empty": lambda: b"",
        "leaves_claimed": lambda: (lambda d: d[:72] + struct.pack("<q", 1 << 31) + d[80:])(_file()),
        "leaf_tuple": lambda: _file(leaf=(1, 0)),
        "leaf_code": lambda: _file(leaf=(0, 1 << 28 | 2 << 14)),
        "entry": lambda: _file(entry=1),
    }[case]()
    p = tmp_path / f"{case}.bbc"
    p.write_bytes(data)
    assert _load(L, p) == bbc.EINVAL, case
    assert needle in bbc.last_error(), (case, bbc.last_error())
