"""Host-side checks of the C ABI (no GPU needed).

* libdtsort.so loads and exports every function include/dtsort.h declares,
  and the Python binding declares exactly those;
* the ctypes mirrors of dtsort_opts / dtsort_stats have the C layout (sizes
  and field offsets printed by a C program compiled against the header);
* argument checks that return before any device work;
* the tuning table's format.
"""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

import paper_2401_00710_amd._lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dtsort.h")
TABLE = os.path.join(ROOT, "paper_2401_00710_amd", "tune_table.txt")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dtsort_[a-z0-9_]+)\s*\(", text)))


def test_header_functions_exported():
    lib = L.load()
    names = _declared()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lib, n), f"{n} declared in dtsort.h but not exported"


def test_binding_matches_header():
    assert sorted(L.exported_symbols()) == _declared()


def _c_layout():
    # every field of the ctypes mirrors, so that a field added on one side only fails here
    fields = [f"  F(dtsort_opts, {n});" for n, _ in L.Opts._fields_]
    fields += [f"  F(dtsort_stats, {n});" for n, _ in L.Stats._fields_]
    src = r'''
#include <stddef.h>
#include <stdio.h>
#include "dtsort.h"
#define F(T, f) printf(#T " " #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("sizeof opts %zu\n", sizeof(dtsort_opts));
  printf("sizeof stats %zu\n", sizeof(dtsort_stats));
''' + "\n".join(fields) + r'''
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    lay = {}
    for line in out.splitlines():
        a, b, v = line.split()
        lay[(a, b)] = int(v)
    return lay


def test_struct_layout_matches_c():
    lay = _c_layout()
    assert lay[("sizeof", "opts")] == C.sizeof(L.Opts)
    assert lay[("sizeof", "stats")] == C.sizeof(L.Stats)
    for (t, f), off in lay.items():
        if t == "sizeof":
            continue
        cls = L.Opts if t == "dtsort_opts" else L.Stats
        assert getattr(cls, f).offset == off, f"{t}.{f}"


def test_host_argument_checks():
    lib = L.load()
    o = L.Opts()
    lib.dtsort_default_opts(C.byref(o))
    assert o.mode == L.MODE_SAMPLING and o.digit_bits == 0 and o.graph == 0
    # nothing to sort: returns before any device work
    assert lib.dtsort_u32(None, 0, C.byref(o), None) == L.OK
    one = (C.c_uint64 * 1)(7)
    assert lib.dtsort_u64(C.addressof(one), 1, C.byref(o), None) == L.OK
    assert lib.dtsort_u64(None, 1, C.byref(o), None) == L.EINVAL
    # invalid arguments are refused on the host
    assert lib.dtsort_u32(None, 10, C.byref(o), None) == L.EINVAL
    assert lib.dtsort_pairs_u64(C.c_void_p(4096), None, 10, C.byref(o), None) == L.EINVAL
    buf = (C.c_uint64 * 16)()
    p = C.addressof(buf)
    assert lib.dtsort_pairs_u64(p, p + 8, 4, C.byref(o), None) == L.EINVAL  # overlapping arrays
    bad = L.Opts()
    lib.dtsort_default_opts(C.byref(bad))
    bad.digit_bits = 11
    assert lib.dtsort_u32(C.c_void_p(4096), 10, C.byref(bad), None) == L.EINVAL
    bad.digit_bits, bad.digit_bits_below = 0, 11
    assert lib.dtsort_u32(C.c_void_p(4096), 10, C.byref(bad), None) == L.EINVAL
    bad.digit_bits_below, bad.tile_shape = 0, 7
    assert lib.dtsort_u32(C.c_void_p(4096), 10, C.byref(bad), None) == L.EINVAL
    bad.tile_shape, bad.graph, bad.mode = 0, 1, L.MODE_LEARNED
    assert lib.dtsort_u32(C.c_void_p(4096), 10, C.byref(bad), None) == L.EINVAL
    bad.graph, bad.mode, bad.key_bits = 0, L.MODE_SAMPLING, 40
    assert lib.dtsort_u32(C.c_void_p(4096), 10, C.byref(bad), None) == L.EINVAL
    assert lib.dtsort_segmented(C.c_void_p(4096), None, 10, None, 3, C.byref(o), None) == L.EINVAL
    assert lib.dtsort_workspace_bytes(4, 0, 1000) >= 4000
    assert lib.dtsort_workspace_bytes(8, 8, 1000) >= 16000
    assert lib.dtsort_strerror(L.EINVAL).decode() == "invalid argument"
    assert lib.dtsort_last_error().decode() != ""


def test_tune_table_format():
    rows = []
    for line in open(TABLE):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x) for x in line.split()]
        assert len(v) == 9, line
        kb, vb, seg, lo, hi, g, cut, tile, g_below = v
        assert kb in (4, 8) and vb in (0, 4, 8) and seg in (0, 1)
        assert 0 <= lo <= hi <= 63
        assert 0 <= g <= 10 and 0 <= cut <= 16384 and 0 <= tile <= 6 and 0 <= g_below <= 10
        rows.append(v)
    # every layout the entry points take has a row
    keys = {(r[0], r[1], r[2]) for r in rows}
    for k in ((4, 0, 0), (8, 0, 0), (8, 8, 0), (4, 4, 0), (4, 0, 1)):
        assert k in keys


def test_autotune_table_writer(tmp_path):
    from paper_2401_00710_amd import autotune
    p = tmp_path / "t.txt"
    autotune.write_table([(4, 0, 0, 0, 63, 9, 8192, 3, 9)], str(p), "test")
    lines = [x for x in open(p) if not x.startswith("#")]
    assert lines == ["4 0 0 0 63 9 8192 3 9\n"]
    # a table written before the last column reads with 0 there
    q = tmp_path / "old.txt"
    q.write_text("# old\n4 0 0 0 63 9 8192 3\n")
    assert autotune.read_table(str(q)) == [(4, 0, 0, 0, 63, 9, 8192, 3, 0)]


def test_noalloc_host_checks():
    """The allocation-free entry point refuses, before any device work, what
    its static scratch cannot hold and the options that need a read-back or
    allocations."""
    lib = L.load()
    o = L.Opts()
    lib.dtsort_default_opts(C.byref(o))
    fake, seg = C.c_void_p(1 << 40), C.c_void_p(1 << 42)
    assert lib.dtsort_segmented_noalloc(None, None, 0, None, 0, C.byref(o), None) == L.OK
    assert lib.dtsort_segmented_noalloc(fake, None, 10, None, 3, C.byref(o), None) == L.EINVAL
    assert lib.dtsort_segmented_noalloc(fake, None, 1 << 23, seg, 1, C.byref(o), None) == L.EINVAL
    msg = lib.dtsort_last_error().decode()
    assert "scratch" in msg and "67108864" in msg
    assert lib.dtsort_segmented_noalloc(fake, C.c_void_p(1 << 41), 1 << 22, seg, 1, C.byref(o), None) == L.EINVAL
    st = L.Stats()
    o2 = L.Opts()
    lib.dtsort_default_opts(C.byref(o2))
    o2.stats = C.pointer(st)
    assert lib.dtsort_segmented_noalloc(fake, None, 1000, seg, 1, C.byref(o2), None) == L.EINVAL
    o3 = L.Opts()
    lib.dtsort_default_opts(C.byref(o3))
    o3.mode = L.MODE_LEARNED
    assert lib.dtsort_segmented_noalloc(fake, None, 1000, seg, 1, C.byref(o3), None) == L.EINVAL
    o4 = L.Opts()
    lib.dtsort_default_opts(C.byref(o4))
    o4.workspace, o4.workspace_bytes = C.c_void_p(1 << 43), 100
    assert lib.dtsort_segmented_noalloc(fake, None, 1000, seg, 1, C.byref(o4), None) == L.EWORKSPACE
