"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every function include/ivf.h declares, and
reject invalid arguments before touching a device.
"""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2511_03298_amd as ivf
    if not os.path.exists(ivf.LIB_PATH):
        pytest.skip("library not built")
    return ivf, ivf.lib()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ivf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ivf_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_function():
    ivf, lib = _lib()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(names) == sorted(ivf.EXPORTED)


def _desc(ivf, n=1000, d=32, L=8, m=16, offsets=None):
    offs = offsets if offsets is not None else np.linspace(0, n, L + 1).astype(np.int64)
    fake = 0x10000  # never dereferenced: validation and sizing are host-only
    desc = ivf.IndexDesc(n=n, d=d, L=L, m=m, metric=0, base_dtype=0, base=fake,
                         centroids=fake, probe_centroids=None, codebooks=fake, codes=fake,
                         list_offsets=offs.ctypes.data, list_ids=fake)
    return desc, offs


def test_table_sizing_matches_layout():
    ivf, lib = _lib()
    desc, offs = _desc(ivf, n=1000, d=32, L=8, m=16)
    nbytes = lib.ivf_tables_bytes(ctypes.byref(desc))
    lens = np.diff(offs)
    blocks = int(((lens + 63) // 64).sum())
    words = 2
    assert nbytes >= blocks * words * 64 * 4 + blocks * 64 * 4
    assert nbytes % 256 == 0


@pytest.mark.parametrize("field,value", [
    ("n", 0), ("d", 0), ("L", 0), ("m", 0), ("m", 300), ("d", 33), ("metric", 7),
    ("base_dtype", 3), ("base", None), ("codes", None), ("list_ids", None),
])
def test_invalid_descriptors_rejected(field, value):
    ivf, lib = _lib()
    desc, offs = _desc(ivf)
    setattr(desc, field, value)
    assert lib.ivf_tables_bytes(ctypes.byref(desc)) == 0
    assert ivf.last_error()
    h = ctypes.c_void_p()
    st = lib.ivf_build_tables(ctypes.byref(desc), 0x100000, 1 << 30, None, ctypes.byref(h))
    assert st == ivf.IVF_ERR_INVALID_ARG
    assert not h.value


def test_filtration_dims_validated():
    ivf, lib = _lib()
    desc, offs = _desc(ivf, d=32, m=16)
    good = np.arange(0, 64, 2, dtype=np.int32)  # 32 kept columns of 64
    desc.d_base, desc.dims = 64, good.ctypes.data
    with_dims = lib.ivf_tables_bytes(ctypes.byref(desc))
    assert with_dims > 0
    desc.dims, desc.d_base = None, 0
    assert lib.ivf_tables_bytes(ctypes.byref(desc)) == with_dims - 256  # the dims section
    bad = [(64, np.arange(32, 0, -1, dtype=np.int32)),           # not ascending
           (40, np.arange(0, 64, 2, dtype=np.int32)),           # column >= d_base
           (16, np.arange(0, 32, dtype=np.int32)),              # d_base < d
           ]
    for d_base, dims in bad:
        desc.d_base, desc.dims = d_base, dims.ctypes.data
        assert lib.ivf_tables_bytes(ctypes.byref(desc)) == 0
        assert "d" in ivf.last_error()
    desc.dims, desc.d_base = None, 40  # d_base without dims must be 0 or d
    assert lib.ivf_tables_bytes(ctypes.byref(desc)) == 0


def test_bad_offsets_rejected():
    ivf, lib = _lib()
    offs = np.array([0, 10, 5, 1000] + [1000] * 5, dtype=np.int64)
    desc, _ = _desc(ivf, offsets=offs)
    assert lib.ivf_tables_bytes(ctypes.byref(desc)) == 0
    offs = np.linspace(0, 1001, 9).astype(np.int64)
    desc, _ = _desc(ivf, offsets=offs)
    assert lib.ivf_tables_bytes(ctypes.byref(desc)) == 0


def test_small_table_memory_rejected_before_device_use():
    ivf, lib = _lib()
    desc, offs = _desc(ivf)
    nbytes = lib.ivf_tables_bytes(ctypes.byref(desc))
    h = ctypes.c_void_p()
    st = lib.ivf_build_tables(ctypes.byref(desc), 0x100000, nbytes - 256, None, ctypes.byref(h))
    assert st == ivf.IVF_ERR_WORKSPACE


def test_valid_build_without_device_reports_device_error():
    ivf, lib = _lib()
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    desc, offs = _desc(ivf)
    nbytes = lib.ivf_tables_bytes(ctypes.byref(desc))
    h = ctypes.c_void_p()
    st = lib.ivf_build_tables(ctypes.byref(desc), 0x100000, nbytes, None, ctypes.byref(h))
    assert st == ivf.IVF_ERR_DEVICE
    assert "device" in ivf.last_error()


def test_search_argument_validation_without_index():
    ivf, lib = _lib()
    o = ivf.make_opts()
    assert lib.ivf_search_workspace_bytes(None, 10, 4, 10, 100, ctypes.byref(o)) == 0
    st = lib.ivf_search(None, None, 1, None, 1, 1, 1, None, None, 0, None, None, None)
    assert st == ivf.IVF_ERR_INVALID_ARG
    mask = ctypes.c_int32(7)
    st = lib.ivf_get_device_error(None, None, ctypes.byref(mask), None)
    assert st == ivf.IVF_ERR_INVALID_ARG and mask.value == 0
    # widen is bounded before any index is looked at (no int32 overflow of
    # widen * nprobe on the device).
    huge = ivf.make_opts(coarse="bf16", widen=1 << 30)
    st = lib.ivf_search(None, None, 1, None, 1, 1, 1, ctypes.byref(huge), None, 0, None, None,
                        None)
    assert st == ivf.IVF_ERR_INVALID_ARG and "widen" in ivf.last_error()
    st = lib.ivf_assign(0x10000, 8, 4, 0, 0x10000, 10, 10, 2, 1 << 30, 0x10000, 1 << 20,
                        0x10000, None)
    assert st == ivf.IVF_ERR_INVALID_ARG and "widen" in ivf.last_error()


def test_every_export_has_a_prototype():
    # Without argtypes ctypes would pass device pointers as 32-bit ints.
    ivf, lib = _lib()
    for name in ivf.EXPORTED:
        assert getattr(lib, name).argtypes is not None, name


def test_default_opts():
    ivf, lib = _lib()
    o = ivf.SearchOpts()
    lib.ivf_default_opts(ctypes.byref(o))
    assert (o.coarse, o.widen, o.form, o.use_graph, o.pool_cap, o.grid, o.rounds) == \
        (0, 2, 0, 0, 0, 0, 0)
    assert (o.spill_cap, o.adaptive) == (0, 0)
    # Auto first-list count; both launch orders longest first.
    assert (o.widen_add, o.first_lists, o.query_order, o.list_order) == (0, 0, 0, 0)
    d = ivf.opts_dict(ivf.make_opts(form="batched", query_order=1, list_order=1))
    assert (d["query_order"], d["list_order"]) == (1, 1)


def test_adaptive_opts_validated():
    ivf, lib = _lib()
    ok = ivf.make_opts(adaptive=dict(nprobe_init=4, nprobe_min=2, reorder_min=10, p0=0.2, p1=0.5))
    assert ivf.opts_dict(ok)["adaptive"]["nprobe_min"] == 2
    for field, value in (("adaptive", 2), ("nprobe_init", 0), ("nprobe_min", 0),
                         ("reorder_min", 0), ("p0", float("nan")), ("p1", float("inf"))):
        o = ivf.make_opts(adaptive=dict(nprobe_init=4, nprobe_min=2, reorder_min=10,
                                        p0=0.2, p1=0.5))
        setattr(o, field, value)
        assert lib.ivf_search_workspace_bytes(None, 1, 1, 1, 1, ctypes.byref(o)) == 0
        assert "opts." in ivf.last_error()


@pytest.mark.parametrize("field,value", [("pool_cap", 100), ("pool_cap", 20000), ("grid", 9),
                                         ("coarse", 7), ("widen", 0), ("form", 3),
                                         ("rounds", 9), ("spill_cap", 100),
                                         ("spill_cap", 20000), ("first_lists", 65),
                                         ("query_order", 2), ("list_order", -1)])
def test_invalid_opts_rejected(field, value):
    ivf, lib = _lib()
    o = ivf.make_opts()
    setattr(o, field, value)
    # Workspace sizing validates the options before the index handle.
    assert lib.ivf_search_workspace_bytes(None, 1, 1, 1, 1, ctypes.byref(o)) == 0
    assert "opts." in ivf.last_error()


def test_spilled_descriptor_validated():
    ivf, lib = _lib()
    # Two copies per point: up to 2n entries, a numbering scratch section.
    offs = np.linspace(0, 2000, 9).astype(np.int64)
    desc, _ = _desc(ivf, n=1000, offsets=offs)
    assert lib.ivf_tables_bytes(ctypes.byref(desc)) == 0       # 2n entries need copies = 2
    desc.copies = 2
    two = lib.ivf_tables_bytes(ctypes.byref(desc))
    assert two > 0
    one_desc, _ = _desc(ivf, n=1000, offsets=np.linspace(0, 1000, 9).astype(np.int64))
    assert lib.ivf_tables_bytes(ctypes.byref(one_desc)) < two
    for bad in (-1, 5):
        desc.copies = bad
        assert lib.ivf_tables_bytes(ctypes.byref(desc)) == 0
        assert "copies" in ivf.last_error()
    desc, _ = _desc(ivf, n=1 << 30, offsets=np.linspace(0, 1000, 9).astype(np.int64))
    desc.copies = 2                                              # n * copies >= 2^31 - 1
    assert lib.ivf_tables_bytes(ctypes.byref(desc)) == 0


def test_assign_spill_arguments_validated():
    ivf, lib = _lib()
    assert lib.ivf_assign_spill_workspace_bytes(1, 8, 100) == 0  # needs a second list
    assert lib.ivf_assign_spill_workspace_bytes(16, 8, 0) == 0
    assert lib.ivf_assign_spill_workspace_bytes(16, 8, 100) > 0
    fake = 0x10000
    for lam in (float("nan"), -1.0, float("inf")):
        st = lib.ivf_assign_spill(fake, 16, 8, fake, 10, fake, lam, 10, fake, 1 << 20, fake, None)
        assert st == ivf.IVF_ERR_INVALID_ARG and "lam" in ivf.last_error()
    st = lib.ivf_assign_spill(fake, 16, 8, fake, 0, fake, 1.0, 10, fake, 1 << 20, fake, None)
    assert st == ivf.IVF_OK                                      # nothing to do


def test_u8_rows_must_be_bytes():
    ivf, lib = _lib()
    X = np.array([[0.0, 1.0], [2.5, 3.0]], np.float32)
    for bad in (X, X - 3.0, X * 200.0):
        with pytest.raises(ValueError):
            ivf.GpuIndex(bad, np.zeros((1, 2), np.float32), np.zeros((1, 16, 2), np.float32),
                         np.zeros((2, 1), np.uint8), [0, 2], [0, 1], "l2", base_dtype="u8",
                         device="cpu")


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    # No fallback: without the HIP library every entry of the binding raises.
    import numpy as np
    import paper_2511_03298_amd as ivf
    monkeypatch.setattr(ivf, "LIB_PATH", str(tmp_path / "libivfpq.so"))
    monkeypatch.setattr(ivf, "_LIB", None)
    with pytest.raises(RuntimeError, match="not built"):
        ivf.lib()
    with pytest.raises(RuntimeError, match="not built"):
        ivf.GpuIndex(np.zeros((4, 2), np.float32), np.zeros((1, 2), np.float32),
                     np.zeros((1, 16, 2), np.float32), np.zeros((4, 1), np.uint8), [0, 4],
                     np.arange(4, dtype=np.int32), "l2", device="cpu")


def test_header_is_plain_c_and_matches_the_binding(tmp_path):
    # A C99 program (warnings as errors) includes the public header, links
    # against the library and calls its host-only entry points; it prints
    # every struct's size and field offsets, which must equal the binding's
    # ctypes layouts (a field the binding names but the header lacks fails
    # the compile).
    import shutil
    import subprocess
    ivf, _ = _lib()
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"ivf_index_desc": ivf.IndexDesc, "ivf_search_opts": ivf.SearchOpts,
               "ivf_table_layout": ivf.TableLayout}
    lines = []
    for cname, ct in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in ct._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    src = tmp_path / "abi_check.c"
    src.write_text("\n".join([
        "#include <stddef.h>", "#include <stdio.h>", "#include <string.h>", '#include "ivf.h"',
        "int main(void) {",
        "  ivf_search_opts o;",
        "  ivf_index_desc d;",
        "  memset(&o, 0xff, sizeof o);",
        "  ivf_default_opts(&o);",
        "  if (o.form != IVF_FORM_PLAIN || o.widen < 1) return 1;",
        "  memset(&d, 0, sizeof d);",
        "  if (ivf_tables_bytes(&d) != 0) return 2;",
        "  if (strlen(ivf_last_error()) == 0) return 3;",
        *lines,
        "  return 0;",
        "}", ""]))
    exe = tmp_path / "abi_check"
    libdir = os.path.dirname(ivf.LIB_PATH)
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                        "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                        "-L", libdir, f"-l:{os.path.basename(ivf.LIB_PATH)}",
                        f"-Wl,-rpath,{libdir}"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stderr)
    got = {}
    for line in r.stdout.splitlines():
        cname, key, val = line.split()
        got[(cname, key)] = int(val)
    for cname, ct in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(ct), cname
        for fname, _ in ct._fields_:
            assert got[(cname, fname)] == getattr(ct, fname).offset, (cname, fname)
