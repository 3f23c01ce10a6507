"""The C-ABI library loads and exports every entry point that include/icrs.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "icrs.h")
LIB = os.path.join(ROOT, "paper_2510_02639_amd", "libicrs.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(icrs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ["icrs_create", "icrs_destroy", "icrs_workspace_bytes", "icrs_magnification",
              "icrs_magnification_given", "icrs_get_sectors", "icrs_point_images", "icrs_status_string"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libicrs.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_binding_names_match_header():
    from paper_2510_02639_amd import icrs
    assert sorted(icrs.EXPORTED) == declared_functions()


def test_host_only_entry_points():
    """Entry points that touch no device memory: defaults, status strings, workspace size."""
    from paper_2510_02639_amd import icrs
    L = icrs.lib()
    cfg = icrs.icrs_config()
    L.icrs_default_config(ctypes.byref(cfg))
    assert cfg.abi_version == 1 and cfg.n_lens == 2 and cfg.n_theta == 256 and cfg.delta_c == 0.1
    assert L.icrs_status_string(-2) == b"workspace too small"
    a = L.icrs_workspace_bytes(None, 1, 200)
    b = L.icrs_workspace_bytes(None, 1, 400)
    assert 0 < a < b and a % 256 == 0
    bad = icrs.icrs_config()
    L.icrs_default_config(ctypes.byref(bad))
    bad.n_lens = 4
    h = ctypes.c_void_p()
    assert L.icrs_create(ctypes.byref(bad), None, ctypes.byref(h)) == -1


def _struct_fields(name):
    """(type, field) pairs of `typedef struct name { ... } name;` in the header."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), text, flags=re.S).group(1)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        typ, fields = decl.split(None, 1)
        out += [(typ, f.strip()) for f in fields.split(",")]
    return out


@pytest.mark.parametrize("name", ["icrs_config", "icrs_profile", "icrs_learned_config", "icrs_learned_stats",
                                  "icrs_hybrid_config"])
def test_binding_structs_match_header(name):
    """The ctypes mirrors of the ABI structs list the header's fields in order, with the same
    widths, so the library and the binding agree on every offset."""
    from paper_2510_02639_amd import icrs
    widths = {"double": 8, "int64_t": 8, "uint64_t": 8, "int32_t": 4, "uint32_t": 4, "int": 4, "float": 4}
    fields = _struct_fields(name)
    mirror = getattr(icrs, name)._fields_
    assert [f for _, f in fields] == [f for f, _ in mirror]
    assert [widths[t] for t, _ in fields] == [ctypes.sizeof(c) for _, c in mirror]


def test_epoch_count_above_the_item_encoding_is_rejected_before_any_launch():
    """FP64-pass work items pack (epoch, sector) into an int32 as 16 e + slot, so a call over
    more than 2^27 epochs is refused with ICRS_EINVAL on the host, before anything is enqueued
    (no device pointer is touched: the stand-in pointers below are never dereferenced)."""
    from paper_2510_02639_amd import icrs
    L = icrs.lib()
    cfg = icrs.icrs_config()
    L.icrs_default_config(ctypes.byref(cfg))
    h = ctypes.c_void_p()
    assert L.icrs_create(ctypes.byref(cfg), None, ctypes.byref(h)) == 0
    try:
        import numpy as np
        p = np.array([[0.9, 0.1, 0.05, 0.6, 0.0, 20.0, 1e-2, 0.5, 0.0, 0.0, 0.0]])
        fake = ctypes.c_void_p(256)
        for n, want in ((icrs.ICRS_MAX_EPOCHS + 1, -1), ((1 << 31) // 10 + 1, -1)):
            off = np.array([0, n], dtype=np.int64)
            code = L.icrs_magnification(h, 1, p.ctypes.data_as(ctypes.c_void_p), off.ctypes.data_as(ctypes.c_void_p),
                                        n, fake, fake, fake, fake, ctypes.c_size_t(1 << 62))
            assert code == want, (n, code)
        # the limit itself passes the host checks and then asks for a larger workspace
        n = icrs.ICRS_MAX_EPOCHS
        off = np.array([0, n], dtype=np.int64)
        code = L.icrs_magnification(h, 1, p.ctypes.data_as(ctypes.c_void_p), off.ctypes.data_as(ctypes.c_void_p),
                                    n, fake, fake, fake, fake, ctypes.c_size_t(0))
        assert code == -2  # ICRS_ENOMEM
    finally:
        L.icrs_destroy(h)
