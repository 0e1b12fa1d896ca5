"""The C ABI library loads and exports every function cddt.h declares.

CPU only: no call here reaches the GPU (validation failures return before any
HIP call; cddt_pair_offset is host-only).
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cddt.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cddt_[a-z_]+)\s*\(", text)))


def _lib():
    from paper_1705_01167_amd import cddt
    if not os.path.exists(cddt.LIB_PATH):
        pytest.fail("libcddt.so is not built (run __graft_entry__.build())")
    return cddt


def test_every_declared_symbol_is_exported():
    cddt = _lib()
    names = _declared()
    assert len(names) >= 25
    L = C.CDLL(cddt.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding covers all of them
    assert set(names) <= set(cddt.SIGNATURES)


def test_validation_needs_no_gpu():
    cddt = _lib()
    L = cddt.lib()
    out = C.c_void_p()
    occ = C.c_void_p(1)   # never dereferenced: validation fails first
    assert L.cddt_create(occ, 0, 5, 8, 0, None, None, C.byref(out)) == cddt.EINVAL
    assert b"width" in L.cddt_last_error()
    assert L.cddt_create(occ, 5, 5, 7, 0, None, None, C.byref(out)) == cddt.EINVAL
    assert L.cddt_create(occ, 5, 5, 8192 + 2, 0, None, None, C.byref(out)) == cddt.EINVAL
    assert L.cddt_create(occ, 5, 16385, 8, 0, None, None, C.byref(out)) == cddt.EINVAL
    assert L.cddt_create(occ, 5, 5, 8, 1 << 7, None, None, C.byref(out)) == cddt.EINVAL
    # bucket width without the bucket flag, and widths outside 2^4..2^10 cells
    assert L.cddt_create(occ, 5, 5, 8, cddt.bucket_flags(7) & ~cddt.FLAG_BUCKETS, None, None,
                         C.byref(out)) == cddt.EINVAL
    assert L.cddt_create(occ, 5, 5, 8, cddt.bucket_flags(3), None, None, C.byref(out)) == cddt.EINVAL
    assert L.cddt_create(occ, 5, 5, 8, cddt.bucket_flags(11), None, None, C.byref(out)) == cddt.EINVAL
    # 16-bit zero points live in the bucket lines: the flag alone is refused
    assert L.cddt_create(occ, 5, 5, 8, cddt.FLAG_ZP16, None, None, C.byref(out)) == cddt.EINVAL
    assert b"BUCKETS" in L.cddt_last_error()
    # pruning is for static maps and is not combined with 16-bit zero points
    assert L.cddt_create(occ, 5, 5, 8, cddt.FLAG_PRUNE, None, None, C.byref(out)) == cddt.EINVAL
    assert b"STATIC" in L.cddt_last_error()
    assert L.cddt_create(occ, 5, 5, 8, cddt.FLAG_PRUNE | cddt.FLAG_STATIC | cddt.FLAG_ZP16 | cddt.FLAG_BUCKETS,
                         None, None, C.byref(out)) == cddt.EINVAL
    assert L.cddt_create(None, 5, 5, 8, 0, None, None, C.byref(out)) == cddt.EINVAL
    assert not out.value
    assert L.cddt_cast(None, None, None, None, 1, 5, None, None) == cddt.EINVAL
    assert L.cddt_update(None, None, None, None, 1, None) == cddt.EINVAL
    assert L.cddt_export_buckets(None, None, 0) == cddt.EINVAL
    assert L.cddt_server_replay_threads(None, 2, 0, None, None, None, None, None, None, None, None) == cddt.EINVAL
    assert L.cddt_destroy(None) == cddt.OK
    assert L.cddt_plan_create(None, 0, None, None, C.byref(out)) == cddt.EINVAL
    # servers: at most 4 lanes (refused before any map is touched)
    cfg = cddt.ServerConfig(1 << 20, 5, 8, 61, 0, cddt.Tuning(8, 2, 8, 7))
    fake = (C.c_void_p * 1)(1)
    offs = (C.c_void_p * 1)(1)
    nr = (C.c_int32 * 1)(61)
    mr = (C.c_int32 * 1)(500)
    assert L.cddt_server_create(fake, 1, offs, nr, offs, mr, C.byref(cfg), C.byref(out)) == cddt.EINVAL
    assert b"1..4" in L.cddt_last_error()
    # resident mode: one lane, search modes 0 and 6..8
    cfg = cddt.ServerConfig(1 << 20, 2, 8, 61, 1, cddt.Tuning(8, 2, 8, 7))
    assert L.cddt_server_create(fake, 1, offs, nr, offs, mr, C.byref(cfg), C.byref(out)) == cddt.EINVAL
    cfg = cddt.ServerConfig(1 << 20, 1, 8, 61, 1, cddt.Tuning(8, 2, 8, 9))
    assert L.cddt_server_create(fake, 1, offs, nr, offs, mr, C.byref(cfg), C.byref(out)) == cddt.EINVAL
    assert b"search modes" in L.cddt_last_error()
    assert L.cddt_batch_weight(None, 1, None, None) == cddt.EINVAL
    f = cddt.Filter()   # map NULL: refused before any device call
    assert L.cddt_batch_weight(C.byref(f), 0, None, None) == cddt.EINVAL
    assert L.cddt_batch_weight(C.byref(f), 1, None, None) == cddt.EINVAL
    assert b"map is NULL" in L.cddt_last_error()


def test_pair_offset_host_helper():
    cddt = _lib()
    from paper_1705_01167_amd import workloads as wl
    assert cddt.pair_offset(wl.ray_offsets(61)) == 40
    assert cddt.pair_offset(wl.ray_offsets(7, fov=np.pi / 2)) == 0
    assert cddt.pair_offset(np.array([0.0, np.pi], np.float32)) == 1
    assert cddt.pair_offset(np.array([0.5], np.float32)) == 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No CPU fallback: every call path goes through lib(), which raises when the
    compiled library is absent."""
    from paper_1705_01167_amd import cddt
    monkeypatch.setattr(cddt, "_lib", None)
    monkeypatch.setattr(cddt, "LIB_PATH", str(tmp_path / "libcddt.so"))
    with pytest.raises(RuntimeError, match="missing"):
        cddt.lib()
    with pytest.raises(RuntimeError, match="missing"):
        cddt.pair_offset(np.zeros(4, np.float32))
