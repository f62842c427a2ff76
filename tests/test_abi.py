"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2402_09356_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "tlrmle.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tlr_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = _declared_symbols()
    assert "tlr_loglik" in names and "tlr_reorder" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) <= set(B._SIGNATURES), set(names) - set(B._SIGNATURES)


def test_version_and_strerror():
    L = B.lib()
    assert L.tlr_version().startswith(b"tlrmle")
    assert L.tlr_strerror(0) == b"ok"
    assert L.tlr_strerror(16) == b"matrix not positive definite"


def test_plan_validation_and_workspace_arithmetic():
    with pytest.raises(B.TlrError):
        B.Plan(0, 200)
    with pytest.raises(B.TlrError):
        B.Plan(1600, 8)
    p = B.Plan(1600, 200)
    assert p.nt == 8 and p.maxrank == 100
    # slots alone: 28 tiles x (U + V) x nb x maxrank doubles
    assert p.ws_bytes >= 28 * 2 * 200 * 100 * 8 + 8 * 200 * 200 * 8
    ragged = B.Plan(1601, 200)
    assert ragged.nt == 9
    full = B.Plan(1600, 200, maxrank=200)
    assert full.maxrank == 200 and full.ws_bytes > p.ws_bytes
    # a rank budget sizes the factor arena: 2 nb w entries per unit of width
    small = B.Plan(1600, 200, rank_budget=500)
    tiny = B.Plan(1600, 200, rank_budget=1)
    assert abs(small.ws_bytes - tiny.ws_bytes - 2 * 200 * 499 * 8) < 256  # 256-byte alignment
    assert small.ws_bytes < p.ws_bytes
    m = B.Plan(1600, 200, precision="mixed_fp32", rank_budget=500)
    mt = B.Plan(1600, 200, precision="mixed_fp32", rank_budget=1)
    assert abs(m.ws_bytes - mt.ws_bytes - 2 * 200 * 499 * 4) < 256


def test_invalid_theta_and_small_workspace_rejected_on_host():
    L = B.lib()
    p = B.Plan(400, 100)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: checks fail first
    bad = B._Theta(1.0, -0.1, 0.5)
    assert L.tlr_gen_tiles(p._h, fake, bad, fake, p.ws_bytes, None) == 1
    nan = B._Theta(float("nan"), 0.1, 0.5)
    assert L.tlr_gen_tiles(p._h, fake, nan, fake, p.ws_bytes, None) == 1
    ok = B._Theta(1.0, 0.1, 0.5)
    # below the fixed part of the workspace (the factor arena may be small, not the rest)
    assert L.tlr_gen_tiles(p._h, fake, ok, fake, 4096, None) == 2
    assert L.tlr_compress(p._h, -1.0, fake, p.ws_bytes, None, None) == 1
    assert L.tlr_compress(p._h, float("inf"), fake, p.ws_bytes, None, None) == 1
    assert L.tlr_potrf(p._h, fake, 4096, None) == 2
    assert L.tlr_loglik(None, fake, fake, ok, 1e-9, fake, 10, fake, None, None) == 1


def test_tgh_argument_checks():
    L = B.lib()
    fake = ctypes.c_void_p(0x1000)
    good = B._Tgh(0.0, 1.0, 0.3, 0.1)
    for bad in (B._Tgh(0.0, 0.0, 0.3, 0.1), B._Tgh(0.0, 1.0, 0.3, -0.1), B._Tgh(float("nan"), 1.0, 0.3, 0.1),
                B._Tgh(0.0, 1.0, float("inf"), 0.1)):
        assert L.tlr_tgh_inverse(fake, 10, bad, fake, None) == 1
    assert L.tlr_tgh_inverse(fake, -1, good, fake, None) == 1
    assert L.tlr_tgh_inverse(None, 0, good, None, None) == 0
    p = B.Plan(400, 100)
    ok = B._Theta(1.0, 0.1, 0.5)
    assert L.tlr_loglik_tgh(p._h, fake, fake, ok, B._Tgh(0.0, -1.0, 0.3, 0.1), 1e-9, fake, p.ws_bytes, fake, fake,
                            None) == 1
    # workspace and theta are checked before the transform is launched
    assert L.tlr_loglik_tgh(p._h, fake, fake, ok, good, 1e-9, fake, 4096, fake, fake, None) == 2
    assert L.tlr_loglik_tgh(p._h, fake, fake, B._Theta(1.0, -0.1, 0.5), good, 1e-9, fake, p.ws_bytes, fake, fake,
                            None) == 1


def test_reorder_argument_checks():
    L = B.lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.tlr_reorder(fake, -1, 2, 0, 0, fake, fake, 1 << 20, None) == 1
    assert L.tlr_reorder(fake, 10, 9, 0, 0, fake, fake, 1 << 20, None) == 1
    assert L.tlr_reorder(fake, 1000, 2, 0, 0, fake, fake, 16, None) == 2
    assert L.tlr_reorder(None, 0, 2, 0, 0, None, None, 0, None) == 0
    assert L.tlr_reorder_ws_bytes(90000, 4) > L.tlr_reorder_ws_bytes(90000, 2)


def test_diag_entry_checks():
    L = B.lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.tlr_diag_gemm(0, 0, 4, 4, 4, 1.0, fake, 2, fake, 4, 0.0, fake, 4, None) == 1
    assert L.tlr_diag_svd(1, 600, fake, 1e-9, fake, fake, fake, fake, None) == 1


def test_launch_timer_host_side():
    """The timer's host bookkeeping works without a device: enabling,
    resetting and reading with nothing pending, and argument checks."""
    L = B.lib()
    assert L.tlr_kstats_read(None, 4) == -1
    # restricting the timer to one class and back needs no device
    L.tlr_kstats_select.restype = ctypes.c_int32
    L.tlr_kstats_select.argtypes = [ctypes.c_char_p]
    assert L.tlr_kstats_select(b"k_chol_small") == 0
    assert L.tlr_kstats_select(None) == 0
    B.kstats_enable(True)
    B.kstats_reset()
    stats = B.kstats()
    assert all(s["launches"] == 0 and s["total_ms"] == 0.0 for s in stats)
    B.kstats_enable(False)


def test_mixed_precision_plan_rules():
    # float32 factors: smaller workspace; dense off-diagonal tiles and the
    # singular-value truncation are not offered with them
    p64 = B.Plan(9000, 900)
    p32 = B.Plan(9000, 900, precision="mixed_fp32")
    assert p32.ws_bytes < p64.ws_bytes
    with pytest.raises(B.TlrError) as e:
        B.Plan(9000, 900, precision="mixed_fp32", dense_tiles=True)
    assert e.value.code == 3
    with pytest.raises(B.TlrError) as e:
        B.Plan(9000, 900, precision="mixed_fp32", truncation="svd")
    assert e.value.code == 3


def test_alloc_counts_call():
    """The pool counters read without a device; a null pointer is rejected."""
    L = B.lib()
    pinned, streams = B.alloc_counts()
    assert pinned >= 0 and streams >= 0
    assert L.tlr_diag_alloc_counts(None, None) == 1
