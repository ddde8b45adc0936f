"""The C-ABI library loads and exports every entry point its header declares
(no GPU needed: only calls that fail validation before touching the device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "smol.h")).read()
    return sorted(set(re.findall(r"\b(smol_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_2407_16559_amd as smol
    if not os.path.exists(smol.LIB_PATH):
        pytest.skip("libsmol.so not built")
    return smol.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "smol_rhs" in names and "smol_integrate" in names
    for name in names:
        assert hasattr(lib, name), name


def test_strerror_and_version(lib):
    import paper_2407_16559_amd as smol
    assert smol.version()
    for code in range(0, -8, -1):
        assert smol.strerror(code) != "unknown status code"
    assert smol.strerror(-99) == "unknown status code"


def test_validation_before_device(lib):
    """Bad sizes, ranks, lambdas and null pointers are rejected up front."""
    p = ctypes.c_void_p(16)
    assert lib.smol_rhs(0, 3, p, p, 0.0, p, ctypes.c_void_p(32), 0, None) == -1
    assert lib.smol_rhs(10, 0, p, p, 0.0, p, ctypes.c_void_p(32), 0, None) == -1
    assert lib.smol_rhs(10, 33, p, p, 0.0, p, ctypes.c_void_p(32), 0, None) == -1
    assert lib.smol_rhs(10, 3, p, p, -1.0, p, ctypes.c_void_p(32), 0, None) == -1
    assert lib.smol_rhs(10, 3, p, p, float("nan"), p, ctypes.c_void_p(32), 0, None) == -1
    assert lib.smol_rhs(10, 3, None, p, 0.0, p, ctypes.c_void_p(32), 0, None) == -1
    assert lib.smol_rhs(10, 3, p, p, 0.0, p, p, 0, None) == -1          # dndt aliases n
    assert lib.smol_rhs(10, 3, p, p, 0.0, p, ctypes.c_void_p(32), 7, None) == -1
    assert lib.smol_rhs(1 << 21, 3, p, p, 0.0, p, ctypes.c_void_p(32), 0, None) == -7
    ms = (ctypes.c_float * 4)()
    assert lib.smol_profile_step(0, 3, p, p, 0.0, p, 1, 5, ms, None) == -1       # M < 1
    assert lib.smol_profile_step(64, 3, p, p, 0.0, None, 1, 5, ms, None) == -1   # no n0
    assert lib.smol_profile_step(64, 3, p, p, 0.0, p, 1, 0, ms, None) == -1      # iters < 1
    assert lib.smol_profile_step(64, 3, p, p, 0.0, p, 2, 5, ms, None) == -1      # not BS3 / DP5
    assert lib.smol_profile_step(64, 3, p, p, 0.0, p, 1, 5, None, None) == -1    # no output


def test_no_fallback_without_library(monkeypatch, tmp_path):
    """The binding never computes on its own: a missing library raises."""
    import paper_2407_16559_amd as smol
    monkeypatch.setattr(smol, "_lib", None)
    monkeypatch.setattr(smol, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        smol.lib()


def test_schedule_variants_host_logic(lib):
    """Which kernel variants exist per transform length (host-side table, no
    device work): variant 0 everywhere; variants 1..3 only for L >= 2^12,
    the radix-4 variants (2, 3) only for transforms of length <= 256, and
    no variant whose LDS exceeds a workgroup's share (the 8-wave row-pair
    pass at L = 2^20)."""
    import paper_2407_16559_amd as smol
    saved = {L: smol.get_schedule(L) for L in range(6, 21)}
    try:
        for logL in range(6, 21):
            N1, N2 = 2 ** ((logL + 1) // 2), 2 ** (logL // 2)
            for ph, N in ((0, N1), (1, N2), (2, N1)):
                for v in range(4):
                    want = [0, 0, 0]
                    want[ph] = v
                    ok = v == 0 or (logL >= 12 and (v < 2 or N <= 256))
                    ok = ok and not (logL == 20 and ph == 1 and v == 1)
                    if ok:
                        smol.set_schedule(logL, want)
                        assert smol.get_schedule(logL) == tuple(want)
                    else:
                        with pytest.raises(smol.SmolError):
                            smol.set_schedule(logL, want)
        for bad in ((4, 0, 0), (-1, 0, 0)):
            with pytest.raises(smol.SmolError):
                smol.set_schedule(16, bad)
        for logL in (5, 21):
            with pytest.raises(smol.SmolError):
                smol.get_schedule(logL)
    finally:
        for L, v in saved.items():
            smol.set_schedule(L, v)
