"""Host-side checks of the C-ABI library (no GPU compute)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "blws.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(blws_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1012_0365_amd import _native

    lib = ctypes.CDLL(_native.LIB_PATH)
    names = _declared()
    assert "blws_svt" in names and "blws_rpca_solve" in names
    for name in names:
        assert hasattr(lib, name), name
    # the binding describes every declared entry point, and nothing else
    assert sorted(_native.SIGNATURES) == names


def test_binding_loads_and_reports_statuses():
    from paper_1012_0365_amd import _native

    L = _native.lib()
    assert L.blws_status_string(0) == b"ok"
    assert L.blws_status_string(-1) == b"invalid argument"
    assert L.blws_status_string(-4) == b"NaN or Inf encountered"


def test_default_options_match_the_documented_values():
    import paper_1012_0365_amd as blws

    o = blws.default_alm_opts()
    assert (o.tol, o.max_iter, o.rho, o.mu0_scale, o.mu_max_factor) == (1e-7, 1000, 1.5, 1.25, 1e7)
    assert (o.sv0, o.sv_step_frac, o.b_round, o.pow_steps) == (10, 0.05, 16, 2)
    with pytest.raises(KeyError):
        blws.default_alm_opts(nonexistent=1)


def test_null_context_is_rejected_without_device_work():
    from paper_1012_0365_amd import _native

    L = _native.lib()
    assert L.blws_svt(None, None, 0, 10, 10, None, 10, 0.0, 1, None, 1, None, 1, 1, None, None,
                      None, 0, None) == -1
    assert L.blws_destroy(None) == -1
    out = ctypes.c_void_p()
    assert L.blws_create(None, 0) == -1
    assert L.blws_create(ctypes.byref(out), -5) == -3


def test_oracle_and_library_share_no_sources():
    """The oracle is independent of the HIP path: no include of the other side."""
    csrc = os.path.join(ROOT, "paper_1012_0365_amd", "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f)).read()
        assert "blws_oracle" not in text and "orc_" not in text, f
    for f in ("blws_oracle.c", "blws_oracle.h"):
        text = open(os.path.join(ROOT, "oracle", f)).read()
        assert "blws_common" not in text and "blws.h" not in text
