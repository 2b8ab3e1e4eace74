"""CPU checks of the C ABI: the library loads, exports every function that
include/srmra.h declares, and rejects bad arguments on the host before
touching the device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "srmra.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(srmra_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_2204_04754_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2204_04754_amd import build
        build.build()
    return binding.lib()


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ["srmra_em_step", "srmra_em_step_prepared", "srmra_prepare_observations",
              "srmra_em_step_workspace_bytes", "srmra_prepared_bytes", "srmra_em_step_debug",
              "srmra_plan_create", "srmra_plan_execute", "srmra_plan_destroy",
              "srmra_status_string"]:
        assert n in names


def test_library_exports_every_declared_symbol(L):
    from paper_2204_04754_amd import binding
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(ln.split()[-1] for ln in out.splitlines() if ln.strip())
    for n in _declared():
        assert n in exported, n
        assert hasattr(L, n)


def test_status_strings(L):
    from paper_2204_04754_amd import binding as B
    assert B.status_string(0) == "ok"
    assert "invalid" in B.status_string(-1)
    assert "unsupported" in B.status_string(-2)


def test_invalid_arguments_rejected_on_host(L):
    from paper_2204_04754_amd import binding as B
    fake = ctypes.c_void_p(0x1000)
    other = ctypes.c_void_p(0x100000)
    out = ctypes.c_void_p(0x200000)
    # null pointers
    assert L.srmra_em_step(None, 10, 8, 2, fake, fake, 1.0, out, out, out, 1, None, 0, None) == B.SRMRA_EINVAL
    # sigma <= 0, NaN
    for s in (0.0, -1.0, float("nan"), float("inf")):
        assert L.srmra_em_step(fake, 10, 8, 2, fake, other, s, out, ctypes.c_void_p(0x300000),
                               ctypes.c_void_p(0x400000), 1, None, 0, None) == B.SRMRA_EINVAL
    # x_new aliasing x
    assert L.srmra_em_step(fake, 10, 8, 2, other, fake, 1.0, other, ctypes.c_void_p(0x300000),
                           ctypes.c_void_p(0x400000), 1, None, 0, None) == B.SRMRA_EINVAL
    # N < 1
    assert L.srmra_em_step(fake, 0, 8, 2, other, fake, 1.0, out, ctypes.c_void_p(0x300000),
                           ctypes.c_void_p(0x400000), 1, None, 0, None) == B.SRMRA_EINVAL
    # unsupported L_low
    assert L.srmra_em_step(fake, 10, 10, 2, other, fake, 1.0, out, ctypes.c_void_p(0x300000),
                           ctypes.c_void_p(0x400000), 1, None, 0, None) == B.SRMRA_EUNSUPPORTED
    # missing workspace
    assert L.srmra_em_step(fake, 10, 8, 2, other, fake, 1.0, out, ctypes.c_void_p(0x300000),
                           ctypes.c_void_p(0x400000), 1, None, 0, None) == B.SRMRA_EWORKSPACE
    # misaligned workspace
    assert L.srmra_em_step(fake, 10, 8, 2, other, fake, 1.0, out, ctypes.c_void_p(0x300000),
                           ctypes.c_void_p(0x400000), 1, ctypes.c_void_p(0x500010), 1 << 30,
                           None) == B.SRMRA_EWORKSPACE
    # unknown precision
    assert L.srmra_em_step_workspace_bytes(100, 8, 2, 7) == 0
    # prepared call without prep
    assert L.srmra_em_step_prepared(fake, None, 0, 10, 8, 2, other, fake, 1.0, out,
                                    ctypes.c_void_p(0x300000), None, ctypes.c_void_p(0x400000), 1,
                                    None, 0, None) == B.SRMRA_EINVAL


def test_workspace_sizes(L):
    from paper_2204_04754_amd import binding as B
    for ll in (8, 12, 16, 24, 32, 48, 64):
        for prec in (B.FP32_PLAIN, B.FP32_MFMA):
            assert L.srmra_em_step_workspace_bytes(1000, ll, 2, prec) > 0
            assert L.srmra_prepared_bytes(1000, ll, 2, prec) >= 8 * 1000
    assert L.srmra_em_step_workspace_bytes(1000, 10, 2, B.FP32_MFMA) == 0
    assert L.srmra_em_step_workspace_bytes(1000, 64, 100, B.FP32_MFMA) == 0   # Lh > 4096


def test_pass_count_query():
    """srmra_em_step_passes: one pass for FP32 MFMA shapes whose K^2 components
    fit one workgroup, two otherwise; errors for unsupported shapes."""
    from paper_2204_04754_amd import binding as B
    assert B.srmra_em_step_passes(100000, 32, 2, "fp32_mfma") == 1
    assert B.srmra_em_step_passes(100000, 16, 4, "fp32_mfma") == 1
    assert B.srmra_em_step_passes(200000, 32, 4, "fp32_mfma") == 2
    assert B.srmra_em_step_passes(20000, 64, 4, "fp32_mfma") == 2
    assert B.srmra_em_step_passes(100000, 32, 2, "fp32_plain") == 2
    assert B.srmra_em_step_passes(100000, 32, 2, "bf16_split3") == 2
    with pytest.raises(B.SrmraError):
        B.srmra_em_step_passes(1000, 20, 2, "fp32_mfma")
