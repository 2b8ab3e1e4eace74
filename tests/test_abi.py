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
              "srmra_plan_create", "srmra_plan_create_tuned", "srmra_plan_default_item_obs",
              "srmra_plan_execute", "srmra_plan_destroy", "srmra_em_step_passes",
              "srmra_project_gaussian", "srmra_project_workspace_bytes", "srmra_prepare_observations_ex",
              "srmra_shift_error", "srmra_shift_error_workspace_bytes",
              "srmra_moments", "srmra_moments_workspace_bytes", "srmra_dft2",
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
    """srmra_em_step_passes: one pass for FP32 MFMA and BF16 split shapes whose
    K^2 components fit one workgroup, two otherwise; errors for unsupported
    shapes."""
    from paper_2204_04754_amd import binding as B
    assert B.srmra_em_step_passes(100000, 32, 2, "fp32_mfma") == 1
    assert B.srmra_em_step_passes(100000, 16, 4, "fp32_mfma") == 1
    assert B.srmra_em_step_passes(200000, 32, 4, "fp32_mfma") == 2
    assert B.srmra_em_step_passes(20000, 64, 4, "fp32_mfma") == 2
    assert B.srmra_em_step_passes(100000, 32, 2, "fp32_plain") == 2
    assert B.srmra_em_step_passes(100000, 32, 2, "bf16_split3") == 1   # one workgroup holds K^2 = 4
    # 512-thread workgroups hold 4 < K^2 <= 16 at L_low 24 and 32
    assert B.srmra_em_step_passes(200000, 32, 4, "bf16_split3") == 1
    assert B.srmra_em_step_passes(5000, 24, 3, "bf16_split4") == 1
    assert B.srmra_em_step_passes(5000, 32, 5, "bf16_split3") == 2
    assert B.srmra_em_step_passes(20000, 64, 4, "bf16_split3") == 2
    assert B.srmra_em_step_passes(50000, 48, 2, "bf16_split3") == 1   # 16x16 tiles, K^2 = 4
    assert B.srmra_em_step_passes(50000, 48, 1, "bf16_split4") == 1
    assert B.srmra_em_step_passes(50000, 48, 3, "bf16_split3") == 2
    with pytest.raises(B.SrmraError):
        B.srmra_em_step_passes(1000, 20, 2, "fp32_mfma")


def test_tuning_table_validated_on_host(L):
    """srmra_plan_create_tuned: a table entry may keep the plan's precision or,
    in a BF16 plan, pick FP32 MFMA; BF16 needs an L_low it is built for; a
    negative item size is rejected; a valid table builds a plan (host only)."""
    import ctypes
    from paper_2204_04754_amd import binding as B
    prob = (B.srmra_problem * 1)()
    p = prob[0]
    p.y, p.prep, p.prep_bytes = 0x1000, 0x100000, 1 << 40
    p.N, p.L_low, p.K = 1000, 32, 2
    p.x, p.log_rho, p.sigma = 0x200000, 0x300000, 1.0
    p.x_new, p.rho_new, p.log_rho_new, p.loglik = 0x400000, 0x500000, 0x600000, 0x700000

    def create(precision, entries):
        tab = (B.srmra_tuning * len(entries))()
        for k, e in enumerate(entries):
            prec, ll, K, form, item = e[:5]
            tab[k].precision, tab[k].L_low, tab[k].K, tab[k].form, tab[k].item_obs = prec, ll, K, form, item
            tab[k].tile = e[5] if len(e) > 5 else 0
        h, ws = ctypes.c_void_p(), ctypes.c_size_t()
        st = L.srmra_plan_create_tuned(prob, 1, precision, tab, len(entries), ctypes.byref(h), ctypes.byref(ws))
        if st == B.SRMRA_OK:
            assert h.value and ws.value > 0
            L.srmra_plan_destroy(h)
        else:
            assert not h.value
        return st

    F32, BF, PL = B.SRMRA_FP32_MFMA, B.SRMRA_BF16_SPLIT3, B.SRMRA_FP32_PLAIN
    assert create(F32, [(F32, 32, 2, BF, 0)]) == B.SRMRA_EINVAL
    assert create(F32, [(F32, 32, 2, PL, 0)]) == B.SRMRA_EINVAL
    assert create(BF, [(BF, 12, 2, BF, 0)]) == B.SRMRA_OK   # BF16 at L_low 12: packed tiles
    assert create(BF, [(BF, 32, 2, F32, -1)]) == B.SRMRA_EINVAL
    assert create(BF, [(BF, 32, 2, F32, 100)]) == B.SRMRA_OK
    assert create(BF, [(F32, 32, 2, F32, 100)]) == B.SRMRA_OK       # other precision: ignored
    assert create(F32, [(F32, 32, 2, F32, 37)]) == B.SRMRA_OK
    # block tiles: only the BF16 split at L_low 16 has a choice (WC in {1, 2, 4})
    p.L_low, p.K = 16, 2
    for wc in (1, 2, 4):
        assert create(BF, [(BF, 16, 2, BF, 0, wc)]) == B.SRMRA_OK
    assert create(BF, [(BF, 16, 2, BF, 0, 3)]) == B.SRMRA_EINVAL
    assert create(BF, [(BF, 16, 2, F32, 0, 2)]) == B.SRMRA_EINVAL     # FP32 MFMA: no choice
    assert create(BF, [(BF, 32, 2, BF, 0, 2)]) == B.SRMRA_EINVAL      # L_low 32: no choice
    assert create(F32, [(F32, 16, 2, F32, 0, 1)]) == B.SRMRA_EINVAL
    assert B.srmra_plan_default_item_obs(1000, 32, 2, "fp32_mfma") > 0


def test_default_item_size_spreads_small_shapes():
    """The plan's default work item is about 2^28 multiply-adds, but a problem
    whose items would then be few (small L_low) is cut into about 128 chunks,
    with no item below 2^24 multiply-adds; the partition depends on the
    problem's own shape only."""
    import math

    from paper_2204_04754_amd import binding as B
    # L_low 8, K 4: 2^28 multiply-adds would be thousands of observations
    for N in (5000, 27500, 50000):
        item = B.srmra_plan_default_item_obs(N, 8, 4, "fp32_mfma")
        assert 100 <= math.ceil(N / item) <= 128 or item * 16 * 8 ** 4 <= 2 ** 24 * 1.01, (N, item)
    assert B.srmra_plan_default_item_obs(50000, 12, 4, "fp32_mfma") <= math.ceil(50000 / 100)
    # large L_low: the 2^28 item already gives many chunks and is kept
    big = B.srmra_plan_default_item_obs(50000, 32, 2, "bf16_split3")
    assert big == B.srmra_plan_default_item_obs(500000, 32, 2, "bf16_split3")
    assert math.ceil(50000 / big) > 128


def test_split4_precision_accepted():
    """SRMRA_BF16_SPLIT4 has the same shapes, preparation and workspace as the
    3-product form, and the same L_low restriction."""
    from paper_2204_04754_amd import binding as B
    for N, ll, K in ((1000, 32, 2), (5000, 24, 4), (1000, 16, 2), (300, 16, 5), (100, 48, 3),
                     (100, 64, 4)):
        assert B.srmra_em_step_workspace_bytes(N, ll, K, "bf16_split4") == \
            B.srmra_em_step_workspace_bytes(N, ll, K, "bf16_split3") > 0
        assert B.srmra_prepared_bytes(N, ll, K, "bf16_split4") == \
            B.srmra_prepared_bytes(N, ll, K, "bf16_split3") > 0
    for ll in (8, 12):   # the packed-tile kernels
        for K in (1, 2, 4, 5, 6):
            assert B.srmra_em_step_workspace_bytes(1000, ll, K, "bf16_split4") == \
                B.srmra_em_step_workspace_bytes(1000, ll, K, "bf16_split3") > 0
        assert B.srmra_plan_form(B.SRMRA_BF16_SPLIT4, ll) == B.SRMRA_BF16_SPLIT4
    assert B.srmra_plan_form(B.SRMRA_BF16_SPLIT4, 32) == B.SRMRA_BF16_SPLIT4
    assert B.srmra_plan_form(B.SRMRA_BF16_SPLIT4, 16) == B.SRMRA_BF16_SPLIT4
    assert B.srmra_plan_form(4, 32) == -1


def test_projection_host_validation(L):
    """srmra_project_gaussian rejects bad sizes, pointers, decay and workspace on
    the host (nothing is enqueued)."""
    import ctypes
    from paper_2204_04754_amd import binding as B
    a, b, s, w = (ctypes.c_void_p(v) for v in (0x1000, 0x2000, 0x3000, 0x10000))
    nb = B.srmra_project_workspace_bytes(64)
    assert nb >= 64 * 64 * 4 and B.srmra_project_workspace_bytes(0) == 0
    assert B.srmra_project_workspace_bytes(5000) == 0
    assert L.srmra_project_gaussian(None, b, 64, s, 0.9, w, nb, None) == B.SRMRA_EINVAL
    assert L.srmra_project_gaussian(a, b, 0, s, 0.9, w, nb, None) == B.SRMRA_EINVAL
    assert L.srmra_project_gaussian(a, b, 64, None, 0.9, w, nb, None) == B.SRMRA_EINVAL
    assert L.srmra_project_gaussian(a, b, 64, s, 0.0, w, nb, None) == B.SRMRA_EINVAL
    assert L.srmra_project_gaussian(a, b, 64, s, float("inf"), w, nb, None) == B.SRMRA_EINVAL
    assert L.srmra_project_gaussian(a, b, 64, s, 0.9, w, nb - 1, None) == B.SRMRA_EWORKSPACE
    assert L.srmra_project_gaussian(a, b, 64, s, 0.9, ctypes.c_void_p(0x10010), nb, None) == B.SRMRA_EWORKSPACE


def test_shift_error_host_validation(L):
    import ctypes
    from paper_2204_04754_amd import binding as B
    a, b, e, w = (ctypes.c_void_p(v) for v in (0x1000, 0x2000, 0x3000, 0x10000))
    nb = B.srmra_shift_error_workspace_bytes(64)
    assert nb == 64 * 64 * 8 and B.srmra_shift_error_workspace_bytes(513) == 0
    assert L.srmra_shift_error(None, b, 64, e, None, w, nb, None) == B.SRMRA_EINVAL
    assert L.srmra_shift_error(a, b, 64, None, None, w, nb, None) == B.SRMRA_EINVAL
    assert L.srmra_shift_error(a, b, 600, e, None, w, nb, None) == B.SRMRA_EINVAL
    assert L.srmra_shift_error(a, b, 64, e, None, w, nb - 8, None) == B.SRMRA_EWORKSPACE


def test_moments_host_validation(L):
    import ctypes
    from paper_2204_04754_amd import binding as B
    y, m1, m2, w = (ctypes.c_void_p(v) for v in (0x1000, 0x2000, 0x3000, 0x10000))
    nb = B.srmra_moments_workspace_bytes(1000, 32)
    assert nb > 0 and B.srmra_moments_workspace_bytes(1000, 33) == 0
    assert B.srmra_moments_workspace_bytes(0, 32) == 0 and B.srmra_moments_workspace_bytes(10, 66) == 0
    assert L.srmra_moments(None, 1000, 32, m1, m2, w, nb, None) == B.SRMRA_EINVAL
    assert L.srmra_moments(ctypes.c_void_p(0x1004), 1000, 32, m1, m2, w, nb, None) == B.SRMRA_EINVAL
    assert L.srmra_moments(y, 0, 32, m1, m2, w, nb, None) == B.SRMRA_EINVAL
    assert L.srmra_moments(y, 1000, 31, m1, m2, w, nb, None) == B.SRMRA_EINVAL
    assert L.srmra_moments(y, 1000, 32, m1, m2, w, nb - 1, None) == B.SRMRA_EWORKSPACE


def test_fft_route_shapes():
    """SRMRA_FP32_FFT: every L_low of the library (powers of two and 3 * 2^m);
    the plan calls do not take it."""
    from paper_2204_04754_amd import binding as B
    for ll in (8, 12, 16, 24, 32, 48, 64):
        assert B.srmra_em_step_workspace_bytes(1000, ll, 2, "fp32_fft") > 0
        assert B.srmra_prepared_bytes(1000, ll, 2, "fp32_fft") >= 1000 * ll * ll * 8
        assert B.srmra_em_step_passes(1000, ll, 2, "fp32_fft") == 2
    for ll in (20, 40):
        assert B.srmra_em_step_workspace_bytes(1000, ll, 2, "fp32_fft") == 0
    assert B.srmra_plan_form(B.SRMRA_FP32_FFT, 32) == -1
