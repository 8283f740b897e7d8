"""CPU checks of the C ABI library: it loads, exports every symbol the header
declares, its host FP64 design math agrees with the oracle, and argument
validation fails with the documented status codes before any device call."""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import hashing as H
from oracle import rsft as OR
from oracle import windows as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rsft():
    from paper_1610_01050_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_1610_01050_amd import build
        build.build_library()
    binding.load_library()
    return binding


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rsft.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsft_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(rsft):
    lib = ctypes.CDLL(rsft.LIB_PATH)
    declared = declared_functions()
    assert sorted(rsft.SYMBOLS) == declared
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("n,atten", [(8, 60), (256, 60), (1024, 60), (1024, 40),
                                     (2048, 60), (33, 50), (64, 0)])
def test_chebyshev_window_matches_oracle(rsft, n, atten):
    """Library (direct cosine sum, C++) vs oracle (inverse FFT, numpy). For
    n ~ 2048 the window is conditioned at the 1e-10 level with respect to x0
    (T_{n-1}'(x0) ~ 5e8 times one ulp of x0), hence 1e-9."""
    assert np.max(np.abs(rsft.chebyshev_window(n, atten) - W.dolph_chebyshev(n, atten))) < 1e-9
    per = rsft.chebyshev_window(n, atten, periodic=True)
    assert np.max(np.abs(per - W.dolph_chebyshev_periodic(n, atten))) < 1e-9


@pytest.mark.parametrize("n,b,atten", [(64, 8, 60), (256, 16, 60), (1024, 64, 60),
                                       (2048, 128, 40), (128, 8, 0)])
def test_flat_window_matches_oracle(rsft, n, b, atten):
    assert np.max(np.abs(rsft.flat_window(n, b, atten) - W.flat_window(n, b, atten))) < 1e-9


def test_mod_inverse_exhaustive(rsft):
    for n in (8, 64, 1024):
        for s in H.odd_sigmas(n):
            assert rsft.mod_inverse(s, n) == H.mod_inverse(s, n)
    with pytest.raises(rsft.RsftError):
        rsft.mod_inverse(6, 64)


def test_stage1_probability_matches_oracle(rsft):
    for pfa, T, mu in [(1e-3, 3, 3), (1e-4, 3, 3), (1e-4, 7, 4), (1e-6, 50, 15)]:
        assert abs(rsft.stage1_probability(pfa, T, mu) - OR.stage1_probability(pfa, T, mu)) < 1e-14


def test_draw_sigma_odd_in_range_and_deterministic(rsft):
    shape = (1024, 64, 8)
    a = rsft.draw_sigma(123, 32, shape)
    b = rsft.draw_sigma(123, 32, shape)
    assert np.array_equal(a, b)
    for d, n in enumerate(shape):
        assert np.all(a[:, d] % 2 == 1) and np.all((a[:, d] >= 1) & (a[:, d] < n))
    # every odd value of a small dimension appears: the draw is not degenerate
    many = rsft.draw_sigma(5, 32, (16,))
    assert len(set(many[:, 0].tolist())) >= 6


def _params(rsft, **kw):
    base = dict(shape=(64, 64), buckets=(8, 8), rounds=3, pfa=1e-3)
    base.update(kw)
    p, keep = rsft._make_params(**base)
    return p, keep


@pytest.mark.parametrize("kw,status", [
    (dict(shape=(60, 64)), 2),                       # NOT_POW2
    (dict(buckets=(64, 8)), 1),                      # B_d == N_d
    (dict(sigma=[[2, 3]] * 3), 3),                   # even sigma
    (dict(sigma=[[65, 3]] * 3), 3),                  # sigma >= N_d
    (dict(pfa=1.5), 1),
    (dict(rounds=0), 1),
    (dict(rounds=65), 1),
    (dict(segments=2), 1),
    (dict(stage1_pfa=1.0), 1),
    (dict(stage1_pfa=-0.1), 1),
    (dict(mu=4), 1),
    (dict(shape=(512, 512), buckets=(256, 8)), 4),   # B_d > 128 unsupported
    (dict(noise_var=0.0), 1),
    (dict(max_detections=1 << 25), 1),
])
def test_invalid_plans_fail_before_device(rsft, kw, status):
    p, keep = _params(rsft, **kw)
    arr = (rsft.Params * 1)(p)
    h = ctypes.c_void_p()
    st = rsft.load_library().rsft_plan(arr, 1, ctypes.byref(h))
    assert st == status
    assert h.value is None
    assert rsft.load_library().rsft_last_error()


def test_reserved_field_must_be_zero(rsft):
    p, keep = _params(rsft)
    p.reserved0 = 7
    arr = (rsft.Params * 1)(p)
    h = ctypes.c_void_p()
    assert rsft.load_library().rsft_plan(arr, 1, ctypes.byref(h)) == 1


def test_status_strings(rsft):
    lib = rsft.load_library()
    for code, name in rsft.STATUS_NAMES.items():
        assert lib.rsft_status_string(code).decode() == name


def test_product_path_has_no_cpu_fallback(rsft, monkeypatch, tmp_path):
    """The binding refuses to run when the HIP library is missing."""
    monkeypatch.setattr(rsft, "_LIB", None)
    monkeypatch.setattr(rsft, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        rsft.load_library()


@pytest.mark.parametrize("bound", ["lower", "upper"])
def test_design_thresholds_match_oracle(rsft, bound):
    """The library's FP64 design (direct sums, C++) against the oracle's
    (literal rounds, numpy) on the setting of Figs. 6 and 7."""
    from oracle import design as DS
    a_bar, b_bar = DS.alpha_beta_bar((1024,), (64,), 40.0, 40.0, (64.5,))
    want = DS.design(50, 4, 64, 1.8, 0.9, 1e-6, a_bar, b_bar, bound=bound)
    got = rsft.design_thresholds((1024,), (64,), 50, 4, 0.9, 1e-6, (64.5,), window_atten_db=40.0,
                                 eta_m=1.8, upper_bound=bound == "upper")
    assert got["feasible"] == 1 and got["mu"] == want["mu"]
    assert abs(got["alpha_bar"] / a_bar - 1) < 1e-9 and abs(got["beta_bar"] / b_bar - 1) < 1e-9
    for key in ("snr_min", "pd_bar", "pfa_bar", "gamma"):
        assert abs(got[key] / want[key] - 1) < 1e-6, key


def test_design_thresholds_two_dim_and_infeasible(rsft):
    from oracle import design as DS
    a_bar, b_bar = DS.alpha_beta_bar((64, 128), (8, 16), 60.0, 60.0, (10.5, 77.25))
    want = DS.design(20, 3, 128, 4.0, 0.9, 1e-4, a_bar, b_bar)
    got = rsft.design_thresholds((64, 128), (8, 16), 20, 3, 0.9, 1e-4, (10.5, 77.25), eta_m=4.0)
    assert got["mu"] == want["mu"] and abs(got["snr_min"] / want["snr_min"] - 1) < 1e-6
    bad = rsft.design_thresholds((1024,), (64,), 50, 40, 0.9, 1e-6, (64.5,), eta_m=1.8)
    assert bad["feasible"] == 0


def test_struct_layouts_match_header(rsft, tmp_path):
    """The ctypes structures have the sizes and field offsets the C compiler
    gives the header's structs."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    fields = {
        "rsft_params": [f for f, _ in rsft.Params._fields_],
        "rsft_detection": [f for f, _ in rsft.Detection._fields_],
        "rsft_plan_info_t": [f for f, _ in rsft.PlanInfo._fields_],
        "rsft_design_params": [f for f, _ in rsft.DesignParams._fields_],
        "rsft_design_result": [f for f, _ in rsft.DesignResult._fields_],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rsft.h"', "int main(void) {"]
    for st, fs in fields.items():
        lines.append(f'  printf("%zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'  printf("%zu\\n", offsetof({st}, {f}));')
    lines.append("  return 0; }")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = []
    for cls in (rsft.Params, rsft.Detection, rsft.PlanInfo, rsft.DesignParams, rsft.DesignResult):
        want.append(ctypes.sizeof(cls))
        want.extend(getattr(cls, f).offset for f, _ in cls._fields_)
    assert got == want
