"""CPU-side checks of the C ABI: the library builds and exports every
function declared in include/expm.h; the host-only helpers (problem (4.20)
and Eq. (4.5)) agree with the paper's worked example and with the oracle.
No GPU call is made here."""
import ctypes
import os
import re

import pytest

import oracle
from paper_2110_04493_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "expm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(expm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_names():
    assert header_functions() == sorted(capi.SYMBOLS)


def test_library_exports_every_symbol():
    L = capi.lib()
    for name in header_functions():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value
        # every binding declares its argument types, so that ctypes converts
        # (and checks) each argument instead of guessing
        assert getattr(L, name).argtypes is not None, name


def test_defaults():
    o = capi.expm_opts_default()
    assert (o.normal, o.filter_mode, o.e_r, o.max_filter_iter, o.keep_checkpoints,
            o.reorder) == (-1, 0, 0.1, 64, 0, -1)
    assert (o.norm, o.exact_ri, o.diagnostics, o.literal_a, o.batch_solo_n) == \
        (capi.EXPM_NORM_FRO, 0, 0, 0, 4096)
    assert capi.expm_last_error() == ""


def test_choose_mn_worked_example():
    assert capi.expm_choose_mn(244.9, 1e-16) == (20, 8)


@pytest.mark.parametrize("nh", [1e-6, 0.01, 0.5, 1.0, 2.0, 3.7, 50.0, 244.9, 2333.6, 1e5])
@pytest.mark.parametrize("eps", [1e-16, 1e-14, 1e-12, 1e-10, 1e-6])
def test_choose_mn_matches_oracle(nh, eps):
    assert capi.expm_choose_mn(nh, eps) == oracle.choose_mn(nh, eps)


@pytest.mark.parametrize("M", [1, 7, 15, 20, 60])
@pytest.mark.parametrize("x", [1e-4, 0.1, 0.7, 1.0])
def test_r0_matches_oracle(M, x):
    a, b = capi.expm_r0(M, x), oracle.r0(M, x)
    assert abs(a - b) <= 1e-15 * b


def test_choose_mn_rejects_bad_input():
    with pytest.raises(capi.ExpmError) as e:
        capi.expm_choose_mn(float("nan"), 1e-12)
    assert e.value.code == capi.EXPM_EINVAL
    assert "norm" in capi.expm_last_error() or capi.expm_last_error()


@pytest.mark.parametrize("field,value", [("filter_mode", 7), ("e_r", -0.5),
                                         ("max_filter_iter", 0), ("normal", 2),
                                         ("checkpoint_interval", -2), ("reorder", 3),
                                         ("profile", 3), ("profile", -1),
                                         ("tile_min_fill", float("nan")), ("norm", 2),
                                         ("filter_mode", 3), ("exact_ri", 2),
                                         ("diagnostics", -1), ("literal_a", 2),
                                         ("batch_solo_n", -1), ("use_symmetry", 2)])
def test_plan_rejects_invalid_options(field, value):
    """Option validation runs before the plan touches the device."""
    o = capi.expm_opts_default()
    setattr(o, field, value)
    with pytest.raises(capi.ExpmError) as e:
        capi.expm_plan(o)
    assert e.value.code == capi.EXPM_EINVAL


@pytest.mark.parametrize("nh,eps", [(244.9, 1e-16), (50.0, 1e-12), (3.0, 1e-10)])
def test_alpha_hat_matches_oracle(nh, eps):
    """Eq. (4.8) and (4.9) from the library's host helper against the
    oracle's (which Table 3 row 3 pins)."""
    M, N = oracle.choose_mn(nh, eps)
    r0 = oracle.r0(M, nh * 2.0 ** -N)
    hk = [nh ** (1.0 - 0.02 * k) for k in range(1, 2 * 30 + 2)]   # a decreasing h sequence
    for i in range(0, N + 1):
        ri = 2.0 ** i * r0
        assert capi.expm_alpha_hat(ri, i, N, norm=nh) == oracle.alpha_hat(ri, i, N, norm=nh)
        assert capi.expm_alpha_hat(ri, i, N, hk=hk) == oracle.alpha_hat(ri, i, N,
                                                                         power_norms=hk)
