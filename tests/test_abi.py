"""The C-ABI library loads on a machine without a GPU and exports every symbol of include/gmt.h."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gmt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gmt_[A-Za-z_0-9]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = _declared()
    for required in ["gmt_build_hierarchy", "gmt_apply_K", "gmt_vcycle", "gmt_solve", "gmt_homogenize"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2604_26518_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libgmt.so not built (run python -m paper_2604_26518_amd.build)")
    L = binding.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(binding.SIGNATURES) == set(_declared())


def test_oracle_rows_match_full_apply():
    import numpy as np
    from gmt_inputs import gyroid_sheet, random_vectors
    from oracle import fem, hierarchy, operators as ops
    lv = hierarchy.build(gyroid_sheet(16, 2, 0.3), 1)[0]
    u = random_vectors(lv.n_n, 18, 1).reshape(lv.n_n, 6, 3)
    rows = np.array([0, 5, 17, lv.n_n - 1])
    full = ops.apply_K(lv, fem.Ke_elastic(), u)
    assert np.abs(ops.apply_K_rows(lv, fem.Ke_elastic(), u, rows) - full[rows]).max() < 1e-13


@pytest.mark.parametrize("attention", [False, True])
def test_network_parameter_count_matches_the_oracle_layout(attention):
    """gmt_nn_param_count (host code, no GPU call) counts the oracle's flat layout, with the
    attention projections appended after every convolutional parameter."""
    from paper_2604_26518_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libgmt.so not built (run python -m paper_2604_26518_amd.build)")
    from oracle import nn as onn
    for chs in ([16, 32, 64], [32, 64, 64], [16, 32, 64, 64, 64, 64]):
        n = binding.nn_param_count(len(chs), chs, attention=attention)
        assert n == onn.UNet(chs, 32, 18, attention=attention).n_params()
        assert binding.nn_param_count(len(chs), chs, physics="thermal", attention=attention) == \
            onn.UNet(chs, 32, 3, attention=attention).n_params()
    with pytest.raises(binding.GmtError):
        cfg = binding.nn_config(3, [16, 32, 64])
        cfg.attention = 2
        import ctypes as ct
        out = ct.c_size_t()
        binding._check(binding.lib().gmt_nn_param_count(ct.byref(cfg), 0, ct.byref(out)))
