"""The paper's timing model reproduces the numbers it prints (Table 1, Secs. 4-5)."""
import json
import os

import pytest

from oracle import perf_model as pm

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))


def _close(a, b, digits_rel=0.05):
    return abs(a - b) <= digits_rel * abs(b)


def test_flop_count_and_cycles():
    assert pm.hop_flops_per_site() == GOLD["flops_per_site"]
    assert pm.t_peak_cycles_per_site() == GOLD["T_peak_cycles_per_site"]
    assert pm.t_fp_cycles_per_site() == GOLD["T_FP_cycles_per_site"]
    frac = pm.t_peak_cycles_per_site() / pm.t_fp_cycles_per_site()
    assert int(100 * frac) == GOLD["max_fraction_of_peak_percent"]


@pytest.mark.parametrize("col", range(4))
def test_table1_columns(col):
    T = pm.table1()
    for key in ("T_peak", "T_FP", "T_ext"):
        assert _close(T[key][col], GOLD[key][col]), (key, col, T[key][col])
    if GOLD["T_mem"][col] is not None:
        assert _close(T["T_mem"][col], GOLD["T_mem"][col]), (col, T["T_mem"][col])
    # T_RF is 187.5 cycles per site in every column (printed values, 2 digits)
    assert _close(GOLD["T_RF"][col] * 1e3 / T["sites_per_spe"][col], 187.5, 0.07)
    # efficiency with Eq. 2 over the printed micro-task times
    printed = {k: GOLD[k][col] for k in ("T_peak", "T_FP", "T_RF", "T_mem", "T_int", "T_ext", "T_EIB")}
    assert round(100 * pm.efficiency(printed)) == GOLD["eps_FP_percent"][col]
    # and with the derived T_peak, T_mem and T_ext in place of the printed ones
    derived = dict(printed, T_peak=T["T_peak"][col], T_ext=T["T_ext"][col],
                   T_mem=T["T_mem"][col] if T["T_mem"][col] is not None else None)
    assert abs(100 * pm.efficiency(derived) - GOLD["eps_FP_percent"][col]) < 1.0


def test_limiting_factors():
    """LS layout and the 2^3 slice are bounded by T_ext, larger slices by T_mem (Sec. 5)."""
    T = pm.table1()
    assert T["T_ext"][0] > GOLD["T_EIB"][0] and T["T_ext"][0] > GOLD["T_FP"][0]
    assert T["T_mem"][1] > T["T_ext"][1] and T["T_mem"][2] > T["T_ext"][2]
    assert T["T_ext"][3] > T["T_mem"][3]


def test_caxpy_and_storage_bounds():
    eps = pm.caxpy_eps_mm()
    assert 0.041 <= eps < 0.042  # printed as "<= 4.1%"
    assert abs(pm.caxpy_ls_ratio() - GOLD["caxpy_ls_tpeak_over_tls"]) < 1e-3
    v = pm.v_spe_bound()
    assert GOLD["V_SPE_about"] <= v < GOLD["V_SPE_about"] + 2
    # 32^3x64 distributed as 2^3x64 per Cell needs 4096 Cells
    assert (32 ** 3 * 64) // (2 ** 3 * 64) == 4096
