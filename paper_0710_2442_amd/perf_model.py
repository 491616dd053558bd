"""The paper's linear timing model (Eqs. 1-2) instantiated for one MI355X.

Each micro-task i moving I_i bytes (or doing I_i flops) through a device of
throughput beta_i takes T_i = I_i / beta_i (Eq. 1); with all tasks
overlapped T_exe = max_i T_i (Eq. 2).  For the single-parity hop the tasks
are HBM traffic and vector ALU work; the byte count can be the algorithmic
one or the one rocprofv3 measured, and beta_HBM the data-sheet peak or a
measured streaming ceiling.
"""
from __future__ import annotations

MI355X = {
    "hbm_peak": 8.0e12,          # B/s, data sheet
    "hbm_read_ceiling": 6.3e12,  # B/s, streaming-read kernel measured on the box
    "copy_ceiling": 5.5e12,      # B/s, copy kernel (read + write) measured on the box
    "fp64_vector": 78.6e12,      # flop/s
    "fp32_vector": 157.3e12,
    "cus": 256,
    "clock": 2.4e9,
    "l2_per_xcd": 4 * 2 ** 20,
    "xcds": 8,
}

HOP_FLOPS = 1320 + 8 * 42      # Eq. 3 (Sec. 5) + rebuilding third link rows
HOP_BYTES = {"f64": 144 * 8, "f32": 144 * 4}


def hop_model(sites, prec, traffic_ratio=1.0, beta=None):
    """Predicted time (s) of one single-parity hop over `sites` output sites."""
    m = MI355X
    beta = beta or m["hbm_peak"]
    t_hbm = sites * HOP_BYTES[prec] * traffic_ratio / beta
    t_alu = sites * HOP_FLOPS / (m["fp64_vector"] if prec == "f64" else m["fp32_vector"])
    return {"T_hbm": t_hbm, "T_valu": t_alu, "T_exe": max(t_hbm, t_alu)}


def report(sites, prec, measured_s, traffic_ratio=None):
    """Model lines for the benchmark: peak, ceiling, and ceiling with measured traffic."""
    out = {
        "T_hbm_peak_us": 1e6 * hop_model(sites, prec)["T_hbm"],
        "T_hbm_read_ceiling_us": 1e6 * hop_model(sites, prec, beta=MI355X["hbm_read_ceiling"])["T_hbm"],
        "T_valu_us": 1e6 * hop_model(sites, prec)["T_valu"],
        "measured_us": 1e6 * measured_s,
    }
    if traffic_ratio:
        out["T_measured_traffic_at_read_ceiling_us"] = 1e6 * hop_model(
            sites, prec, traffic_ratio, MI355X["hbm_read_ceiling"])["T_hbm"]
    return {k: round(v, 2) for k, v in out.items()}
