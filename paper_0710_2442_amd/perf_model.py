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
    # measured with the library's streaming probe (wd_micro_stream, 16-byte lanes):
    "hbm_read_ceiling": 6.3e12,  # B/s, one read stream, cached loads
    "copy_ceiling": 6.65e12,     # B/s, one read + one write stream, non-temporal
    "hop_mix_ceiling": 6.05e12,  # B/s, five read + one write streams (the hop's mix), non-temporal
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


# One FP64 eo-CGLS iteration (the library's cgls_iteration), bytes per even
# site: q = M p is a plain hop and a hop with the xpay epilogue (+1 spinor
# read) and norm; the CG update reads x, p, s, q and writes x, s; r = M^dag s
# is the same two hops; p = r + beta p reads two spinors and writes one.
SPINOR_BYTES = {"f64": 24 * 8, "f32": 24 * 4}


def cg_iteration_bytes(prec="f64"):
    sp = SPINOR_BYTES[prec]
    hop = HOP_BYTES[prec]
    return {"hops": 2 * hop + 2 * (hop + sp), "blas": 6 * sp + 3 * sp}


def cg_iteration_model(vh, prec="f64", hop_traffic_ratio=1.0):
    """Eqs. 1-2 for one eo-CGLS iteration on vh even sites: the hops' bytes
    (times the measured traffic ratio) at the hop-mix ceiling, the BLAS bytes
    at the copy ceiling; the tasks run one after another (T = sum)."""
    b = cg_iteration_bytes(prec)
    t_hops = vh * b["hops"] * hop_traffic_ratio / MI355X["hop_mix_ceiling"]
    t_blas = vh * b["blas"] / MI355X["copy_ceiling"]
    return {"T_hops": t_hops, "T_blas": t_blas, "T_iter": t_hops + t_blas}


def caxpy_model(sites, prec="f64"):
    """Eqs. 1-2 for y += c x over `sites` sites: 2 spinors read, 1 written."""
    return 3 * SPINOR_BYTES[prec] * sites / MI355X["copy_ceiling"]
