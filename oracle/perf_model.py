"""The paper's linear timing model (Eqs. 1-2) and its Table 1 arithmetic.

Test infrastructure only.  Eq. 1: a micro-task moving I_i bytes (or doing
I_i operations) over a device of throughput beta_i takes T_i ~ I_i / beta_i;
Eq. 2: with everything overlapped, T_exe ~ max_i T_i; efficiency
eps_FP = T_peak / T_exe (Sec. 3).  The Cell parameters below are the ones
the paper states (Secs. 2, 4, 5), in SPE cycles at 3.2 GHz.
"""
from __future__ import annotations

CLOCK = 3.2e9            # Hz (Sec. 2, footnote)
N_SPE = 8
DP_FLOP_PER_CYCLE = 4    # Enhanced Cell SPE, DP: T_peak = 1320 / 4 = 330 cycles per site
MEM_BW = 25.6e9          # B/s, main memory (Sec. 2, footnote)
EXT_BW = 6.0e9           # B/s, torus bandwidth per Cell (Sec. 5)
DP_WORD = 8


def hop_flops_per_site():
    """Eq. 3 on one site: per hop a projection (6 complex adds), two SU(3)
    mat-vecs (9 complex mul + 6 complex add each) and the accumulation of the
    reconstructed 4-spinor (12 complex adds); the first accumulation is a copy."""
    cadd, cmul = 2, 6
    proj = 6 * cadd
    matvec = 2 * (9 * cmul + 6 * cadd)
    accum = 12 * cadd
    return 8 * (proj + matvec + accum) - accum


def t_peak_cycles_per_site():
    return hop_flops_per_site() / DP_FLOP_PER_CYCLE


def t_fp_cycles_per_site(madds=840, madd_per_cycle=2):
    """At least 840 multiply-adds, two per cycle (Sec. 5)."""
    return madds / madd_per_cycle


def bytes_per_site_streamed():
    """Per-site main-memory traffic with perfect reuse: psi in + 4 links + psi out (DP words)."""
    return (24 + 4 * 18 + 24) * DP_WORD


def t_mem_cycles(sites_per_cell):
    """Eq. 1 for main memory: all SPEs of a Cell share its memory bandwidth."""
    return sites_per_cell * bytes_per_site_streamed() / MEM_BW * CLOCK


def t_ext_cycles(a_ext_per_spe):
    """Eq. 1 for the torus: a projected half spinor (12 DP words) per boundary site."""
    return a_ext_per_spe * 12 * DP_WORD * N_SPE / EXT_BW * CLOCK


def table1():
    """Columns of Table 1 that follow from Eqs. 1-2 and the stated parameters.

    Returns dict of lists (1000 cycles) for T_peak, T_FP, T_mem, T_ext and
    eps_FP (percent, using the printed T_i for the micro-tasks this model does
    not derive).  T_RF, T_int and T_EIB are taken as printed.
    """
    sites_per_spe = [2 * 2 * 2 * 64 // N_SPE, 8 * 8 * 8 // N_SPE, 4 * 4 * 4 // N_SPE, 2 * 2 * 2 // N_SPE]
    sites_per_cell = [s * N_SPE for s in sites_per_spe]
    a_ext = [192, 48, 12, 3]
    T_peak = [s * t_peak_cycles_per_site() / 1e3 for s in sites_per_spe]
    T_FP = [s * t_fp_cycles_per_site() / 1e3 for s in sites_per_spe]
    T_mem = [None] + [t_mem_cycles(n) / 1e3 for n in sites_per_cell[1:]]
    T_ext = [t_ext_cycles(a) / 1e3 for a in a_ext]
    return {"sites_per_spe": sites_per_spe, "T_peak": T_peak, "T_FP": T_FP, "T_mem": T_mem, "T_ext": T_ext}


def efficiency(T):
    """eps_FP = T_peak / max_i T_i (Eq. 2 and Sec. 3)."""
    vals = [v for k, v in T.items() if k != "T_peak" and v is not None]
    return T["T_peak"] / max(vals)


def caxpy_eps_mm(dp_peak_flops=N_SPE * DP_FLOP_PER_CYCLE * CLOCK):
    """caxpy c*psi + psi' from main memory (Sec. 4): per spin-colour vector
    12 complex multiply-adds (96 flops) against 3 vectors of 192 bytes."""
    t_peak = 96 / dp_peak_flops
    t_mem = 3 * 192 / MEM_BW
    return t_peak / t_mem


def caxpy_ls_ratio(ls_bytes_per_cycle=16):
    """caxpy from the local store: T_peak / T_LS per complex element
    (8 flops at 4 per cycle vs 3 complex loads/stores of 16 bytes)."""
    return (8 / DP_FLOP_PER_CYCLE) / (3 * 16 / ls_bytes_per_cycle)


def v_spe_bound(ls_bytes=256 * 1024, spinors=8, links=12):
    """Largest local volume with 8 spinors and 3x4 links per site in 256 kB (Sec. 5)."""
    return ls_bytes / (spinors * 24 * DP_WORD + links * 18 * DP_WORD)
