"""The paper's linear timing model (Sec. 3, Eqs. 1-2) for one MI355X.

The abstract machine of Sec. 3 is a set of storage devices and processing
devices, each with a throughput beta_i.  A kernel is split into micro-tasks;
task i handles I_i units on device i and takes T_i = I_i / beta_i (Eq. 1);
with every task overlapped and latencies hidden the kernel takes
T_exe = max_i T_i (Eq. 2).  For MI355X the tasks are:

  T_HBM   bytes that must cross the HBM interface (the algorithmic bytes)
  T_MALL  bytes fetched again through the 256 MB Infinity Cache (L2 misses
          beyond the algorithmic bytes, from the rocprofv3 counters)
  T_L2    bytes the kernel's vector loads and stores move between the L2
          caches and the CUs (every gather, every re-read neighbour)
  T_LDS   bytes through the CUs' local data share
  T_VALU  vector ALU work, in lane fused multiply-adds (the fewest
          instructions the flops need; FP32 without packed math and FP64
          both issue 16 lanes per SIMD per clock on gfx950)
  T_MFMA  matrix-core work, in flops at the dense BF16 peak (the network's
          spin mixing)

beta_HBM, beta_MALL and beta_L2 are measured by the library's probes:
wd_micro_stream (HBM read/write mixes) and wd_micro_resident (reads served by
L2 or the Infinity Cache); beta_LDS and beta_VALU follow from the unit counts
and the clock.  Besides Eq. 2's fully overlapped T_exe the model reports the
no-overlap sum of the tasks: a kernel whose waves cannot hide memory behind
arithmetic lands between the two.
"""
from __future__ import annotations

UNITS = {
    "cus": 256,
    "simds_per_cu": 4,
    "lanes_per_simd": 16,   # lanes issued per SIMD per clock (FP32 without packed math, FP64)
    "clock": 2.4e9,
    "lds_bytes_per_clk_per_cu": 128,
    "xcds": 8,
    "l2_per_xcd": 4 * 2 ** 20,
    "mall": 256 * 2 ** 20,
    "hbm_peak": 8.0e12,
    "mfma_bf16_peak": 2.5e15,  # dense BF16 matrix-core flops per second
}

# Throughputs measured on MI355X with the probes above (the benchmark measures
# them again on the box it runs on and uses those).
BETAS = {
    "hbm_read": 6.15e12,    # B/s, reads of a 2 GiB buffer (wd_micro_resident)
    "hbm_copy": 6.62e12,    # B/s, one read + one write stream, non-temporal (wd_micro_stream)
    "hbm_hop_mix": 6.13e12,  # B/s, five read + one write streams, non-temporal (the hop's mix)
    "mall": 6.83e12,        # B/s, reads of a 128 MiB buffer held by the Infinity Cache (wd_micro_resident)
    "l2": 30.2e12,          # B/s, reads of a 16 MiB buffer held by the XCDs' L2 (wd_micro_resident)
}


def beta_valu():
    """Lane fused multiply-adds per second (a flop pair each)."""
    u = UNITS
    return u["cus"] * u["simds_per_cu"] * u["lanes_per_simd"] * u["clock"]


def beta_lds():
    u = UNITS
    return u["cus"] * u["lds_bytes_per_clk_per_cu"] * u["clock"]


# ----------------------------------------------------------- byte accounting
SPINOR_BYTES = {"f64": 24 * 8, "f32": 24 * 4, "f16": 52, "bf16": 48}
LINK_REAL_BYTES = {"f64": 8, "f32": 4, "f16": 4, "bf16": 4}   # hop links: FP64 for FP64, else FP32
HOP_FLOPS = 1320 + 8 * 42      # Eq. 3 (Sec. 5) + rebuilding the third link rows
HOP_BYTES = {p: 96 * LINK_REAL_BYTES[p] + 2 * SPINOR_BYTES[p] for p in SPINOR_BYTES}  # 1152 B FP64, 576 B FP32


def hop_counts(prec):
    """Per output site of the single-parity hop: algorithmic HBM bytes (8 x 12
    link reals + the input spinor once + the output), bytes through L2 (the
    links, six full and two half neighbour spinors, the output) and lane FMAs."""
    sp, lk = SPINOR_BYTES[prec], 96 * LINK_REAL_BYTES[prec]
    return {"hbm": lk + 2 * sp, "l2": lk + 6 * sp + sp + sp, "lds": 0.0, "fma": HOP_FLOPS / 2}


def dirac_counts(prec, staged=True):
    """Per site (both parities) of the one-launch D_W marching along x4:
    algorithmic HBM bytes 4 x 12 link reals + the input spinor once + the
    output.  Through L2: the own spinor, the own 4 links, the three
    neighbours' forward links read as U^dag, the output and, staged, the
    side-face spinors of the brick (384 of 640 staged sites per 256 sites),
    else the six spatial neighbour spinors.  Through LDS (staged): the staged
    sites written once, six neighbour spinors read.  Lane FMAs: the hopping
    term, the third link rows, the a-scaled half spinors and the X term."""
    sp, lr = SPINOR_BYTES[prec], LINK_REAL_BYTES[prec]
    nb = 1.5 * sp if staged else 6 * sp
    return {"hbm": 48 * lr + 2 * sp, "l2": sp + 48 * lr + 36 * lr + nb + sp,
            "lds": (2.5 * sp + 6 * sp) if staged else 0.0, "fma": (HOP_FLOPS + 8 * 12 + 24) / 2}


def mrhs_counts(prec, nrhs):
    """Per site (all nrhs right-hand sides) of the multi-RHS hop: each link
    loaded once for the nrhs spinor sets (FP64 links for FP64, FP32 otherwise)."""
    sp, lk = SPINOR_BYTES[prec], 96 * LINK_REAL_BYTES[prec]
    return {"hbm": lk + 2 * nrhs * sp, "l2": lk + nrhs * 8 * sp, "lds": 0.0,
            "fma": nrhs * 1320 / 2 + 8 * 42 / 2}


def ptc_layer_counts(cin, cout, act="bf16", out="f32", fp16_products=False):
    """Per site of one network layer (9 hops: identity + 8 parallel
    transports; complex 4 x 4 spin weights per hop and channel pair): the
    input channels once, FP32 links (FP16 with FP16 products), the output;
    through L2 the 8 neighbour inputs per channel.  Each transport is 4 spins
    x a 3 x 3 complex mat-vec (36 complex MACs per input channel), each spin
    mixing 16 x 3 complex MACs per channel pair; a complex MAC is 4 FMAs, or
    2 dot2 instructions with FP16 products."""
    a, o = SPINOR_BYTES[act], SPINOR_BYTES[out]
    lk = 96 * (2 if fp16_products else 4)
    cmacs = 8 * 36 * cin + 9 * 48 * cin * cout
    return {"hbm": cin * a + lk + cout * o, "l2": 9 * cin * a + lk + cout * o, "lds": 0.0,
            "fma": cmacs * (2 if fp16_products else 4)}


def cg_iteration_bytes(prec="f64"):
    """One even-odd CGLS iteration (the library's cgls_iteration), bytes per
    even site: q = M p is a plain hop and a hop with the xpay epilogue (+1
    spinor read) and norm; the CG update reads x, p, s, q and writes x, s;
    r = M^dag s is the same two hops; p = r + beta p reads two spinors and
    writes one."""
    sp = SPINOR_BYTES[prec]
    hop = HOP_BYTES[prec]
    return {"hops": 2 * hop + 2 * (hop + sp), "blas": 6 * sp + 3 * sp}


def ptc_network_counts():
    """The whole network as wd_ptc_apply runs it: the FP32 input converted to
    BF16 activations, layer 1 (1 -> 2, BF16 out), layer 2 (2 -> 1, FP32 out)."""
    c1 = ptc_layer_counts(1, 2, "bf16", "bf16")
    c2 = ptc_layer_counts(2, 1, "bf16", "f32")
    c = {k: c1[k] + c2[k] for k in c1}
    conv = SPINOR_BYTES["f32"] + SPINOR_BYTES["bf16"]
    c["hbm"] += conv
    c["l2"] += conv
    return c


def ptc_even_counts():
    """The even-parity application the solver uses (FP16 products, BF16
    fields): layer 1 writes the hidden channels on odd sites, layer 2 the
    output on even sites; per output site of one parity."""
    c1 = ptc_layer_counts(1, 2, "bf16", "bf16", fp16_products=True)
    c2 = ptc_layer_counts(2, 1, "bf16", "bf16", fp16_products=True)
    return {k: c1[k] + c2[k] for k in c1}


def ptc_even_mfma_counts():
    """The even-parity application on the matrix cores (WD_PTC_BF16_MFMA), per
    site pair (one odd site of launch 1, one even site of launch 2), BF16
    fields and links.  HBM: launch 1 reads the input once and the odd links
    (8 x 24 B) and writes two hidden channels; launch 2 reads the hidden
    channels and the input once, the even links, and writes the output (BF16).
    L2: every neighbour spinor read (8 per site and channel).  VALU: the 16
    transports (each 4 spins x 9 complex MACs = 72 two-product dot
    instructions) and the third link rows (12 dot instructions each, 8 in
    launch 1 and 16 in launch 2, where two lane groups rebuild each link).
    MFMA: the spin mixing, 6 (launch 1) and 15 (launch 2) 16x16x32 products
    per 16 sites, including the zero blocks of the A operands."""
    sp = SPINOR_BYTES["bf16"]
    lk = 8 * 24
    hbm = (sp + lk + 2 * sp) + (2 * sp + sp + lk + sp)
    l2 = (8 * sp + lk + 2 * sp) + (8 * 2 * sp + sp + lk + sp)
    dots = 16 * 72 + (8 + 16) * 12
    return {"hbm": hbm, "l2": l2, "lds": 0.0, "fma": dots, "mfma": (6 + 15) * 16 * 16 * 32 * 2 / 16}


def batch_iteration_counts(prec):
    """One inner CG iteration of the batched solver, per even site: four hops
    in the storage precision and the BLAS (the CG update reads the FP32
    solution, p, s, q and writes the solution and s; p = r + beta p reads two
    and writes one: 9 spinor passes)."""
    c = hop_counts(prec)
    cnt = {k: 4 * c[k] for k in c}
    cnt["hbm"] += 9 * SPINOR_BYTES[prec]
    cnt["l2"] += 9 * SPINOR_BYTES[prec]
    return cnt


def kernel_model(kernel, prec, units, traffic_ratio=1.0, betas=None):
    """Eqs. 1-2 for one of the benchmark's kernels: a dict of task times T_i,
    T_exe (Eq. 2, full overlap), T_sum (no overlap) and the bound."""
    if kernel == "hop":
        c = hop_counts(prec)
        refetch = (traffic_ratio - 1.0) * c["hbm"] if traffic_ratio > 1.0 else 0.0
        return predict(units, c, betas, hbm_beta="hbm_hop_mix", mall_bytes=refetch)
    if kernel == "dirac_one_launch":
        c = dirac_counts(prec)
        refetch = (traffic_ratio - 1.0) * c["hbm"] if traffic_ratio > 1.0 else 0.0
        return predict(units, c, betas, hbm_beta="hbm_hop_mix", mall_bytes=refetch)
    if kernel == "mrhs12":
        c = mrhs_counts(prec, 12)
        refetch = (traffic_ratio - 1.0) * c["hbm"] if traffic_ratio > 1.0 else 0.0
        return predict(units, c, betas, mall_bytes=refetch)
    if kernel == "ptc_network":
        return predict(units, ptc_network_counts(), betas)
    if kernel == "ptc_even_fp16_products":
        return predict(units, ptc_even_counts(), betas)
    if kernel == "ptc_even_bf16_mfma":
        return predict(units, ptc_even_mfma_counts(), betas)
    if kernel == "batch8_inner_iteration":
        return predict(units, batch_iteration_counts(prec), betas, resident=True)
    if kernel == "cg_iteration":
        t = cg_iteration_model(units, prec, traffic_ratio, betas)
        return {"T_exe": t["T_iter"], "T_sum": t["T_iter"], "bound": "T_HBM", "T_HBM": t["T_iter"]}
    if kernel == "caxpy":
        t = caxpy_model(units, prec, betas)
        return {"T_exe": t, "T_sum": t, "bound": "T_HBM", "T_HBM": t}
    raise ValueError(kernel)


# --------------------------------------------------------------- Eqs. 1-2
def predict(units, counts, betas=None, hbm_beta="hbm_read", mall_bytes=0.0, resident=False):
    """T_i = I_i / beta_i (Eq. 1) for `units` sites of a kernel with per-site
    `counts`; T_exe = max_i T_i (Eq. 2) and the no-overlap sum.  mall_bytes:
    bytes per site fetched again beyond the algorithmic ones (from the
    counters).  resident: the kernel's data fits the Infinity Cache and stays
    there between launches, so its algorithmic bytes are served there."""
    b = dict(BETAS, **(betas or {}))
    t = {}
    if resident:
        t["T_HBM"] = 0.0
        t["T_MALL"] = units * (counts["hbm"] + mall_bytes) / b["mall"]
    else:
        t["T_HBM"] = units * counts["hbm"] / b[hbm_beta]
        t["T_MALL"] = units * mall_bytes / b["mall"]
    t["T_L2"] = units * counts["l2"] / b["l2"]
    t["T_LDS"] = units * counts["lds"] / beta_lds()
    t["T_VALU"] = units * counts["fma"] / beta_valu()
    t["T_MFMA"] = units * counts.get("mfma", 0.0) / UNITS["mfma_bf16_peak"]
    tasks = ("T_HBM", "T_MALL", "T_L2", "T_LDS", "T_VALU", "T_MFMA")
    t["T_exe"] = max(t[k] for k in tasks)
    t["T_sum"] = sum(t[k] for k in tasks)
    t["bound"] = max(tasks, key=lambda k: t[k])
    return t


def report(t, measured_s):
    """The model beside a measured time, in microseconds."""
    out = {k: round(v * 1e6, 2) for k, v in t.items() if k.startswith("T_")}
    out["bound"] = t["bound"]
    out["measured_us"] = round(measured_s * 1e6, 2)
    out["measured_over_T_exe"] = round(measured_s / t["T_exe"], 3) if t["T_exe"] > 0 else None
    return out


def cg_iteration_model(vh, prec="f64", hop_traffic_ratio=1.0, betas=None):
    """Eqs. 1-2 for one eo-CGLS iteration on vh even sites.  The hop launches
    are modelled as the hop kernel is: their algorithmic bytes at the hop-mix
    ceiling, the bytes fetched again beyond them (the measured traffic ratio)
    as an Infinity-Cache task overlapping it (Eq. 2 within a launch).  The
    BLAS bytes run at the copy ceiling, and the launches follow one another
    (T = sum over the launches)."""
    b = dict(BETAS, **(betas or {}))
    c = cg_iteration_bytes(prec)
    refetch = max(hop_traffic_ratio - 1.0, 0.0)
    t_hops = max(vh * c["hops"] / b["hbm_hop_mix"], vh * c["hops"] * refetch / b["mall"])
    t_blas = vh * c["blas"] / b["hbm_copy"]
    return {"T_hops": t_hops, "T_blas": t_blas, "T_iter": t_hops + t_blas}


def caxpy_model(sites, prec="f64", betas=None):
    """Eqs. 1-2 for y += c x over `sites` sites: 2 spinors read, 1 written."""
    b = dict(BETAS, **(betas or {}))
    return 3 * SPINOR_BYTES[prec] * sites / b["hbm_copy"]
