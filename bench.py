#!/usr/bin/env python3
"""Wilson-Dirac hop bandwidth and time-to-solution on one MI355X.

Headline: algorithmic GB/s of the single-parity hop (Eq. 3 on one
checkerboard, 12-real compressed links) on a 32^3x64 lattice with near-unit
random SU(3) links (eps = 0.3) and Gaussian spinors, and its fraction of the
8 TB/s HBM peak.  One step = the hop on the even sites followed by the hop on
the odd sites (two launches, ping-pong: each output feeds the next input;
kappa = 1/8 keeps the values O(1)).  Algorithmic bytes per output site: 8
links x 12 reals + 24 input reals + 24 output reals = 144 reals (1152 B in
FP64, 576 B in FP32).

Also reported:
* the FP32 hop with the same protocol;
* time to a true FP64 residual of 1e-10 on 32^3x64, kappa = 0.124: plain FP64
  even-odd CG on the normal equations vs FP64 defect correction with FP32
  inner arithmetic and FP32 / FP16 / BF16 vector storage;
* the CPU oracle (numpy FP64) timed on one single-parity application of the
  same workload (cpu_baseline);
* HBM traffic per launch from the committed rocprofv3 counter summary when it
  was taken on the current kernel source.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-solve] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DIMS = (32, 32, 32, 64)
HBM_PEAK_GBS = 8000.0
FP64_PEAK_FLOPS = 78.6e12  # MI355X dense FP64 vector
BYTES_PER_SITE = {"f64": 144 * 8, "f32": 144 * 4}
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "dslash_hop_32x32x32x64_traffic.txt")
# pre-tuned hop variants for MI355X (written by wd_tune_dslash; used without re-timing)
TUNE_TABLE = os.path.join(ROOT, "paper_0710_2442_amd", "tuned", "mi355x_hop.jsonl")
# what the hop kernel is built from: its sources and the compile flags
KERNEL_SOURCES = ["paper_0710_2442_amd/csrc/dslash.hip", "paper_0710_2442_amd/csrc/wd_hop.h",
                  "paper_0710_2442_amd/csrc/wd_device.h"]
MRHS_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "mrhs_24x24x24x48_traffic.txt")
MRHS_SOURCES = ["paper_0710_2442_amd/csrc/mrhs.hip", "paper_0710_2442_amd/csrc/wd_hop.h",
                "paper_0710_2442_amd/csrc/wd_device.h"]
DIRAC_SOURCES = ["paper_0710_2442_amd/csrc/dirac.hip", "paper_0710_2442_amd/csrc/wd_hop.h",
                 "paper_0710_2442_amd/csrc/wd_device.h"]
DIRAC_TRAFFIC = os.path.join(ROOT, "profiles", "dirac_one_launch_32x32x32x64_traffic.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_median(torch, fn, reps=3):
    """Wall time of fn() (device synchronised before and after): one warm-up
    run, then the median of `reps` timed runs; returns (seconds, last result)."""
    fn()
    torch.cuda.synchronize()
    secs, r = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t)
    return float(np.median(secs)), r


def kernel_hash(sources=None):
    """Hash of a kernel's sources (default: the single-RHS hop's) and of the
    hipcc flags it is built with (the flags, not the whole build script, so
    build options that leave the library unchanged do not invalidate a
    counter summary)."""
    from paper_0710_2442_amd import build as B

    h = hashlib.sha256()
    for p in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    h.update(" ".join(B.HIP_FLAGS).replace(ROOT, "<root>").encode())
    return h.hexdigest()[:16]


def read_traffic(prec, variant, summary=TRAFFIC_SUMMARY, sources=None):
    """HBM bytes per launch from a committed counter summary, if current."""
    if not os.path.exists(summary):
        return None, "no counter summary"
    vals = {}
    with open(summary) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_hash(sources):
        return None, "kernel changed since counters were taken"
    key = f"hbm_bytes_per_launch_{prec}_{'_'.join(str(v) for v in variant)}"
    if key not in vals:
        return None, f"no counter entry for variant {variant}"
    return float(vals[key]), "ok"


def time_hop(wd, torch, g, psi, prec, steps, warmup):
    """Ping-pong single-parity hops; returns (seconds per launch, launches, total ms)."""
    from paper_0710_2442_amd.fields import canon_to_field, half

    f = canon_to_field(g, psi, prec)
    E, O = half(f, g, prec, 0), half(f, g, prec, 1)
    kappa = 0.125

    def step():
        wd.wd_dslash_ex(g, O, E, kappa, wd.WD_EVEN, prec)
        wd.wd_dslash_ex(g, E, O, kappa, wd.WD_ODD, prec)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(s)
    for _ in range(steps):
        step()
    t1.record(s)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    return ms / 1e3 / (2 * steps), 2 * steps, ms


def measure_betas(wd):
    """The throughputs of the timing model's tasks (Eqs. 1-2), measured here:
    reads held by the XCDs' L2 (16 MiB) and by the Infinity Cache (128 MiB)
    and reads from HBM (2 GiB) with the resident-data probe; a copy and the
    hop's five-read + one-write mix from HBM with the streaming probe."""
    mib = 1 << 20
    b = {}
    b["l2"] = 16 * mib / wd.wd_micro_resident(16 * mib, passes=100, reps=5)
    b["mall"] = 128 * mib / wd.wd_micro_resident(128 * mib, passes=10, reps=5)
    b["hbm_read"] = 2048 * mib / wd.wd_micro_resident(2048 * mib, passes=2, reps=3)
    b["hbm_copy"] = 2 * 1024 * mib / wd.wd_micro_stream(1, 1, 1, 1024 * mib, 10)
    b["hbm_hop_mix"] = 6 * 512 * mib / wd.wd_micro_stream(5, 1, 1, 512 * mib, 10)
    for k, v in b.items():
        log(f"beta {k}: {v / 1e12:.2f} TB/s")
    return b


def time_hop_flushed(wd, torch, g, psi, prec, reps=10):
    """The same hop with the caches emptied first: before every launch a 512 MiB
    device buffer (twice the 256 MB Infinity Cache) is written, so the launch
    finds neither its input nor its links in L2 or the Infinity Cache; HIP
    events on the hop's stream bracket the hop alone.  Returns seconds per launch."""
    from paper_0710_2442_amd.fields import canon_to_field, half

    f = canon_to_field(g, psi, prec)
    E, O = half(f, g, prec, 0), half(f, g, prec, 1)
    scratch = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    tot = 0.0
    for r in range(reps + 1):
        scratch.fill_(r & 0xFF)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        if r % 2 == 0:
            wd.wd_dslash_ex(g, O, E, 0.125, wd.WD_EVEN, prec)
        else:
            wd.wd_dslash_ex(g, E, O, 0.125, wd.WD_ODD, prec)
        e1.record(s)
        torch.cuda.synchronize()
        if r > 0:  # the first launch warms the instruction cache
            tot += e0.elapsed_time(e1)
    del scratch, f
    return tot / 1e3 / reps


def use_tuned(wd, g, table, retune, precs=("f64", "f32", "f16", "bf16")):
    """Hop variants for every storage precision a solver may use, from the
    tuning table (tuned and appended where it has no entry)."""
    for prec in precs:
        b, gr, oc, us = wd.wd_tune_dslash(g, prec, table, force=retune)
        log(f"hop {prec} {g.dims}: block {b}, groups {gr}, occ {oc} ({us:.1f} us)")
        if prec in ("f64", "f32"):
            sl, ti, us = wd.wd_tune_dirac(g, prec, table, force=retune)
            log(f"one-launch D_W {prec} {g.dims}: slices {sl}, tile {ti} ({us:.1f} us)")


def solve_leg(wd, torch, syn, log_every=True, table=None, retune=False):
    """Time to |b - D x|/|b| <= 1e-10 on 32^3x64, kappa = 0.124."""
    from paper_0710_2442_amd.fields import canon_to_field

    kappa, tol = 0.124, 1e-10
    gseed, sseed = syn.CONFIG_SEEDS["mixed_32x32x32x64"]
    U = syn.gauge_field(DIMS, 0.3, gseed)
    b = syn.gaussian_spinor(DIMS, sseed)
    g = wd.Gauge(U, DIMS, -1, "f64")
    use_tuned(wd, g, table, retune)
    fb = canon_to_field(g, b, "f64")
    x = wd.wd_new_field(DIMS, "f64")
    out = {}
    cases = [
        ("fp64_cg", dict(solver=wd.WD_SOLVER_CG)),
        ("defect_f32", dict(solver=wd.WD_SOLVER_DEFECT_CG, inner_prec="f32", inner_tol=1e-4)),
        ("defect_f16", dict(solver=wd.WD_SOLVER_DEFECT_CG, inner_prec="f16", inner_tol=1e-2)),
        ("defect_bf16", dict(solver=wd.WD_SOLVER_DEFECT_CG, inner_prec="bf16", inner_tol=1e-2)),
        # context: CGLS on the full-lattice D_W, without the even-odd reduction
        ("fp64_cgls_full_lattice", dict(solver=wd.WD_SOLVER_CGLS_FULL)),
    ]
    for name, kw in cases:
        p = wd.wd_solve_params_default(**kw)
        wall, (rc, info) = timed_median(torch, lambda: wd.wd_solve(g, fb, x, kappa, tol, p))
        out[name] = {
            "seconds": round(wall, 4),
            "iters": info["iters"],
            "outer_iters": info["outer_iters"],
            "dslash_calls": info["dslash_calls"],
            "true_rel_resid": info["true_rel_resid"],
            "status": rc,
        }
        if name == "fp64_cg":
            xref = x.clone()
        else:
            # |x - x_fp64cg| / |x_fp64cg| with the library's caxpy and norm (both solves
            # are within cond(D) * 1e-10 of the exact solution)
            d = x.clone()
            wd.wd_caxpy(g, -1.0, xref, d, 2, "f64")
            out[name]["rel_diff_vs_fp64_cg_solution"] = float(
                (wd.wd_norm2(g, d, 2, "f64") / wd.wd_norm2(g, xref, 2, "f64")) ** 0.5)
        log(f"solve {name}: {wall:.3f} s (median of 3), iters {info['iters']}, outer {info['outer_iters']}, "
            f"resid {info['true_rel_resid']:.2e}")
    base = out["fp64_cg"]["seconds"]
    for name in out:
        out[name]["speedup_vs_fp64_cg"] = round(base / out[name]["seconds"], 3)
    g.close()
    return out



def _defect(wd, prec, tol_inner=1e-3):
    return wd.wd_solve_params_default(solver=wd.WD_SOLVER_DEFECT_CG, inner_prec=prec, inner_tol=tol_inner)


def mrhs_leg(wd, torch, syn, table=None, retune=False, betas=None, solves=True):
    """12 spin-colour point sources on 24^3x48 (kappa 0.124, eps 0.3), solved together."""
    from paper_0710_2442_amd import perf_model
    from paper_0710_2442_amd.fields import canon_to_field

    dims, kappa, tol = (24, 24, 24, 48), 0.124, 1e-10
    gseed, _ = syn.CONFIG_SEEDS["mrhs_24x24x24x48"]
    U = syn.gauge_field(dims, 0.3, gseed)
    g = wd.Gauge(U, dims, -1, "f64")
    nb = wd.wd_field_bytes(dims, "f64")
    B = torch.cat([canon_to_field(g, syn.point_source(dims, s, c), "f64") for s in range(4) for c in range(3)])
    X = wd.wd_new_field(dims, "f64", 12)
    out = {}
    for prec in ("f32", "bf16", "f64"):
        tb, tg, tr, tus = wd.wd_tune_dslash_mrhs(g, prec, 12, table, force=retune)
        log(f"tuned mrhs hop {prec}: block {tb}, groups {tg}, rhs per lane {tr} ({tus:.1f} us)")
    use_tuned(wd, g, table, retune)

    def timed(fn):
        return timed_median(torch, fn)

    for prec, tin in ((("f32", 1e-3), ("bf16", 1e-2)) if solves else ()):
        sec, (rc, infos) = timed(lambda: wd.wd_solve_mrhs(g, B, X, 12, kappa, tol, _defect(wd, prec, tin)))
        out[f"mrhs12_defect_{prec}"] = {"seconds": round(sec, 4),
                                        "max_resid": max(i["true_rel_resid"] for i in infos),
                                        "iters": max(i["iters"] for i in infos), "status": rc}

    def seq(params):
        res = []
        for r in range(12):
            res.append(wd.wd_solve(g, B[r * nb:(r + 1) * nb], X[r * nb:(r + 1) * nb], kappa, tol, params))
        return res

    if solves:
        sec, res = timed(lambda: seq(_defect(wd, "f32")))
        out["sequential12_defect_f32"] = {"seconds": round(sec, 4),
                                          "max_resid": max(i["true_rel_resid"] for _, i in res)}
        sec, res = timed(lambda: seq(wd.wd_solve_params_default(solver=wd.WD_SOLVER_CG)))
        out["sequential12_fp64_cg"] = {"seconds": round(sec, 4),
                                       "max_resid": max(i["true_rel_resid"] for _, i in res)}
        base = out["sequential12_fp64_cg"]["seconds"]
        for k in out:
            out[k]["speedup_vs_fp64_cg"] = round(base / out[k]["seconds"], 3)
    # multi-RHS hop throughput on 12 Gaussian sources, per site per RHS: in +
    # out spinor (2 x 96 B FP32, 2 x 48 B BF16, 2 x 192 B FP64) + 96/12 link
    # reals (FP32 links; FP64 links for the FP64 hop)
    vh = int(np.prod(dims)) // 2
    tmp = wd.wd_new_field(dims, "f32", 1, wd.WD_ODD)
    for prec, spin_b in (("f32", 96), ("bf16", 48), ("f64", 192)):
        hb = wd.wd_field_bytes(dims, prec, 1, wd.WD_ODD)
        src = wd.wd_new_field(dims, prec, 12, wd.WD_ODD)
        dst = wd.wd_new_field(dims, prec, 12, wd.WD_EVEN)
        for r in range(12):
            if prec in ("f32", "f64"):
                wd.wd_gaussian_field(g, src[r * hb:(r + 1) * hb], wd.WD_ODD, prec, 7, r)
            else:
                wd.wd_gaussian_field(g, tmp, wd.WD_ODD, "f32", 7, r)
                wd.wd_convert(g, tmp, "f32", src[r * hb:(r + 1) * hb], prec, 1, 1.0)
        for _ in range(3):
            wd.wd_dslash_mrhs(g, src, dst, 1.0, wd.WD_EVEN, prec, 12)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            wd.wd_dslash_mrhs(g, src, dst, 1.0, wd.WD_EVEN, prec, 12)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / 20
        per = 2 * spin_b + 96 * (8 if prec == "f64" else 4) // 12
        gbs = vh * 12 * per / (us * 1e-6) / 1e9
        e0.record()
        for _ in range(5):
            for r in range(12):
                wd.wd_dslash_ex(g, src[r * hb:(r + 1) * hb], dst[r * hb:(r + 1) * hb], 1.0, wd.WD_EVEN, prec)
        e1.record()
        torch.cuda.synchronize()
        us12 = e0.elapsed_time(e1) * 1e3 / 5
        out[f"mrhs12_hop_{prec}"] = {"us_per_launch": round(us, 2), "bytes_per_site_rhs": per,
                                     "twelve_single_rhs_hops_us": round(us12, 2),
                                     "speedup_vs_twelve_single_hops": round(us12 / us, 3),
                                     "algorithmic_GBps": round(gbs, 1), "frac_of_8TBps": round(gbs / HBM_PEAK_GBS, 4),
                                     "site_rhs_per_s": round(vh * 12 / (us * 1e-6), 0),
                                     "variant_block_groups_rpl": list(wd.wd_get_dslash_mrhs_variant(g, prec)),
                                     "sources": "12 Gaussian fields"}
        # rocprofv3 counters of this kernel and variant (committed summary), and
        # Eqs. 1-2 with the bytes fetched beyond the algorithmic ones charged to
        # the Infinity Cache
        var = list(wd.wd_get_dslash_mrhs_variant(g, prec))
        traffic, why = read_traffic(prec, var, MRHS_TRAFFIC_SUMMARY, MRHS_SOURCES)
        rec = out[f"mrhs12_hop_{prec}"]
        rec["traffic"] = traffic
        if traffic is None:
            rec["traffic_note"] = why
        ratio = traffic / (vh * 12 * per) if traffic else 1.0
        rec["model_eq1_eq2"] = perf_model.report(perf_model.kernel_model("mrhs12", prec, vh, ratio, betas), us * 1e-6)
        del src, dst
    g.close()
    return out


def batch_leg(wd, torch, syn, table=None, retune=False, betas=None):
    """Eight lattices of uneven size (689,408 sites) in one persistent batched solve."""
    from paper_0710_2442_amd.fields import canon_to_field

    kappa, tol = 0.124, 1e-10
    gs, bs, xs = [], [], []
    for dims, eps, seed in syn.batch_lattices():
        g = wd.Gauge(syn.gauge_field(dims, eps, seed), dims, -1, "f64")
        gs.append(g)
        bs.append(canon_to_field(g, syn.gaussian_spinor(dims, seed + 1000), "f64"))
        xs.append(wd.wd_new_field(dims, "f64"))
    out = {}

    def timed(fn):
        return timed_median(torch, fn)

    for prec, tin in (("f32", 1e-3), ("bf16", 1e-2)):
        p = _defect(wd, prec, tin)
        tile, bpc, tsec = wd.wd_tune_batch(gs, bs, xs, [kappa] * 8, tol, p, table, force=retune)
        p.batch_tile, p.batch_blocks_per_cu = tile, bpc
        log(f"tuned batch {prec}: tile {tile}, blocks per CU {bpc} ({tsec * 1e3:.1f} ms in the tuner)")
        sec, (rc, infos) = timed(lambda: wd.wd_solve_batch(gs, bs, xs, [kappa] * 8, tol, p))
        out[f"batch8_persistent_graph_{prec}"] = {"seconds": round(sec, 4), "status": rc,
                                                 "max_resid": max(i["true_rel_resid"] for i in infos),
                                                 "tile": tile, "blocks_per_cu": bpc}
        # Eqs. 1-2 for one inner CG iteration of the whole batch (4 hops and the
        # BLAS of the storage precision, every field resident in the Infinity
        # Cache: 689,408 sites, ~200 MB per hop launch), beside the measured
        # time per inner iteration (the solve's total over the largest lattice
        # iteration count, outer steps included)
        from paper_0710_2442_amd import perf_model
        vh = sum(int(np.prod(d)) for d, _, _ in syn.batch_lattices()) // 2
        iters = max(i["iters"] for i in infos)
        out[f"batch8_persistent_graph_{prec}"]["model_eq1_eq2_per_inner_iteration"] = perf_model.report(
            perf_model.kernel_model("batch8_inner_iteration", prec, vh, betas=betas), sec / max(1, iters))
    sec, res = timed(lambda: [wd.wd_solve(g, b, x, kappa, tol, _defect(wd, "f32")) for g, b, x in zip(gs, bs, xs)])
    out["sequential8_defect_f32"] = {"seconds": round(sec, 4),
                                     "max_resid": max(i["true_rel_resid"] for _, i in res)}
    sec, res = timed(lambda: [wd.wd_solve(g, b, x, kappa, tol, wd.wd_solve_params_default(solver=wd.WD_SOLVER_CG))
                              for g, b, x in zip(gs, bs, xs)])
    out["sequential8_fp64_cg"] = {"seconds": round(sec, 4),
                                  "max_resid": max(i["true_rel_resid"] for _, i in res)}
    base = out["sequential8_fp64_cg"]["seconds"]
    for k in out:
        out[k]["speedup_vs_fp64_cg"] = round(base / out[k]["seconds"], 3)
    for g in gs:
        g.close()
    return out


def learned_leg(wd, torch, syn, steps, table=None, retune=False):
    """Train the PTC network on 16^4 (kappa 0.124, eps 0.3); test FGCR on 32^3x64."""
    from paper_0710_2442_amd import learn
    from paper_0710_2442_amd.fields import canon_to_field

    kappa, tol = 0.124, 1e-10
    gseed, sseed = syn.CONFIG_SEEDS["ptc_16x16x16x16"]
    gtr = wd.Gauge(syn.gauge_field((16, 16, 16, 16), 0.3, gseed), (16, 16, 16, 16), -1, "f64")
    W, hist = learn.train(gtr, kappa, steps=steps, batch=8, lr=2e-3, seed=sseed, act="bf16", log_every=100,
                          log=log)
    gtr.close()
    out = {"training": {"steps": steps, "pairs": hist["pairs"], "sources": hist["sources"],
                        "seconds": round(hist["seconds"], 2),
                        "pair_generation_seconds": round(hist["pair_generation_seconds"], 2),
                        "loss_first": hist["losses"][0][1], "loss_last": hist["losses"][-1][1]}}
    gt = wd.Gauge(syn.gauge_field(DIMS, 0.3, gseed + 100), DIMS, -1, "f64")
    use_tuned(wd, gt, table, retune)
    fb = canon_to_field(gt, syn.gaussian_spinor(DIMS, sseed + 100), "f64")
    fx = wd.wd_new_field(DIMS, "f64")
    net = wd.Ptc(gt, W, "bf16")
    cases = [("defect_fgcr_trained_bf16", dict(solver=wd.WD_SOLVER_DEFECT_FGCR, fgcr_m=4, inner_tol=1e-2,
                                                precond=net)),
             ("defect_fgcr_identity", dict(solver=wd.WD_SOLVER_DEFECT_FGCR, fgcr_m=4, inner_tol=1e-2)),
             # the same with the inner residual and directions stored in BF16
             ("defect_fgcr_trained_bf16_store_bf16", dict(solver=wd.WD_SOLVER_DEFECT_FGCR, fgcr_m=4, inner_tol=1e-2,
                                                          inner_prec="bf16", precond=net)),
             ("defect_fgcr_identity_store_bf16", dict(solver=wd.WD_SOLVER_DEFECT_FGCR, fgcr_m=4, inner_tol=1e-2,
                                                      inner_prec="bf16")),
             # the FP64 full-lattice FGCR; m = 2 is its fastest restart length here (2 .. 16 measured)
             ("fgcr_trained_bf16", dict(solver=wd.WD_SOLVER_FGCR, fgcr_m=2, precond=net)),
             ("fgcr_identity", dict(solver=wd.WD_SOLVER_FGCR, fgcr_m=2)),
             ("fp64_cg", dict(solver=wd.WD_SOLVER_CG)),
             ("defect_bf16", dict(solver=wd.WD_SOLVER_DEFECT_CG, inner_prec="bf16", inner_tol=1e-2))]
    for name, kw in cases:
        p = wd.wd_solve_params_default(**kw)
        sec, (rc, info) = timed_median(torch, lambda: wd.wd_solve(gt, fb, fx, kappa, tol, p))
        out[name] = {"seconds": round(sec, 4), "iters": info["iters"], "fgcr_m": kw.get("fgcr_m"),
                     "dslash_calls": info["dslash_calls"], "true_rel_resid": info["true_rel_resid"],
                     "fallback_used": info["fallback_used"], "status": rc}
        log(f"learned leg {name}: {out[name]}")
    base = out["fp64_cg"]["seconds"]
    for k in cases:
        out[k[0]]["speedup_vs_fp64_cg"] = round(base / out[k[0]]["seconds"], 3)
    # training time over the time one solve saves: against FP64 CG, and
    # against the same solver without the network (what the network itself buys)
    best = "defect_fgcr_trained_bf16_store_bf16"
    saved = base - out[best]["seconds"]
    out["training"]["solves_to_amortise_vs_fp64_cg"] = round(hist["seconds"] / saved, 1) if saved > 0 else None
    saved_n = out["defect_fgcr_identity_store_bf16"]["seconds"] - out[best]["seconds"]
    out["training"]["solves_to_amortise_vs_same_solver_without_network"] = (
        round(hist["seconds"] / saved_n, 1) if saved_n > 0 else None)
    net.close()
    gt.close()
    return out


def kernels_leg(wd, torch, syn, U, psi, betas=None):
    """Level-1 kernels (Sec. 4's caxpy), full D_W and the network at 32^3x64."""
    import numpy as np

    from paper_0710_2442_amd import perf_model

    from paper_0710_2442_amd import learn
    from paper_0710_2442_amd.fields import canon_to_field

    V = int(np.prod(DIMS))
    out = {}
    g = wd.Gauge(U, DIMS, -1, "f64")
    use_tuned(wd, g, TUNE_TABLE, False, ("f64", "f32"))
    x = canon_to_field(g, psi, "f64")
    y = x.clone()
    z = wd.wd_new_field(DIMS, "f64")

    def ev_time(fn, n=20):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / n

    # caxpy y += c x on full FP64 fields: 3 x 192 B and 12 x 8 flop per site
    t = ev_time(lambda: wd.wd_caxpy(g, 1e-3, x, y, 2, "f64"))
    gbs = V * 576 / t / 1e9
    out["caxpy_f64"] = {"us": round(t * 1e6, 2), "GBps": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                        "eps_fp": round(V * 96 / t / FP64_PEAK_FLOPS, 5),
                        "eps_fp_hbm_bound": round(96 / 576 * HBM_PEAK_GBS * 1e9 / FP64_PEAK_FLOPS, 5),
                        "model_eq1_eq2_us": round(perf_model.caxpy_model(V, "f64", betas) * 1e6, 1)}
    # |x|^2 with the result read back (one synchronisation per call)
    for _ in range(3):
        wd.wd_norm2(g, x, 2, "f64")
    t0 = time.perf_counter()
    for _ in range(20):
        wd.wd_norm2(g, x, 2, "f64")
    t = (time.perf_counter() - t0) / 20
    out["norm2_f64_with_readback"] = {"us": round(t * 1e6, 2), "GBps": round(V * 192 / t / 1e9, 1)}
    # full D_W = 1 - kappa H in one launch: 4 x 12 link + 24 + 24 reals per site
    t = ev_time(lambda: wd.wd_dslash_ex(g, x, z, 0.124, wd.WD_FULL, "f64", wd.WD_ONE_PASS))
    out["dirac_full_f64_one_launch"] = {"us": round(t * 1e6, 2), "GBps": round(V * 768 / t / 1e9, 1),
                                        "frac_hbm": round(V * 768 / t / 1e9 / HBM_PEAK_GBS, 4),
                                        "bytes_per_site": 768}
    # the same with two single-parity launches (each link read twice, xpay operand read)
    t2 = ev_time(lambda: wd.wd_dslash(g, x, z, 0.124, DIMS, wd.WD_FULL))
    out["dirac_full_f64_two_pass"] = {"us": round(t2 * 1e6, 2), "GBps": round(V * 1344 / t2 / 1e9, 1),
                                      "bytes_per_site": 1344, "one_launch_speedup": round(t2 / t, 3)}
    dvar = list(wd.wd_get_dirac_variant(g, "f64"))
    out["dirac_full_f64_one_launch"]["variant_slices_tile"] = dvar
    tb, why = read_traffic("f64", dvar, DIRAC_TRAFFIC, DIRAC_SOURCES)
    ratio = tb / (V * 768) if tb else 1.0
    out["dirac_full_f64_one_launch"]["traffic_ratio_counters"] = round(ratio, 3) if tb else None
    out["dirac_full_f64_one_launch"]["model_eq1_eq2"] = perf_model.report(
        perf_model.kernel_model("dirac_one_launch", "f64", V, ratio, betas), t)
    # the same in FP32 (FP32 links and spinors: 384 B per site in one launch, 672 B in two)
    x32 = canon_to_field(g, psi, "f32")
    z32 = wd.wd_new_field(DIMS, "f32")
    t = ev_time(lambda: wd.wd_dslash_ex(g, x32, z32, 0.124, wd.WD_FULL, "f32", wd.WD_ONE_PASS))
    t2 = ev_time(lambda: wd.wd_dslash_ex(g, x32, z32, 0.124, wd.WD_FULL, "f32", 0))
    dvar = list(wd.wd_get_dirac_variant(g, "f32"))
    tb, why = read_traffic("f32", dvar, DIRAC_TRAFFIC, DIRAC_SOURCES)
    ratio = tb / (V * 384) if tb else 1.0
    out["dirac_full_f32_one_launch"] = {"us": round(t * 1e6, 2), "GBps": round(V * 384 / t / 1e9, 1),
                                        "frac_hbm": round(V * 384 / t / 1e9 / HBM_PEAK_GBS, 4),
                                        "bytes_per_site": 384, "variant_slices_tile": dvar,
                                        "two_pass_us": round(t2 * 1e6, 2), "one_launch_speedup": round(t2 / t, 3),
                                        "traffic_ratio_counters": round(ratio, 3) if tb else None,
                                        "model_eq1_eq2": perf_model.report(
                                            perf_model.kernel_model("dirac_one_launch", "f32", V, ratio, betas), t)}
    del x32, z32
    # one rank's share of an 8-way time decomposition (32^3 x 8 slab): the slab hop, with its two
    # time faces read from packed face buffers, and the face packing (what a GPU would send)
    R, nt = 8, DIMS[3] // 8
    vs = V // DIMS[3] // 2
    sb = nt * vs * 192
    fb = wd.wd_halo_face_bytes(DIMS, "f64")
    xin = wd.wd_new_field(DIMS, "f64", 1, wd.WD_ODD)
    wd.wd_convert(g, x[V // 2 * 192:], "f64", xin, "f64", 1, 1.0)
    slab_out = torch.empty(sb, dtype=torch.uint8, device="cuda")
    faces = [torch.empty(fb, dtype=torch.uint8, device="cuda") for _ in range(2)]
    r = 3
    slab_in = xin[r * sb:(r + 1) * sb]
    tp = ev_time(lambda: (wd.wd_halo_pack(g, slab_in, nt, 0, 0, "f64", faces[0]),
                          wd.wd_halo_pack(g, slab_in, nt, 1, 0, "f64", faces[1])))
    ts = ev_time(lambda: wd.wd_dslash_slab(g, slab_in, faces[1], faces[0], slab_out, 1.0, 0, r * nt, nt, 0, "f64"))
    # the same slab hop with nothing of it left in the caches: the 151 MB slab fits the 256 MB
    # Infinity Cache, so a 512 MiB buffer is written before every launch and events bracket
    # the launch alone
    scratch = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    tf = 0.0
    for rep in range(11):
        scratch.fill_(rep & 0xFF)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        wd.wd_dslash_slab(g, slab_in, faces[1], faces[0], slab_out, 1.0, 0, r * nt, nt, 0, "f64")
        e1.record()
        torch.cuda.synchronize()
        if rep > 0:  # the first launch warms the instruction cache
            tf += e0.elapsed_time(e1) * 1e-3
    tf /= 10
    del scratch
    out["slab_32x32x32x8_of_8_f64"] = {"hop_us": round(ts * 1e6, 2),
                                      "hop_GBps": round(nt * vs * 1152 / ts / 1e9, 1),
                                      "hop_us_cache_flushed": round(tf * 1e6, 2),
                                      "hop_GBps_cache_flushed": round(nt * vs * 1152 / tf / 1e9, 1),
                                      "pack_two_faces_us": round(tp * 1e6, 2),
                                      "face_bytes": fb, "faces_per_hop": 2,
                                      "xgmi_us_at_153GBps_per_link": round(fb / 153e9 * 1e6, 2)}
    del xin, slab_out, faces
    # the PTC network (FP32 fields, BF16 activations), one application on the full lattice
    net = wd.Ptc(g, learn.init_weights(1), "bf16")
    r32 = wd.wd_new_field(DIMS, "f32")
    wd.wd_convert(g, x, "f64", r32, "f32", 2, 1.0)
    o32 = wd.wd_new_field(DIMS, "f32")
    t = ev_time(lambda: wd.wd_ptc_apply(net, r32, o32))
    out["ptc_apply_bf16"] = {"us": round(t * 1e6, 2), "sites": V,
                             "model_eq1_eq2": perf_model.report(
                                 perf_model.kernel_model("ptc_network", "bf16", V, betas=betas), t)}
    # the even-parity application with FP16 products (BF16 fields in and out)
    xe = wd.wd_new_field(DIMS, "bf16", 1, wd.WD_EVEN)
    ye = wd.wd_new_field(DIMS, "bf16", 1, wd.WD_EVEN)
    wd.wd_convert(g, r32, "f32", xe, "bf16", 1, 1.0)
    t = ev_time(lambda: wd.wd_ptc_apply_even(net, xe, "bf16", ye, "bf16", wd.WD_PTC_FP16_PRODUCTS))
    out["ptc_apply_even_fp16_products"] = {
        "us": round(t * 1e6, 2), "sites": V // 2,
        "model_eq1_eq2": perf_model.report(
            perf_model.kernel_model("ptc_even_fp16_products", "bf16", V // 2, betas=betas), t)}
    # the same on the matrix cores (the path the mixed FGCR takes)
    t = ev_time(lambda: wd.wd_ptc_apply_even(net, xe, "bf16", ye, "bf16", wd.WD_PTC_BF16_MFMA))
    out["ptc_apply_even_bf16_mfma"] = {
        "us": round(t * 1e6, 2), "sites": V // 2,
        "model_eq1_eq2": perf_model.report(
            perf_model.kernel_model("ptc_even_bf16_mfma", "bf16", V // 2, betas=betas), t)}
    net.close()
    g.close()
    return out


def micro_leg(wd):
    """Global -> LDS block copies vs size and misalignment, fitted to the form
    of the paper's DMA model (Eq. 4): T = l0 + la * N_a + N_b * c, with N_b the
    128-byte blocks touched and N_a = N_b for a source off a 128-byte boundary
    (0 when aligned)."""
    import numpy as np

    rows = []
    for nbytes in (128, 256, 512, 1024, 2048, 4096, 8192, 16384, 32768):
        for off in (0, 4, 64, 128, 132):
            cyc, _ = wd.wd_micro_lds_copy(nbytes, off, 64)
            t = float(np.median(cyc[4:]))
            nb = -(-((off % 128) + nbytes) // 128)
            na = nb if off % 128 else 0
            rows.append((nbytes, off, nb, na, t))
    A = np.array([[1.0, r[3], r[2]] for r in rows])
    y = np.array([r[4] for r in rows])
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    fit = A @ coef
    return {"lambda0_cycles": round(float(coef[0]), 1), "lambda_a_cycles_per_block": round(float(coef[1]), 2),
            "cycles_per_128B_block": round(float(coef[2]), 2),
            "max_rel_misfit": round(float(np.max(np.abs(fit - y) / y)), 3),
            "samples": [{"bytes": r[0], "offset": r[1], "cycles": r[4]} for r in rows]}


def cpu_leg(syn, U, psi):
    """Oracle single-parity hop on the full 32^3x64 workload (one application)."""
    import numpy as np

    from oracle import wilson

    t = time.perf_counter()
    wilson.hop_parity(U, psi, 0)
    dt = time.perf_counter() - t
    vh = int(np.prod(DIMS)) // 2
    return {
        "value": round(vh * BYTES_PER_SITE["f64"] / dt / 1e9, 4),
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"one FP64 single-parity hop (numpy oracle) on the full 32^3x64 lattice, {dt:.1f} s",
        "host_cpus": os.cpu_count(),
        "host_cpu_model": _cpu_model(),
    }


def paper_context(sites_per_s):
    """The paper's Cell BE numbers for the same hop, quoted beside this run as
    context (other hardware, model estimates; not a target)."""
    # Table 1 (Sec. 5), data in main memory: the memory time per site is
    # 120 DP words (spinor in, 4 links, spinor out) = 960 B over 25.6 GB/s.
    cell_sites = 25.6e9 / 960.0
    return {
        "enhanced_cell_be_model_dp": {
            "msite_per_s": round(cell_sites / 1e6, 1),
            "gflop_per_s": round(cell_sites * 1320 / 1e9, 1),
            "eps_fp": 0.34,
            "basis": "Table 1 (Sec. 5), 8^3 slices streamed from main memory: 960 B per site at 25.6 GB/s; "
                     "model estimate for a chip not yet built",
        },
        "cell_measurements": "Sec. 5: a benchmark of the hop's access pattern ran within 20% of the memory-time "
                             "prediction; Sec. 4: caxpy at <= 4.1% of peak on PS3 / QS20 / Mercury CAB "
                             "(single-precision benchmarks)",
        "this_run_fp64_hop_msite_per_s": round(sites_per_s / 1e6, 1),
    }


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _device(torch):
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", None), "compute_units": p.multi_processor_count,
            "hbm_bytes": p.total_memory}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mrhs", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-learn", action="store_true")
    ap.add_argument("--no-kernels", action="store_true")
    ap.add_argument("--learn-steps", type=int, default=1250, help="training steps of 8 pairs (1250: 10^4 pairs)")
    ap.add_argument("--no-tune", action="store_true", help="use the default hop variant")
    ap.add_argument("--tune-table", default=TUNE_TABLE, help="JSON-lines tuning table (read, appended)")
    ap.add_argument("--retune", action="store_true", help="time all variants even if the table has an entry")
    ap.add_argument("--variant", default=None, help="force the hop variant 'block,groups,occ' (no tuning)")
    ap.add_argument("--only", choices=["f64", "f32"], default=None, help="time one precision only")
    ap.add_argument("--no-flushed", action="store_true", help="skip the cache-flushed hop timing")
    ap.add_argument("--no-betas", action="store_true", help="skip the probes of the timing model's throughputs")
    ap.add_argument("--no-mrhs-solve", action="store_true", help="multi-RHS leg: time the hops only")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (its time-slab "
              "decomposition, wd_halo_pack / wd_dslash_slab, runs a rank's share on one GPU).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0710_2442_amd as wd
    import synthetic as syn

    torch.cuda.set_device(0)
    gseed, sseed = syn.CONFIG_SEEDS["dslash_32x32x32x64"]
    t = time.perf_counter()
    U = syn.gauge_field(DIMS, 0.3, gseed)
    psi = syn.gaussian_spinor(DIMS, sseed)
    log(f"inputs generated in {time.perf_counter() - t:.1f} s")

    vh = int(np.prod(DIMS)) // 2
    betas = None if args.no_betas else measure_betas(wd)
    results = {}
    precs = [args.only] if args.only else ["f64", "f32"]
    for prec in precs:
        g = wd.Gauge(U, DIMS, -1, prec)
        if args.variant:
            vb, vg, vo = (int(x) for x in args.variant.split(","))
            wd.wd_set_dslash_variant(g, prec, vb, vg, vo)
        elif not args.no_tune:
            tb, tg, to, tus = wd.wd_tune_dslash(g, prec, args.tune_table, force=args.retune)
            log(f"tuned hop {prec}: block {tb}, XCD groups {tg}, occ {to} ({tus:.1f} us in the tuner)")
        sec, n, ms = time_hop(wd, torch, g, psi, prec, args.steps, args.warmup)
        gbs = vh * BYTES_PER_SITE[prec] / sec / 1e9
        results[prec] = {"sec_per_launch": sec, "gbs": gbs, "ms_total": ms, "launches": n,
                         "variant": list(wd.wd_get_dslash_variant(g, prec))}
        log(f"hop {prec}: {sec * 1e6:.1f} us/launch, {gbs:.0f} GB/s algorithmic, "
            f"{100 * gbs / HBM_PEAK_GBS:.1f}% of 8 TB/s")
        if not args.no_flushed:
            fsec = time_hop_flushed(wd, torch, g, psi, prec)
            results[prec]["flushed_sec"] = fsec
            log(f"hop {prec} after a 512 MiB cache flush: {fsec * 1e6:.1f} us/launch, "
                f"{100 * vh * BYTES_PER_SITE[prec] / fsec / 1e9 / HBM_PEAK_GBS:.1f}% of 8 TB/s")
        g.close()
        torch.cuda.empty_cache()

    if args.calib_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    head = "f64" if "f64" in results else precs[0]
    r = results[head]
    traffic, why = read_traffic(head, r["variant"])
    roof = {
        "bound": "hbm",
        "achieved": round(r["gbs"], 2),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(r["gbs"] / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": f"k_dslash<{head}> single-parity hop, 32^3x64, 1,048,576 output sites per launch",
        "algorithmic_bytes_per_launch": vh * BYTES_PER_SITE[head],
        "avg_launch_us": round(r["sec_per_launch"] * 1e6, 2),
        "variant_block_groups_occ": r["variant"],
    }
    if traffic is None:
        roof["traffic_note"] = why
    if "flushed_sec" in r:
        # the same kernel with L2 and the Infinity Cache emptied before each launch
        fg = vh * BYTES_PER_SITE[head] / r["flushed_sec"] / 1e9
        roof["cache_flushed"] = {"avg_launch_us": round(r["flushed_sec"] * 1e6, 2), "achieved": round(fg, 2),
                                 "frac": round(fg / HBM_PEAK_GBS, 4),
                                 "note": "512 MiB written before every launch; the headline is the solver's "
                                         "ping-pong pattern, where an output may be re-read from the caches"}
    from paper_0710_2442_amd import perf_model

    ratio = traffic / roof["algorithmic_bytes_per_launch"] if traffic else None
    roof["model_eq1_eq2"] = perf_model.report(
        perf_model.kernel_model("hop", head, vh, ratio or 1.0, betas), r["sec_per_launch"])
    line = {
        "metric": "dslash_hbm_GBps",
        "value": round(r["gbs"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_total"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic: random SU(3) links exp(i*0.3*H), Gaussian spinors, seeded",
        "config": {
            "workload": "single-parity Wilson hop (Eq. 3), 32^3x64, 12-real links, even+odd per step",
            "lattice": "32x32x32x64",
            "sites_per_launch": vh,
            "parallelism": "single GPU",
        },
        "roofline": roof,
        "device": _device(torch),
        "paper_context": paper_context(vh / r["sec_per_launch"]),
    }
    if "f32" in results and head != "f32":
        line["f32"] = {"value": round(results["f32"]["gbs"], 2), "unit": "GB/s",
                       "frac": round(results["f32"]["gbs"] / HBM_PEAK_GBS, 4),
                       "avg_launch_us": round(results["f32"]["sec_per_launch"] * 1e6, 2)}
        if "flushed_sec" in results["f32"]:
            fg = vh * BYTES_PER_SITE["f32"] / results["f32"]["flushed_sec"] / 1e9
            line["f32"]["cache_flushed"] = {"avg_launch_us": round(results["f32"]["flushed_sec"] * 1e6, 2),
                                            "frac": round(fg / HBM_PEAK_GBS, 4)}
    if not args.no_solve:
        sl = solve_leg(wd, torch, syn, table=args.tune_table, retune=args.retune)
        if head == "f64":
            # Eqs. 1-2 for one eo-CGLS iteration against the measured time per iteration
            cg = perf_model.cg_iteration_model(vh, "f64", ratio or 1.0, betas)
            meas = sl["fp64_cg"]["seconds"] / sl["fp64_cg"]["iters"]
            sl["fp64_cg"]["model_eq1_eq2"] = {
                "bytes_per_site": perf_model.cg_iteration_bytes("f64"),
                "T_hops_us": round(cg["T_hops"] * 1e6, 1), "T_blas_us": round(cg["T_blas"] * 1e6, 1),
                "T_iter_us": round(cg["T_iter"] * 1e6, 1), "measured_us_per_iter": round(meas * 1e6, 1),
                "measured_over_model": round(meas / cg["T_iter"], 3)}
        line["solve_32x32x32x64_kappa0124"] = sl
    if not args.no_mrhs:
        line["mrhs_24x24x24x48_12_point_sources"] = mrhs_leg(wd, torch, syn, args.tune_table, args.retune, betas,
                                                             solves=not args.no_mrhs_solve)
    if not args.no_batch:
        line["batch_8_lattices_689408_sites"] = batch_leg(wd, torch, syn, args.tune_table, args.retune, betas)
    if not args.no_learn:
        line["learned_ptc_fgcr_32x32x32x64"] = learned_leg(wd, torch, syn, args.learn_steps, args.tune_table,
                                                          args.retune)
    if not args.no_kernels:
        line["kernels_32x32x32x64"] = kernels_leg(wd, torch, syn, U, psi, betas)
        line["micro_lds_copy_eq4_fit"] = micro_leg(wd)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_leg(syn, U, psi)
    if betas:
        line["model_betas_TBps"] = {k: round(v / 1e12, 3) for k, v in betas.items()}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
