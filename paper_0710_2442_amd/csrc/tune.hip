// Autotuner for the single-RHS and multi-RHS hops (block size, block -> tile
// order, register budget, store policy, resident-block cap, link preloading;
// RHS per lane for the multi-RHS hop).
//
// Each candidate is first checked for parity -- its output must equal the
// reference variant's byte for byte, which holds because every site's
// arithmetic is the same in every variant (the comparison runs on the
// device) -- and then timed with HIP events.  The fastest valid candidate is stored in the handle
// and, if a cache path is given, appended to a JSON-lines cache keyed by
// (architecture, kernel, precision, lattice; and the number of right-hand
// sides for the multi-RHS hop).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <algorithm>
#include <array>
#include <vector>

#include "wd_internal.h"
#include "wd_solver.h"

namespace wd {

// nrhs > 0: the multi-RHS hop; nrhs < 0: the one-launch D_W
static std::string tune_key(const wd_gauge *g, wd_prec prec, int nrhs = 0) {
  hipDeviceProp_t prop;
  char arch[64] = "unknown";
  if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) {
    snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
    char *colon = strchr(arch, ':');
    if (colon) *colon = 0;
  }
  char kern[32] = "hop";
  if (nrhs > 0) snprintf(kern, sizeof kern, "hop_mrhs%d", nrhs);
  if (nrhs < 0) snprintf(kern, sizeof kern, "dirac");
  char buf[160];
  snprintf(buf, sizeof buf, "%s/%s/p%d/%dx%dx%dx%d", arch, kern, (int)prec, g->dims[0], g->dims[1], g->dims[2],
           g->dims[3]);
  return buf;
}

// A cache line: {"key": K, "block": B, "groups": G, "<third>": V, "us": T}
// with <third> "occ" (single-RHS hop) or "rpl" (multi-RHS hop).
static bool cache_lookup(const char *path, const std::string &key, int &bs, int &groups, int &occ, double &us,
                         const char *third = "occ") {
  FILE *f = fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    char k[200];
    int b, gr, oc;
    double t;
    char fmt[128];
    snprintf(fmt, sizeof fmt, " {\"key\": \"%%199[^\"]\", \"block\": %%d, \"groups\": %%d, \"%s\": %%d, \"us\": %%lf",
             third);
    if (sscanf(line, fmt, k, &b, &gr, &oc, &t) == 5 && key == k) {
      bs = b; groups = gr; occ = oc; us = t; found = true;  // last entry wins
    }
  }
  fclose(f);
  return found;
}

static void cache_append(const char *path, const std::string &key, int bs, int groups, int occ, double us,
                         const char *third = "occ") {
  FILE *f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "{\"key\": \"%s\", \"block\": %d, \"groups\": %d, \"%s\": %d, \"us\": %.3f}\n", key.c_str(), bs,
          groups, third, occ, us);
  fclose(f);
}

// occ value: bits 0..7 register budget (0 or 4), WD_TUNE_CACHED_STORE,
// WD_TUNE_PRELOAD_LINKS, log2 of the sites per lane at WD_TUNE_SPL_SHIFT and
// the dynamic LDS per block in KiB at WD_TUNE_LDS_SHIFT (0..64)
static wd_status decode_occ(int occ, int &o, int &nts, int &lkb, int &pre, int &spl, int &stage) {
  o = occ & 0xff;
  nts = (occ & WD_TUNE_CACHED_STORE) ? 0 : 1;
  pre = (occ & WD_TUNE_PRELOAD_LINKS) ? 1 : 0;
  stage = (occ & WD_TUNE_STAGE_LDS) ? 1 : 0;
  lkb = (occ >> WD_TUNE_LDS_SHIFT) & 0xff;
  const int sp = (occ >> WD_TUNE_SPL_SHIFT) & 3;
  spl = 1 << sp;
  const int rest = occ & ~(0xff | WD_TUNE_CACHED_STORE | WD_TUNE_PRELOAD_LINKS | WD_TUNE_STAGE_LDS |
                           (3 << WD_TUNE_SPL_SHIFT) | (0xff << WD_TUNE_LDS_SHIFT));
  if ((o != 0 && o != 4) || rest || lkb > 64 || sp == 3)
    return set_error(WD_ERR_ARG,
                     "occ = 0x%x: register budget 0 or 4, | WD_TUNE_CACHED_STORE, | WD_TUNE_PRELOAD_LINKS, "
                     "| WD_TUNE_STAGE_LDS, | (0, 1, 2) << WD_TUNE_SPL_SHIFT, | KiB << %d (<= 64)",
                     occ, WD_TUNE_LDS_SHIFT);
  if (stage && (pre || spl != 1))
    return set_error(WD_ERR_ARG, "occ = 0x%x: LDS staging takes one site per lane and no link preloading", occ);
  return WD_OK;
}

static int log2i(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

static int encode_occ(const wd_gauge *g, wd_prec prec) {
  return g->hop_occ[prec] | (g->hop_ntst[prec] ? 0 : WD_TUNE_CACHED_STORE) |
         (g->hop_pre[prec] ? WD_TUNE_PRELOAD_LINKS : 0) | (g->hop_stage[prec] ? WD_TUNE_STAGE_LDS : 0) |
         (log2i(g->hop_spl[prec]) << WD_TUNE_SPL_SHIFT) | ((g->hop_lds[prec] / 1024) << WD_TUNE_LDS_SHIFT);
}

// *differ = 1 if the n 16-byte words of a and b are not all equal (vector
// stores only; the flag is cleared by the caller).
__global__ __launch_bounds__(256) void k_differ(const uint4 *a, const uint4 *b, size_t n, int *differ) {
  bool d = false;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const uint4 x = a[i], y = b[i];
    d |= (x.x != y.x) | (x.y != y.y) | (x.z != y.z) | (x.w != y.w);
  }
  if (d) *differ = 1;
}

// true when the hb bytes at a and b are equal (synchronises st)
static wd_status same_bytes(const void *a, const void *b, size_t hb, int *flag_dev, bool &same, hipStream_t st) {
  WD_HIP(hipMemsetAsync(flag_dev, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_differ, dim3(1024), dim3(256), 0, st, (const uint4 *)a, (const uint4 *)b, hb / 16, flag_dev);
  WD_HIP(hipGetLastError());
  int h = 1;
  WD_HIP(hipMemcpyAsync(&h, flag_dev, sizeof(int), hipMemcpyDeviceToHost, st));
  WD_HIP(hipStreamSynchronize(st));
  same = (h == 0);
  return WD_OK;
}

}  // namespace wd

using namespace wd;

extern "C" {

wd_status wd_set_dslash_variant(wd_gauge *g, wd_prec prec, int block, int groups, int occ) {
  if (!g) return set_error(WD_ERR_ARG, "gauge handle is NULL");
  if ((int)prec < 0 || (int)prec > 3) return set_error(WD_ERR_PREC, "prec = %d", (int)prec);
  if (block < 64 || !dslash_variant_ok(g->geom, block, groups))
    return set_error(WD_ERR_ARG, "variant (block %d, groups %d) does not fit this lattice", block, groups);
  int o, nts, lkb, pre, spl, stage;
  WD_TRY(decode_occ(occ, o, nts, lkb, pre, spl, stage));
  if (!dslash_variant_ok(g->geom, block, groups, spl))
    return set_error(WD_ERR_ARG, "variant (block %d, groups %d, %d sites per lane) does not fit this lattice", block,
                     groups, spl);
  if (pre && prec == WD_F64) return set_error(WD_ERR_ARG, "link preloading is for FP32-arithmetic hops");
  if (stage && prec != WD_F64 && prec != WD_F32)
    return set_error(WD_ERR_ARG, "LDS staging is for FP64 and FP32 storage");
  if (stage && !dslash_stage_ok(g->geom, block))
    return set_error(WD_ERR_ARG, "LDS staging needs tiles of whole x1 rows of one plane, or whole planes (block %d)",
                     block);
  if (stage && dslash_stage_lds_bytes(g->geom, block, prec) + (size_t)lkb * 1024 > (size_t)g->lds_per_block)
    return set_error(WD_ERR_ARG, "LDS staging of %d-site tiles needs %zu bytes of LDS, the device allows %d", block,
                     dslash_stage_lds_bytes(g->geom, block, prec) + (size_t)lkb * 1024, g->lds_per_block);
  g->hop_block[prec] = block;
  g->hop_groups[prec] = groups;
  g->hop_occ[prec] = o;
  g->hop_ntst[prec] = nts;
  g->hop_lds[prec] = lkb * 1024;
  g->hop_pre[prec] = pre;
  g->hop_spl[prec] = spl;
  g->hop_stage[prec] = stage;
  return WD_OK;
}

wd_status wd_set_dslash_mrhs_variant(wd_gauge *g, wd_prec prec, int block, int groups, int rpl) {
  if (!g) return set_error(WD_ERR_ARG, "gauge handle is NULL");
  if ((int)prec < 0 || (int)prec > 3) return set_error(WD_ERR_PREC, "prec = %d", (int)prec);
  if (prec == WD_F64) {
    const bool tiles16 = block == 16 && rpl == 4 && groups > -100 && dslash_variant_ok(g->geom, 16, groups);
    const bool box = (block == 64 || block == 128 || block == 256) && rpl == 1 && mrhs_box_ok(g->geom, block, groups);
    if (!tiles16 && !box)
      return set_error(WD_ERR_ARG,
                       "FP64 multi-RHS variant: block 16, rpl 4 and a groups value that fits, or block 64..256, "
                       "rpl 1 and a box order (groups -101 .. -108) that fits");
  } else {
    if (block != 64 && block != 128 && block != 256)
      return set_error(WD_ERR_ARG, "multi-RHS block %d (64, 128 or 256)", block);
    if (rpl < 1 || rpl > 16) return set_error(WD_ERR_ARG, "multi-RHS rpl %d (1..16)", rpl);
    if (!dslash_variant_ok(g->geom, block, groups) && !mrhs_box_ok(g->geom, block, groups))
      return set_error(WD_ERR_ARG, "variant (block %d, groups %d) does not fit this lattice", block, groups);
  }
  g->mrhs_block[prec] = block;
  g->mrhs_groups[prec] = groups;
  g->mrhs_rpl[prec] = rpl;
  return WD_OK;
}

wd_status wd_get_dslash_mrhs_variant(const wd_gauge *g, wd_prec prec, int *block, int *groups, int *rpl) {
  if (!g || !block || !groups || !rpl) return set_error(WD_ERR_ARG, "NULL argument");
  if ((int)prec < 0 || (int)prec > 3) return set_error(WD_ERR_PREC, "prec = %d", (int)prec);
  *block = g->mrhs_block[prec];
  *groups = g->mrhs_groups[prec];
  *rpl = g->mrhs_rpl[prec];
  return WD_OK;
}

wd_status wd_get_dslash_variant(const wd_gauge *g, wd_prec prec, int *block, int *groups, int *occ) {
  if (!g || !block || !groups || !occ) return set_error(WD_ERR_ARG, "NULL argument");
  if ((int)prec < 0 || (int)prec > 3) return set_error(WD_ERR_PREC, "prec = %d", (int)prec);
  *block = g->hop_block[prec];
  *groups = g->hop_groups[prec];
  *occ = encode_occ(g, prec);
  return WD_OK;
}

wd_status wd_tune_dslash(wd_gauge *g, wd_prec prec, const char *cache_path, int force, int *out_block,
                         int *out_groups, int *out_occ, double *out_us) {
  if (!g) return set_error(WD_ERR_ARG, "gauge handle is NULL");
  if ((int)prec < 0 || (int)prec > 3) return set_error(WD_ERR_PREC, "prec = %d", (int)prec);
  WD_HIP(hipSetDevice(g->device));
  const std::string key = tune_key(g, prec);
  int bs = 256, groups = 0, occ = 0;
  double best_us = -1.0;
  if (cache_path && !force && cache_lookup(cache_path, key, bs, groups, occ, best_us) &&
      dslash_variant_ok(g->geom, bs, groups) && wd_set_dslash_variant(g, prec, bs, groups, occ) == WD_OK) {
  } else {
    const Geom &G = g->geom;
    const size_t hb = half_bytes(G, prec);
    const size_t V = 2 * (size_t)G.vh;
    hipStream_t st = g->own_stream;
    void *in = nullptr, *ref = nullptr, *cand = nullptr, *canon = nullptr;
    int *flag = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    wd_status rc = WD_OK;
    do {
      if ((rc = hip_check(hipMalloc(&in, hb), "tune alloc")) != WD_OK) break;
      if ((rc = hip_check(hipMalloc(&ref, hb), "tune alloc")) != WD_OK) break;
      if ((rc = hip_check(hipMalloc(&cand, hb), "tune alloc")) != WD_OK) break;
      if ((rc = hip_check(hipMalloc(&canon, V * 24 * sizeof(double)), "tune alloc")) != WD_OK) break;
      if ((rc = hip_check(hipMalloc(&flag, 256), "tune alloc")) != WD_OK) break;
      {
        // deterministic input: a simple integer hash mapped to [-1, 1)
        std::vector<double> h(V * 24);
        uint64_t s = 0x9E3779B97F4A7C15ull;
        for (size_t n = 0; n < h.size(); ++n) {
          s ^= s << 13; s ^= s >> 7; s ^= s << 17;
          h[n] = (double)(s >> 11) * (2.0 / 9007199254740992.0) - 1.0;
        }
        if ((rc = hip_check(hipMemcpy(canon, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice),
                            "tune upload")) != WD_OK)
          break;
      }
      if ((rc = launch_pack_spinor(g, canon, in, WD_ODD, prec, st)) != WD_OK) break;
      if ((rc = hip_check(hipEventCreate(&e0), "event")) != WD_OK) break;
      if ((rc = hip_check(hipEventCreate(&e1), "event")) != WD_OK) break;
      const int save_b = g->hop_block[prec], save_g = g->hop_groups[prec], save_o = g->hop_occ[prec];
      const int save_n = g->hop_ntst[prec], save_l = g->hop_lds[prec], save_p = g->hop_pre[prec];
      const int save_s = g->hop_spl[prec], save_t = g->hop_stage[prec];
      DslashArgs a;
      a.in = in; a.a = 1.0; a.parity = WD_EVEN;
      // reference variant
      g->hop_block[prec] = 256; g->hop_groups[prec] = 0; g->hop_occ[prec] = 0; g->hop_ntst[prec] = 1;
      g->hop_lds[prec] = 0; g->hop_pre[prec] = 0; g->hop_spl[prec] = 1; g->hop_stage[prec] = 0;
      a.out = ref;
      if ((rc = launch_dslash(g, prec, a, st)) != WD_OK) break;
      const int blocks[] = {64, 128, 256, 512};
      const int grps[] = {0, 2, 4, 8, 16, -8, -16, -101, -102, -104, -108};
      best_us = 1e30;
      int nbest_b = 256, nbest_g = 0, nbest_o = 0, nbest_n = 1, nbest_l = 0, nbest_p = 0, nbest_s = 1, nbest_t = 0;
      size_t lds_max = 65536;
      {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) lds_max = prop.sharedMemPerBlock;
      }
      // the candidates, listed first so that one loop runs them and a failure
      // ends the whole search
      struct Cand { int spl, pre, lkb, nts, oc, b, gr, stg; };
      std::vector<Cand> cands;
      for (int stg : {0, 1})
        for (int spl : {1, 2, 4})
          for (int pre : {0, 1})
            for (int lkb : {0, 24, 40, 60})
              for (int nts : {1, 0})
                for (int oc : {0, 4})
                  for (int b : blocks)
                    for (int gr : grps) {
                      if (!dslash_variant_ok(G, b, gr, spl)) continue;
                      if (pre && prec == WD_F64) continue;
                      if (oc == 4 && lkb != 0) continue;  // both only lower occupancy; keep the grid small
                      if ((size_t)lkb * 1024 + 1024 > lds_max) continue;
                      if (stg && (spl != 1 || pre || lkb || (prec != WD_F64 && prec != WD_F32))) continue;
                      if (stg && (!dslash_stage_ok(G, b) || dslash_stage_lds_bytes(G, b, prec) > (size_t)g->lds_per_block))
                        continue;
                      cands.push_back({spl, pre, lkb, nts, oc, b, gr, stg});
                    }
      for (const Cand &c : cands) {
        const int spl = c.spl, pre = c.pre, lkb = c.lkb, nts = c.nts, oc = c.oc, b = c.b, gr = c.gr;
        g->hop_block[prec] = b; g->hop_groups[prec] = gr; g->hop_occ[prec] = oc; g->hop_ntst[prec] = nts;
        g->hop_lds[prec] = lkb * 1024;
        g->hop_pre[prec] = pre;
        g->hop_spl[prec] = spl;
        g->hop_stage[prec] = c.stg;
        if ((rc = launch_pack_spinor(g, canon, in, WD_ODD, prec, st)) != WD_OK) break;
        a.out = cand;
        if ((rc = hip_check(hipMemsetAsync(cand, 0xff, hb, st), "memset")) != WD_OK) break;
        if ((rc = launch_dslash(g, prec, a, st)) != WD_OK) break;
        bool same = false;
        if ((rc = same_bytes(ref, cand, hb, flag, same, st)) != WD_OK) break;
        if (!same) continue;  // parity first
        // time the pattern of a solver: even and odd hops alternate, so the
        // two parities' link arrays stream through the caches in turn
        const int reps = 6;
        DslashArgs b2 = a;
        b2.in = cand; b2.out = in; b2.parity = WD_ODD;
        auto pair = [&]() { (void)launch_dslash(g, prec, a, st); (void)launch_dslash(g, prec, b2, st); };
        for (int w = 0; w < 2; ++w) pair();
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps; ++r) pair();
        (void)hipEventRecord(e1, st);
        if ((rc = hip_check(hipEventSynchronize(e1), "tune timing")) != WD_OK) break;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double us = 1e3 * ms / (2 * reps);
        if (getenv("WD_TUNE_VERBOSE"))
          fprintf(stderr, "tune %s: block %d groups %d occ %d ntstore %d lds %dK preload %d spl %d stage %d: %.2f us\n",
                  key.c_str(), b, gr, oc, nts, lkb, pre, spl, c.stg, us);
        if (us < best_us) {
          best_us = us; nbest_b = b; nbest_g = gr; nbest_o = oc; nbest_n = nts; nbest_l = lkb; nbest_p = pre;
          nbest_s = spl; nbest_t = c.stg;
        }
      }
      if (rc != WD_OK) {
        g->hop_block[prec] = save_b; g->hop_groups[prec] = save_g; g->hop_occ[prec] = save_o;
        g->hop_ntst[prec] = save_n;
        g->hop_lds[prec] = save_l;
        g->hop_pre[prec] = save_p;
        g->hop_spl[prec] = save_s;
        g->hop_stage[prec] = save_t;
        break;
      }
      g->hop_block[prec] = nbest_b;
      g->hop_groups[prec] = nbest_g;
      g->hop_occ[prec] = nbest_o;
      g->hop_ntst[prec] = nbest_n;
      g->hop_lds[prec] = nbest_l * 1024;
      g->hop_pre[prec] = nbest_p;
      g->hop_spl[prec] = nbest_s;
      g->hop_stage[prec] = nbest_t;
      bs = nbest_b; groups = nbest_g;
      occ = encode_occ(g, prec);
      if (cache_path) cache_append(cache_path, key, bs, groups, occ, best_us);
    } while (0);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (in) (void)hipFree(in);
    if (ref) (void)hipFree(ref);
    if (cand) (void)hipFree(cand);
    if (canon) (void)hipFree(canon);
    if (flag) (void)hipFree(flag);
    if (rc != WD_OK) return rc;
  }
  if (out_block) *out_block = bs;
  if (out_groups) *out_groups = groups;
  if (out_occ) *out_occ = occ;
  if (out_us) *out_us = best_us;
  return WD_OK;
}

// Multi-RHS hop: tune the block size (FP32 arithmetic: 64..256 sites; FP64:
// fixed 16-site tiles), the right-hand sides per lane (FP32 arithmetic) and
// the block -> tile order for nrhs right-hand sides; candidates checked byte
// for byte against the linear 128-site, 4-RHS (FP64: 16-site) variant.
wd_status wd_tune_dslash_mrhs(wd_gauge *g, wd_prec prec, int nrhs, const char *cache_path, int force,
                              int *out_block, int *out_groups, int *out_rpl, double *out_us) {
  if (!g) return set_error(WD_ERR_ARG, "gauge handle is NULL");
  if ((int)prec < 0 || (int)prec > 3) return set_error(WD_ERR_PREC, "prec = %d", (int)prec);
  if (nrhs < 1 || nrhs > 64) return set_error(WD_ERR_ARG, "nrhs = %d", nrhs);
  WD_HIP(hipSetDevice(g->device));
  const std::string key = tune_key(g, prec, nrhs);
  {
    int cb, cg, cr;
    double cus;
    if (cache_path && !force && cache_lookup(cache_path, key, cb, cg, cr, cus, "rpl") &&
        wd_set_dslash_mrhs_variant(g, prec, cb, cg, cr) == WD_OK) {
      if (out_block) *out_block = cb;
      if (out_groups) *out_groups = cg;
      if (out_rpl) *out_rpl = cr;
      if (out_us) *out_us = cus;
      return WD_OK;
    }
  }
  const Geom &G = g->geom;
  const size_t hb = half_bytes(G, prec) * (size_t)nrhs;
  hipStream_t st = g->own_stream;
  void *in = nullptr, *ref = nullptr, *cand = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  wd_status rc = WD_OK;
  int *flag = nullptr;
  const int save = g->mrhs_groups[prec], save_b = g->mrhs_block[prec], save_r = g->mrhs_rpl[prec];
  const int ref_b = (prec == WD_F64) ? 16 : 128;
  int best_g = 0, best_b = ref_b, best_r = 4;
  double best_us = 1e30;
  do {
    if ((rc = hip_check(hipMalloc(&in, hb), "tune alloc")) != WD_OK) break;
    if ((rc = hip_check(hipMalloc(&ref, hb), "tune alloc")) != WD_OK) break;
    if ((rc = hip_check(hipMalloc(&cand, hb), "tune alloc")) != WD_OK) break;
    if ((rc = hip_check(hipMalloc(&flag, 256), "tune alloc")) != WD_OK) break;
    {
      std::vector<unsigned char> h(hb);
      uint64_t s = 0x243F6A8885A308D3ull;
      for (size_t n = 0; n < hb; ++n) {
        s ^= s << 13; s ^= s >> 7; s ^= s << 17;
        h[n] = (unsigned char)(s >> 56);
      }
      // keep every value a finite number in every precision: clear the exponent MSBs
      if (prec == WD_F64) for (size_t n = 7; n < hb; n += 8) h[n] &= 0x3f;
      else for (size_t n = 1; n < hb; n += 2) h[n] &= 0x3f;
      if ((rc = hip_check(hipMemcpy(in, h.data(), hb, hipMemcpyHostToDevice), "upload")) != WD_OK) break;
    }
    if ((rc = hip_check(hipEventCreate(&e0), "event")) != WD_OK) break;
    if ((rc = hip_check(hipEventCreate(&e1), "event")) != WD_OK) break;
    g->mrhs_groups[prec] = 0;
    g->mrhs_block[prec] = ref_b;
    g->mrhs_rpl[prec] = 4;
    if ((rc = launch_dslash_mrhs(g, prec, in, ref, 1.0, WD_EVEN, 0, nrhs, st)) != WD_OK) break;
    std::vector<int> blocks, rpls;
    if (prec == WD_F64) {
      blocks = {16, 64, 128, 256};
      rpls = {1, 4};
    } else {
      blocks = {64, 128, 256};
      for (int r : {1, 2, 3, 4, 6, 8, 12, 16})
        if (r <= nrhs) rpls.push_back(r);
    }
    // candidates listed first: one loop runs them, and a failure ends the search
    std::vector<std::array<int, 3>> cands;
    for (int rp : rpls)
      for (int bs : blocks)
        for (int gr : {0, 2, 4, 8, -8, -16, -101, -102, -104, -108}) {
          const bool box = gr <= -100;
          bool ok;
          if (prec == WD_F64)  // 16-site tiles with 4 RHS per group, or one RHS per block in box order
            ok = box ? (bs != 16 && rp == 1 && mrhs_box_ok(G, bs, gr))
                     : (bs == 16 && rp == 4 && dslash_variant_ok(G, bs, gr));
          else
            ok = box ? mrhs_box_ok(G, bs, gr) : dslash_variant_ok(G, bs, gr);
          if (ok) cands.push_back({rp, bs, gr});
        }
    for (const auto &c : cands) {
      const int rp = c[0], bs = c[1], gr = c[2];
      g->mrhs_groups[prec] = gr;
      g->mrhs_block[prec] = bs;
      g->mrhs_rpl[prec] = rp;
      if ((rc = hip_check(hipMemsetAsync(cand, 0xff, hb, st), "memset")) != WD_OK) break;
      if ((rc = launch_dslash_mrhs(g, prec, in, cand, 1.0, WD_EVEN, 0, nrhs, st)) != WD_OK) break;
      bool same = false;
      if ((rc = same_bytes(ref, cand, hb, flag, same, st)) != WD_OK) break;
      if (!same) continue;
      const int reps = 6;
      for (int w = 0; w < 2; ++w) (void)launch_dslash_mrhs(g, prec, in, cand, 1.0, WD_EVEN, 0, nrhs, st);
      (void)hipEventRecord(e0, st);
      for (int r = 0; r < reps; ++r) (void)launch_dslash_mrhs(g, prec, in, cand, 1.0, WD_EVEN, 0, nrhs, st);
      (void)hipEventRecord(e1, st);
      if ((rc = hip_check(hipEventSynchronize(e1), "tune timing")) != WD_OK) break;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double us = 1e3 * ms / reps;
      if (getenv("WD_TUNE_VERBOSE"))
        fprintf(stderr, "tune mrhs p%d nrhs %d: block %d groups %d rpl %d: %.2f us\n", (int)prec, nrhs, bs, gr, rp,
                us);
      if (us < best_us) { best_us = us; best_g = gr; best_b = bs; best_r = rp; }
    }
  } while (0);
  g->mrhs_groups[prec] = (rc == WD_OK) ? best_g : save;
  g->mrhs_block[prec] = (rc == WD_OK) ? best_b : save_b;
  g->mrhs_rpl[prec] = (rc == WD_OK) ? best_r : save_r;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (in) (void)hipFree(in);
  if (ref) (void)hipFree(ref);
  if (cand) (void)hipFree(cand);
  if (flag) (void)hipFree(flag);
  if (rc != WD_OK) return rc;
  if (cache_path) cache_append(cache_path, key, best_b, best_g, best_r, best_us, "rpl");
  if (out_block) *out_block = best_b;
  if (out_rpl) *out_rpl = best_r;
  if (out_groups) *out_groups = best_g;
  if (out_us) *out_us = best_us;
  return WD_OK;
}

wd_status wd_set_dirac_variant(wd_gauge *g, wd_prec prec, int slices, int tile) {
  if (!g) return set_error(WD_ERR_ARG, "gauge handle is NULL");
  if ((int)prec < 0 || (int)prec > 3) return set_error(WD_ERR_PREC, "prec = %d", (int)prec);
  if (!dirac_variant_ok(g, prec, slices, tile))
    return set_error(WD_ERR_ARG, "one-launch D_W variant: slices %d, tile %d does not fit %dx%dx%dx%d", slices,
                     tile, g->dims[0], g->dims[1], g->dims[2], g->dims[3]);
  g->dirac_slices[prec] = slices;
  g->dirac_tile[prec] = tile;
  return WD_OK;
}

wd_status wd_get_dirac_variant(const wd_gauge *g, wd_prec prec, int *slices, int *tile) {
  if (!g) return set_error(WD_ERR_ARG, "gauge handle is NULL");
  if ((int)prec < 0 || (int)prec > 3) return set_error(WD_ERR_PREC, "prec = %d", (int)prec);
  if (slices) *slices = g->dirac_slices[prec];
  if (tile) *tile = g->dirac_tile[prec];
  return WD_OK;
}

wd_status wd_tune_dirac(wd_gauge *g, wd_prec prec, const char *cache_path, int force, int *out_slices,
                        int *out_tile, double *out_us) {
  if (!g) return set_error(WD_ERR_ARG, "gauge handle is NULL");
  if ((int)prec < 0 || (int)prec > 3) return set_error(WD_ERR_PREC, "prec = %d", (int)prec);
  WD_HIP(hipSetDevice(g->device));
  const std::string key = tune_key(g, prec, -1);
  {
    int cb, ct, cs;
    double cus;
    if (cache_path && !force && cache_lookup(cache_path, key, cb, ct, cs, cus, "slices") &&
        wd_set_dirac_variant(g, prec, cs, ct) == WD_OK) {
      if (out_slices) *out_slices = cs;
      if (out_tile) *out_tile = ct;
      if (out_us) *out_us = cus;
      return WD_OK;
    }
  }
  const Geom &G = g->geom;
  const size_t fb = 2 * half_bytes(G, prec);
  hipStream_t st = g->own_stream;
  void *in = nullptr, *ref = nullptr, *cand = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  wd_status rc = WD_OK;
  int *flag = nullptr;
  const int save_s = g->dirac_slices[prec], save_t = g->dirac_tile[prec];
  int best_s = save_s, best_t = save_t;
  double best_us = 1e30;
  DiracArgs a;
  a.a = -0.124;
  do {
    if ((rc = hip_check(hipMalloc(&in, fb), "tune alloc")) != WD_OK) break;
    if ((rc = hip_check(hipMalloc(&ref, fb), "tune alloc")) != WD_OK) break;
    if ((rc = hip_check(hipMalloc(&cand, fb), "tune alloc")) != WD_OK) break;
    if ((rc = hip_check(hipMalloc(&flag, 256), "tune alloc")) != WD_OK) break;
    {
      std::vector<unsigned char> h(fb);
      uint64_t s = 0x13198A2E03707344ull;
      for (size_t n = 0; n < fb; ++n) {
        s ^= s << 13; s ^= s >> 7; s ^= s << 17;
        h[n] = (unsigned char)(s >> 56);
      }
      // keep every value a finite number in every precision: clear the exponent MSBs
      if (prec == WD_F64) for (size_t n = 7; n < fb; n += 8) h[n] &= 0x3f;
      else for (size_t n = 1; n < fb; n += 2) h[n] &= 0x3f;
      if ((rc = hip_check(hipMemcpy(in, h.data(), fb, hipMemcpyHostToDevice), "upload")) != WD_OK) break;
    }
    if ((rc = hip_check(hipEventCreate(&e0), "event")) != WD_OK) break;
    if ((rc = hip_check(hipEventCreate(&e1), "event")) != WD_OK) break;
    a.in = in;
    a.X = in;
    a.out = ref;
    if ((rc = launch_dirac(g, prec, a, st)) != WD_OK) break;
    std::vector<std::array<int, 2>> cands;
    for (int tile : {3, 2, 0})
      for (int sl = 8;; sl *= 2) {
        const int S = std::min(sl, G.L[3]);
        if (dirac_variant_ok(g, prec, S, tile)) cands.push_back({S, tile});
        if (S == G.L[3]) break;
      }
    a.out = cand;
    for (const auto &c : cands) {
      g->dirac_slices[prec] = c[0];
      g->dirac_tile[prec] = c[1];
      if ((rc = hip_check(hipMemsetAsync(cand, 0xff, fb, st), "memset")) != WD_OK) break;
      if ((rc = launch_dirac(g, prec, a, st)) != WD_OK) break;
      bool same = false;
      if ((rc = same_bytes(ref, cand, fb, flag, same, st)) != WD_OK) break;
      if (!same) continue;
      const int reps = 6;
      for (int w = 0; w < 2; ++w) (void)launch_dirac(g, prec, a, st);
      (void)hipEventRecord(e0, st);
      for (int r = 0; r < reps; ++r) (void)launch_dirac(g, prec, a, st);
      (void)hipEventRecord(e1, st);
      if ((rc = hip_check(hipEventSynchronize(e1), "tune timing")) != WD_OK) break;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double us = 1e3 * ms / reps;
      if (getenv("WD_TUNE_VERBOSE"))
        fprintf(stderr, "tune dirac p%d: slices %d tile %d: %.2f us\n", (int)prec, c[0], c[1], us);
      if (us < best_us) { best_us = us; best_s = c[0]; best_t = c[1]; }
    }
  } while (0);
  g->dirac_slices[prec] = (rc == WD_OK) ? best_s : save_s;
  g->dirac_tile[prec] = (rc == WD_OK) ? best_t : save_t;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (in) (void)hipFree(in);
  if (ref) (void)hipFree(ref);
  if (cand) (void)hipFree(cand);
  if (flag) (void)hipFree(flag);
  if (rc != WD_OK) return rc;
  if (cache_path) cache_append(cache_path, key, 256, best_t, best_s, best_us, "slices");
  if (out_slices) *out_slices = best_s;
  if (out_tile) *out_tile = best_t;
  if (out_us) *out_us = best_us;
  return WD_OK;
}

}  // extern "C"

// ------------------------------------------------------------ batched solver
extern "C" wd_status wd_tune_batch(const wd_gauge *const *gs, int n, const void *const *b, void *const *x,
                                   const double *kappa, double tol, const wd_solve_params *p, const char *cache_path,
                                   int force, int *out_tile, int *out_blocks_per_cu, double *out_seconds) {
  if (!gs || !b || !x || !kappa) return set_error(WD_ERR_ARG, "tune_batch: NULL argument");
  if (n < 1 || n > 4096) return set_error(WD_ERR_ARG, "tune_batch: n = %d", n);
  wd_solve_params prm;
  for (int l = 0; l < n; ++l) {
    WD_TRY(solve_args(gs[l], b[l], x[l], kappa[l], tol, p, prm));
    if (gs[l]->device != gs[0]->device) return set_error(WD_ERR_ARG, "tune_batch: handles on different devices");
  }
  if (prm.solver != WD_SOLVER_DEFECT_CG) return set_error(WD_ERR_ARG, "tune_batch: only defect-correction CG");
  // key: arch, inner storage precision and the lattices in order
  std::string key = tune_key(gs[0], prm.inner_prec);
  key = key.substr(0, key.find("/hop/"));
  char part[64];
  snprintf(part, sizeof part, "/batch%d/p%d/", n, (int)prm.inner_prec);
  key += part;
  for (int l = 0; l < n && key.size() < 180; ++l) {
    snprintf(part, sizeof part, "%s%dx%dx%dx%d", l ? "+" : "", gs[l]->dims[0], gs[l]->dims[1], gs[l]->dims[2],
             gs[l]->dims[3]);
    key += part;
  }
  int tile = 256, bpc = 0, nl = 0;
  double us = -1.0;
  if (cache_path && !force && cache_lookup(cache_path, key, tile, bpc, nl, us, "nlat") && nl == n &&
      (tile == 64 || tile == 128 || tile == 256) && bpc >= -1 && bpc <= 64) {
    if (out_tile) *out_tile = tile;
    if (out_blocks_per_cu) *out_blocks_per_cu = bpc;
    if (out_seconds) *out_seconds = us * 1e-6;
    return WD_OK;
  }
  // candidates: tile size x persistent blocks per CU (0: as many as fit; -1: one block per tile);
  // each is run once to warm up and twice timed, and only solves that reach tol count
  std::vector<wd_solve_info> infos((size_t)n);
  double best = 1e30;
  int best_tile = 256, best_bpc = 0;
  for (int t : {256, 128, 64})
    for (int c : {0, 1, 2, 4, 8, -1}) {
      prm.batch_tile = t;
      prm.batch_blocks_per_cu = c;
      double sec = 1e30;
      bool ok = true;
      for (int rep = 0; rep < 3 && ok; ++rep) {
        const wd_status rc = solve_batch(gs, n, b, x, kappa, tol, prm, infos.data());
        if (rc < 0) return rc;
        ok = rc == WD_OK;
        if (rep > 0) sec = std::min(sec, infos[0].seconds);
      }
      if (getenv("WD_TUNE_VERBOSE"))
        fprintf(stderr, "tune %s: tile %d blocks/CU %d: %s %.3f ms\n", key.c_str(), t, c, ok ? "ok" : "not converged",
                sec * 1e3);
      if (ok && sec < best) { best = sec; best_tile = t; best_bpc = c; }
    }
  if (best >= 1e30) return set_error(WD_NOT_CONVERGED, "tune_batch: no candidate reached the tolerance");
  if (cache_path) cache_append(cache_path, key, best_tile, best_bpc, n, best * 1e6, "nlat");
  if (out_tile) *out_tile = best_tile;
  if (out_blocks_per_cu) *out_blocks_per_cu = best_bpc;
  if (out_seconds) *out_seconds = best;
  return WD_OK;
}
