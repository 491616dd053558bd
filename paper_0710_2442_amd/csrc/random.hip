// Gaussian random fields on the device, from a counter-based generator.
//
// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
// as easy as 1, 2, 3", SC 2011): a 4 x 64-bit counter and a 2 x 64-bit key
// go through 10 rounds of
//   (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with the key advanced by the Weyl constants (W0, W1) after every round.
// Every output block depends only on (counter, key), so any site can be
// drawn by any thread in any order and the field is the same for every
// launch shape.  Normal deviates come from the Box-Muller transform.
#include <math.h>

#include "wd_device.h"

namespace wd {

namespace {

constexpr uint64_t PH_M0 = 0xD2E7470EE14C6C93ull, PH_M1 = 0xCA5A826395121157ull;
constexpr uint64_t PH_W0 = 0x9E3779B97F4A7C15ull, PH_W1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64_10(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(PH_M0, c[0]), lo0 = PH_M0 * c[0];
    const uint64_t hi1 = __umul64hi(PH_M1, c[2]), lo1 = PH_M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += PH_W0;
    k1 += PH_W1;
  }
}

// u in (0, 1] from the top 53 bits
__device__ __forceinline__ double unit_open0(uint64_t x) { return (double)((x >> 11) + 1) * 0x1.0p-53; }
// v in [0, 1) from the top 53 bits
__device__ __forceinline__ double unit_closed0(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

// (re, im) = sqrt(-2 ln u) (cos 2 pi v, sin 2 pi v)
__device__ __forceinline__ cplx<double> box_muller(uint64_t a, uint64_t b) {
  const double r = sqrt(-2.0 * log(unit_open0(a)));
  double s, c;
  sincospi(2.0 * unit_closed0(b), &s, &c);
  return {r * c, r * s};
}

struct KRand {
  Geom g;
  char *field;
  size_t half;  // bytes per half field
  int q0;       // parity of the first half in the field
  uint64_t seed, stream;
};

template <int P>
__global__ __launch_bounds__(256) void k_gaussian(KRand k) {
  using T = typename Spinor<P>::real;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int h = blockIdx.y;
  if (i >= k.g.vpad) return;
  char *f = k.field + (size_t)h * k.half;
  cplx<T> s[12];
  if (i < k.g.vh) {
    const uint64_t q = (uint64_t)(k.q0 + h);
    const uint64_t site = q * (uint64_t)k.g.vh + (uint64_t)i;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      uint64_t c[4] = {site * 6 + (uint64_t)j, k.stream, 0, 0};
      philox4x64_10(c, k.seed, 0);
      const cplx<double> a = box_muller(c[0], c[1]), b = box_muller(c[2], c[3]);
      s[2 * j] = {(T)a.re, (T)a.im};
      s[2 * j + 1] = {(T)b.re, (T)b.im};
    }
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) s[c] = {(T)0, (T)0};
  }
  Spinor<P>::store(f, i, s);
}

}  // namespace

wd_status launch_gaussian(const wd_gauge *g, void *field, int parity, wd_prec prec, uint64_t seed, uint64_t stream,
                          hipStream_t st) {
  KRand k{};
  k.g = g->geom;
  k.field = (char *)field;
  k.half = half_bytes(g->geom, prec);
  k.q0 = (parity == WD_FULL) ? 0 : parity;
  k.seed = seed;
  k.stream = stream;
  dim3 grid((unsigned)((g->geom.vpad + 255) / 256), parity == WD_FULL ? 2 : 1);
  switch (prec) {
    case WD_F64: hipLaunchKernelGGL(k_gaussian<WD_F64>, grid, dim3(256), 0, st, k); break;
    case WD_F32: hipLaunchKernelGGL(k_gaussian<WD_F32>, grid, dim3(256), 0, st, k); break;
    default: return set_error(WD_ERR_PREC, "gaussian field: FP64 or FP32 only");
  }
  return hip_check(hipGetLastError(), "gaussian field launch");
}

}  // namespace wd
