// Device helpers for the Wilson-Dirac kernels (gfx950, wave64).
//
// Complex arithmetic, the storage formats of spinor fields, the 12-real link
// compression, the spin projectors of Eq. 3 in the chiral basis and the
// fixed-order block reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wd_internal.h"

namespace wd {

// ------------------------------------------------------------------ complex
template <class T>
struct cplx {
  T re, im;
};

template <class T>
__device__ __forceinline__ cplx<T> cmk(T r, T i) { return {r, i}; }
template <class T>
__device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a) { return {-a.re, -a.im}; }
// complex products with the fused multiply-adds written out (the code is
// built without implicit contraction, so every kernel rounds alike)
template <class T>
__device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
template <class T>
__device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
// i * a
template <class T>
__device__ __forceinline__ cplx<T> mul_i(cplx<T> a) { return {-a.im, a.re}; }
template <class T>
__device__ __forceinline__ cplx<T> conj(cplx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <class T>
__device__ __forceinline__ cplx<T> cjmul(cplx<T> a, cplx<T> b) {
  return {fma(a.re, b.re, a.im * b.im), fma(a.re, b.im, -a.im * b.re)};
}
// acc += a * b
template <class T>
__device__ __forceinline__ void cfma(cplx<T> &acc, cplx<T> a, cplx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}

// ------------------------------------------------------- bfloat16 / half
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  // round to nearest, ties to even, on the upper 16 bits of the binary32 word
  uint32_t u = __float_as_uint(f);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ uint16_t f32_to_f16(float f) {
  _Float16 h = (_Float16)f;
  return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_to_f32(uint16_t h) {
  return (float)__builtin_bit_cast(_Float16, h);
}

// ---------------------------------------------------------- memory access
// 16-byte vector types (clang ext vectors, so the nontemporal builtins apply)
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Streaming (read-once / write-once) accesses bypass cache retention so the
// reused neighbour spinors keep the L2.
template <class T>
__device__ __forceinline__ T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }
template <class T>
__device__ __forceinline__ void st_stream(T v, T *p) { __builtin_nontemporal_store(v, p); }
// NT: streaming store (no retention); otherwise an ordinary store, which can
// leave a freshly written field in the caches for the next kernel to read.
template <bool NT, class T>
__device__ __forceinline__ void st_policy(T v, T *p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// -------------------------------------------------------- spinor storage
// Spinor: 12 complex components, c = 3*spin + colour, in 16-byte packets.
// Fields are chunked by 64 sites (one wave): packet k of checkerboard site i
// sits at packet (i / 64) * CHUNK + 64 * k + i % 64, so the packets of a wave
// of sites form one contiguous block and each packet load of a wave is one
// 1 KiB run.  CHUNK = 64 * (packets per site), plus 16 packets of per-site
// scales for FP16.
template <int CHUNK>
__device__ __forceinline__ size_t chunk_base(size_t i) {
  return (i >> 6) * CHUNK + (i & 63);
}

template <int P>
struct Spinor;

template <>
struct Spinor<WD_F64> {
  using real = double;
  static constexpr size_t bytes_per_slot = 192;
  static constexpr int CHUNK = 12 * 64;
  __device__ static void load(const void *base, size_t i, cplx<double> (&s)[12]) {
    const v2d *p = (const v2d *)base + chunk_base<CHUNK>(i);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      v2d v = p[64 * c];
      s[c] = {v.x, v.y};
    }
  }
  // spins 0,1 (LOWER = false) or spins 2,3 (LOWER = true): components 6h .. 6h+5
  template <bool LOWER>
  __device__ static void load_half(const void *base, size_t i, cplx<double> (&s)[6]) {
    const v2d *p = (const v2d *)base + chunk_base<CHUNK>(i) + (LOWER ? 6 * 64 : 0);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      v2d v = p[64 * c];
      s[c] = {v.x, v.y};
    }
  }
  template <bool NT = true>
  __device__ static void store(void *base, size_t i, const cplx<double> (&s)[12]) {
    v2d *p = (v2d *)base + chunk_base<CHUNK>(i);
#pragma unroll
    for (int c = 0; c < 12; ++c) st_policy<NT>(v2d{s[c].re, s[c].im}, p + 64 * c);
  }
};

template <>
struct Spinor<WD_F32> {
  using real = float;
  static constexpr size_t bytes_per_slot = 96;
  static constexpr int CHUNK = 6 * 64;
  __device__ static void load(const void *base, size_t i, cplx<float> (&s)[12]) {
    const v4f *p = (const v4f *)base + chunk_base<CHUNK>(i);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      v4f v = p[64 * k];
      s[2 * k] = {v.x, v.y};
      s[2 * k + 1] = {v.z, v.w};
    }
  }
  template <bool LOWER>
  __device__ static void load_half(const void *base, size_t i, cplx<float> (&s)[6]) {
    const v4f *p = (const v4f *)base + chunk_base<CHUNK>(i) + (LOWER ? 3 * 64 : 0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      v4f v = p[64 * k];
      s[2 * k] = {v.x, v.y};
      s[2 * k + 1] = {v.z, v.w};
    }
  }
  template <bool NT = true>
  __device__ static void store(void *base, size_t i, const cplx<float> (&s)[12]) {
    v4f *p = (v4f *)base + chunk_base<CHUNK>(i);
#pragma unroll
    for (int k = 0; k < 6; ++k)
      st_policy<NT>(v4f{s[2 * k].re, s[2 * k].im, s[2 * k + 1].re, s[2 * k + 1].im}, p + 64 * k);
  }
};

// 16-byte packet of eight 16-bit reals
struct alignas(16) pk8 {
  uint32_t w[4];
};

// FP16: 3 packets of halves per site, then (per chunk) the 64 sites' scales.
template <>
struct Spinor<WD_F16> {
  using real = float;
  static constexpr size_t bytes_per_slot = 52;
  static constexpr int CHUNK = 3 * 64 + 16;
  __device__ static float scale(const void *base, size_t i) {
    return ((const float *)((const v4u *)base + (i >> 6) * CHUNK + 3 * 64))[i & 63];
  }
  __device__ static void load(const void *base, size_t i, cplx<float> (&s)[12]) {
    const v4u *p = (const v4u *)base + chunk_base<CHUNK>(i);
    const float nrm = scale(base, i);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      v4u v = p[64 * k];
      uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        s[4 * k + j] = {nrm * f16_to_f32((uint16_t)(w[j] & 0xffffu)),
                        nrm * f16_to_f32((uint16_t)(w[j] >> 16))};
      }
    }
  }
  // components 6h .. 6h+5 live in packets (0, 1) or (1, 2)
  template <bool LOWER>
  __device__ static void load_half(const void *base, size_t i, cplx<float> (&s)[6]) {
    const v4u *p = (const v4u *)base + chunk_base<CHUNK>(i);
    const float nrm = scale(base, i);
    const v4u a = p[(LOWER ? 1 : 0) * 64], b = p[(LOWER ? 2 : 1) * 64];
    const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    const int o = LOWER ? 2 : 0;
#pragma unroll
    for (int j = 0; j < 6; ++j)
      s[j] = {nrm * f16_to_f32((uint16_t)(w[o + j] & 0xffffu)), nrm * f16_to_f32((uint16_t)(w[o + j] >> 16))};
  }
  template <bool NT = true>
  __device__ static void store(void *base, size_t i, const cplx<float> (&s)[12]) {
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(s[c].re), fabsf(s[c].im)));
    const float inv = m > 0.f ? 1.0f / m : 0.f;
    v4u *p = (v4u *)base + chunk_base<CHUNK>(i);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint32_t w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const cplx<float> z = s[4 * k + j];
        w[j] = (uint32_t)f32_to_f16(z.re * inv) | ((uint32_t)f32_to_f16(z.im * inv) << 16);
      }
      st_policy<NT>(v4u{w[0], w[1], w[2], w[3]}, p + 64 * k);
    }
    st_policy<NT>(m, (float *)((v4u *)base + (i >> 6) * CHUNK + 3 * 64) + (i & 63));
  }
};

template <>
struct Spinor<WD_BF16> {
  using real = float;
  static constexpr size_t bytes_per_slot = 48;
  static constexpr int CHUNK = 3 * 64;
  __device__ static void load(const void *base, size_t i, cplx<float> (&s)[12]) {
    const v4u *p = (const v4u *)base + chunk_base<CHUNK>(i);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      v4u v = p[64 * k];
      uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 4; ++j)
        s[4 * k + j] = {bf16_to_f32((uint16_t)(w[j] & 0xffffu)), bf16_to_f32((uint16_t)(w[j] >> 16))};
    }
  }
  template <bool LOWER>
  __device__ static void load_half(const void *base, size_t i, cplx<float> (&s)[6]) {
    const v4u *p = (const v4u *)base + chunk_base<CHUNK>(i);
    const v4u a = p[(LOWER ? 1 : 0) * 64], b = p[(LOWER ? 2 : 1) * 64];
    const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    const int o = LOWER ? 2 : 0;
#pragma unroll
    for (int j = 0; j < 6; ++j)
      s[j] = {bf16_to_f32((uint16_t)(w[o + j] & 0xffffu)), bf16_to_f32((uint16_t)(w[o + j] >> 16))};
  }
  template <bool NT = true>
  __device__ static void store(void *base, size_t i, const cplx<float> (&s)[12]) {
    v4u *p = (v4u *)base + chunk_base<CHUNK>(i);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint32_t w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const cplx<float> z = s[4 * k + j];
        w[j] = (uint32_t)f32_to_bf16(z.re) | ((uint32_t)f32_to_bf16(z.im) << 16);
      }
      st_policy<NT>(v4u{w[0], w[1], w[2], w[3]}, p + 64 * k);
    }
  }
};

// ------------------------------------------------------ compressed links
// A hop link is stored as its rows 0 and 1 (6 complex = 12 reals); row 2 is
// conj(row0 x row1).  double: 6 packets of v2d; float: 3 packets of v4f.
//
// Layout of one output parity's hop links (chunks of 64 sites = one wave):
//   packet (hop d, k, site i) at ((i / 64) * 8 + d) * NP * 64 + k * 64 + i % 64
// so a wave's 8 x NP link loads read one contiguous block of 8*NP KiB.
template <int NP>
__device__ __forceinline__ size_t link_packet(int d, int k, size_t i) {
  return (((i >> 6) * 8 + (size_t)d) * NP + (size_t)k) * 64 + (i & 63);
}

template <class R>
struct Link;

// NT = true (default): streaming loads, for links read once per launch;
// NT = false: ordinary loads, for links another site of the launch re-reads.
template <>
struct Link<double> {
  static constexpr int NP = 6;
  template <bool NT = true>
  __device__ static void load(const void *base, int d, size_t i, cplx<double> (&u)[6]) {
    const v2d *p = (const v2d *)base;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const v2d *a = p + link_packet<6>(d, k, i);
      v2d v = NT ? ld_stream(a) : *a;
      u[k] = {v.x, v.y};
    }
  }
};
template <>
struct Link<float> {
  static constexpr int NP = 3;
  template <bool NT = true>
  __device__ static void load(const void *base, int d, size_t i, cplx<float> (&u)[6]) {
    const v4f *p = (const v4f *)base;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const v4f *a = p + link_packet<3>(d, k, i);
      v4f v = NT ? ld_stream(a) : *a;
      u[2 * k] = {v.x, v.y};
      u[2 * k + 1] = {v.z, v.w};
    }
  }
};

// Full 3x3 from the two stored rows a = u[0..2], b = u[3..5].
template <class T>
__device__ __forceinline__ void rebuild_row2(const cplx<T> (&u)[6], cplx<T> (&c)[3]) {
  const cplx<T> a0 = u[0], a1 = u[1], a2 = u[2], b0 = u[3], b1 = u[4], b2 = u[5];
  // conj(x y - z w), as y x - (z w) with the second product accumulated by fma
  auto det2 = [](cplx<T> x, cplx<T> y, cplx<T> z, cplx<T> w) {
    cplx<T> t = z * w;
    t = {-t.re, -t.im};
    cfma(t, x, y);
    return conj(t);
  };
  c[0] = det2(a1, b2, a2, b1);
  c[1] = det2(a2, b0, a0, b2);
  c[2] = det2(a0, b1, a1, b0);
}

// y = M v for the 3x3 matrix with rows (u[0..2], u[3..5], r2[0..2])
template <class T>
__device__ __forceinline__ void su3_mul(const cplx<T> (&u)[6], const cplx<T> (&r2)[3],
                                        const cplx<T> (&v)[3], cplx<T> (&y)[3]) {
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    cplx<T> acc = u[3 * a] * v[0];
    cfma(acc, u[3 * a + 1], v[1]);
    cfma(acc, u[3 * a + 2], v[2]);
    y[a] = acc;
  }
  cplx<T> acc = r2[0] * v[0];
  cfma(acc, r2[1], v[1]);
  cfma(acc, r2[2], v[2]);
  y[2] = acc;
}

// y = M^dag v for the same M (columns of M conjugated)
template <class T>
__device__ __forceinline__ void su3_mul_dag(const cplx<T> (&u)[6], const cplx<T> (&r2)[3],
                                            const cplx<T> (&v)[3], cplx<T> (&y)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx<T> acc = cjmul(u[a], v[0]);
    cfma(acc, conj(u[3 + a]), v[1]);
    cfma(acc, conj(r2[a]), v[2]);
    y[a] = acc;
  }
}

// --------------------------------------------------------- spin projection
// Fields are stored in the spin basis where gamma_4 is diagonal: psi' = S psi
// with S = (1/sqrt 2) [[1, 1], [1, -1]] (2x2 spin blocks; real, orthogonal,
// S = S^-1) applied to the chiral-basis spinor.  There gamma_4' =
// diag(1, 1, -1, -1) and gamma_k' = [[0, -A_k], [A_k, 0]] with A_k the
// upper-right block of the chiral gamma_k (A_1 = i s_x, A_2 = -i s_y,
// A_3 = i s_z).  For the projector (1 + S gamma_MU), S = +-1:
//   MU=0: h = (p0 - S i p3, p1 - S i p2);  lower rows = S i (g1, g0)
//   MU=1: h = (p0 + S p3,   p1 - S p2);    lower rows = S (-g1, g0)
//   MU=2: h = (p0 - S i p2, p1 + S i p3);  lower rows = S (i g0, -i g1)
//   MU=3: S = +1: h = 2 (p0, p1), upper rows only;
//         S = -1: h = 2 (p2, p3), lower rows only
// where g = U h is the transported half spinor.  A time hop therefore reads
// only half of the neighbour spinor.
template <int MU, int S, class T>
__device__ __forceinline__ void project(const cplx<T> (&p)[12], cplx<T> (&h)[6]) {
  static_assert(MU < 3, "time hops use the half-spinor path");
  const T s = (T)S;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cplx<T> p0 = p[a], p1 = p[3 + a], p2 = p[6 + a], p3 = p[9 + a];
    if constexpr (MU == 0) {
      h[a] = p0 - s * mul_i(p3);
      h[3 + a] = p1 - s * mul_i(p2);
    } else if constexpr (MU == 1) {
      h[a] = p0 + s * p3;
      h[3 + a] = p1 - s * p2;
    } else {
      h[a] = p0 - s * mul_i(p2);
      h[3 + a] = p1 + s * mul_i(p3);
    }
  }
}

// acc += full spinor rebuilt from the transported half spinor (g0, g1)
template <int MU, int S, class T>
__device__ __forceinline__ void reconstruct_add(cplx<T> (&acc)[12], const cplx<T> (&g)[6]) {
  const T s = (T)S;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cplx<T> g0 = g[a], g1 = g[3 + a];
    if constexpr (MU == 3) {
      if constexpr (S > 0) {
        acc[a] = acc[a] + g0;
        acc[3 + a] = acc[3 + a] + g1;
      } else {
        acc[6 + a] = acc[6 + a] + g0;
        acc[9 + a] = acc[9 + a] + g1;
      }
    } else {
      acc[a] = acc[a] + g0;
      acc[3 + a] = acc[3 + a] + g1;
      if constexpr (MU == 0) {
        acc[6 + a] = acc[6 + a] + s * mul_i(g1);
        acc[9 + a] = acc[9 + a] + s * mul_i(g0);
      } else if constexpr (MU == 1) {
        acc[6 + a] = acc[6 + a] - s * g1;
        acc[9 + a] = acc[9 + a] + s * g0;
      } else {
        acc[6 + a] = acc[6 + a] + s * mul_i(g0);
        acc[9 + a] = acc[9 + a] - s * mul_i(g1);
      }
    }
  }
}

// ------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sums over the block (blockDim.x a multiple of 64, at most 1024), valid in
// thread 0.  Fixed order: wave sums, then waves in index order.
template <int N>
__device__ __forceinline__ void block_sum_n(double (&v)[N]) {
  __shared__ double red[N][16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double s = wave_sum(v[j]);
    if (lane == 0) red[j][w] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double t = 0.0;
      for (int k = 0; k < nw; ++k) t += red[j][k];
      v[j] = t;
    }
  }
  __syncthreads();
}

// Block sums of v (fixed order) stored as this block's partials,
// partials[j * nblocks + bid]; a finishing kernel (launch_finish_sums) adds
// them up after the launch.  No atomics and no fences: the kernel boundary
// makes the stores visible.
template <int N>
__device__ __forceinline__ void block_sum_store(double (&v)[N], double *partials, unsigned nblocks, unsigned bid) {
  block_sum_n<N>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < N; ++j) partials[(size_t)j * nblocks + bid] = v[j];
  }
}

}  // namespace wd
