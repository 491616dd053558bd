// Micro-benchmark of a global memory -> LDS block copy: the MI355X analogue
// of the paper's DMA measurements (Sec. 6, Eq. 4), whose model charges a
// transfer a start-up latency, a penalty per misaligned block and the bytes
// over the bandwidth.
//
// One workgroup of 256 threads copies `bytes` bytes that start `offset`
// bytes past a 256-byte boundary into LDS, `reps` times, each time from a
// fresh 1 MiB-spaced source block; 512 MB are written elsewhere first so
// that the sources are not in the Infinity Cache and come from HBM.  Each thread
// moves 16-byte words (dword-aligned loads, so any offset that is a multiple
// of 4 is allowed).  Thread 0 reads the shader clock before and after each
// copy (with barriers), and the per-copy cycles are written out.  A checksum
// of the LDS contents after every copy proves the data arrived.
#include <algorithm>

#include "wd_internal.h"

namespace wd {

namespace {

constexpr int MC_BS = 256;
constexpr size_t MC_STRIDE = 1 << 20;
constexpr int MC_MAX_BYTES = 32768;

struct __attribute__((aligned(4))) word4 {
  uint32_t x, y, z, w;
};

__global__ __launch_bounds__(MC_BS) void k_lds_copy(const char *src, int bytes, int offset, int reps,
                                                   unsigned long long *cycles, uint32_t *sums) {
  extern __shared__ uint4 lds[];
  const int nw = bytes / 16;
  __shared__ uint32_t part[MC_BS / 64];
  for (int r = 0; r < reps; ++r) {
    const word4 *s = (const word4 *)(src + (size_t)r * MC_STRIDE + offset);
    __syncthreads();
    unsigned long long t0 = 0;
    if (threadIdx.x == 0) t0 = clock64();
    __syncthreads();
    for (int i = threadIdx.x; i < nw; i += MC_BS) {
      const word4 v = s[i];
      lds[i] = uint4{v.x, v.y, v.z, v.w};
    }
    __syncthreads();
    if (threadIdx.x == 0) cycles[r] = clock64() - t0;
    // checksum of what LDS holds: sum of all 32-bit words (mod 2^32)
    uint32_t acc = 0;
    for (int i = threadIdx.x; i < nw; i += MC_BS) {
      const uint4 v = lds[i];
      acc += v.x + v.y + v.z + v.w;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t = 0;
      for (int w = 0; w < MC_BS / 64; ++w) t += part[w];
      sums[r] = t;
    }
  }
}

// Streaming probe: R read streams (and W = 0/1 write stream) of 16-byte
// lanes, non-temporal (NT) or cached, one element per thread.
typedef double mv2d __attribute__((ext_vector_type(2)));

template <int R, int W, int NT>
__global__ __launch_bounds__(256) void k_stream(const mv2d *const *in, mv2d *out, long n) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  mv2d s = {0.0, 0.0};
#pragma unroll
  for (int r = 0; r < R; ++r) s += NT ? __builtin_nontemporal_load(in[r] + i) : in[r][i];
  if (W) {
    if (NT) __builtin_nontemporal_store(s, out + i);
    else out[i] = s;
  } else if (s.x == 1234.5678) {
    out[i] = s;  // never true for the zero-filled inputs; keeps the loads live
  }
}

template <int R, int W, int NT>
void launch_stream(const mv2d *const *in, mv2d *out, long n, hipStream_t st) {
  hipLaunchKernelGGL((k_stream<R, W, NT>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
}

// Resident-data probe: a persistent grid reads an n-element buffer `passes`
// times over (16-byte lanes, cached loads, grid-stride, so a block reads the
// same addresses on every pass).  Blocks are dealt round-robin over the XCDs
// and stay on theirs, so from the second pass on the buffer comes from the
// level that holds it: the XCDs' L2 (4 MB each) while an XCD's share fits,
// the 256 MB Infinity Cache while the buffer fits, else HBM.  The compiler
// barrier between passes makes every pass load again.
__global__ __launch_bounds__(256) void k_resident(const mv2d *in, long n, int passes, mv2d *sink) {
  mv2d s = {0.0, 0.0};
  for (int p = 0; p < passes; ++p) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) s += in[i];
    asm volatile("" ::: "memory");
  }
  if (s.x == 1234.5678) sink[0] = s;  // never true for the zero-filled input; keeps the loads live
}

}  // namespace

}  // namespace wd

using namespace wd;

extern "C" wd_status wd_micro_stream(int device, int nread, int write, int nontemporal, size_t bytes, int reps,
                                     double *seconds) {
  if (nread < 1 || nread > 8) return set_error(WD_ERR_ARG, "micro stream: nread = %d (1..8)", nread);
  if (write != 0 && write != 1) return set_error(WD_ERR_ARG, "micro stream: write = %d", write);
  if (bytes < 16 || bytes % 16 || bytes > ((size_t)4 << 30))
    return set_error(WD_ERR_ARG, "micro stream: bytes = %zu (16 B .. 4 GiB, multiple of 16)", bytes);
  if (reps < 1 || reps > 1000) return set_error(WD_ERR_ARG, "micro stream: reps = %d", reps);
  if (!seconds) return set_error(WD_ERR_ARG, "micro stream: NULL output");
  WD_HIP(hipSetDevice(device));
  const long n = (long)(bytes / 16);
  void *buf[9] = {nullptr};
  mv2d **d_in = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  wd_status rc = WD_OK;
  do {
    for (int r = 0; r <= nread; ++r) {
      if ((rc = hip_check(hipMalloc(&buf[r], bytes), "micro alloc")) != WD_OK) break;
      if ((rc = hip_check(hipMemset(buf[r], 0, bytes), "micro fill")) != WD_OK) break;
    }
    if (rc != WD_OK) break;
    if ((rc = hip_check(hipMalloc(&d_in, 8 * sizeof(mv2d *)), "micro alloc")) != WD_OK) break;
    mv2d *h_in[8] = {nullptr};
    for (int r = 0; r < nread; ++r) h_in[r] = (mv2d *)buf[r];
    if ((rc = hip_check(hipMemcpy(d_in, h_in, sizeof h_in, hipMemcpyHostToDevice), "micro upload")) != WD_OK) break;
    mv2d *out = (mv2d *)buf[nread];
    auto run = [&]() {
#define WD_ST(RR)                                                                              \
  if (nread == RR) {                                                                           \
    if (write && nontemporal) launch_stream<RR, 1, 1>(d_in, out, n, 0);                        \
    else if (write) launch_stream<RR, 1, 0>(d_in, out, n, 0);                                  \
    else if (nontemporal) launch_stream<RR, 0, 1>(d_in, out, n, 0);                            \
    else launch_stream<RR, 0, 0>(d_in, out, n, 0);                                             \
  }
      WD_ST(1) WD_ST(2) WD_ST(3) WD_ST(4) WD_ST(5) WD_ST(6) WD_ST(7) WD_ST(8)
#undef WD_ST
    };
    for (int w = 0; w < 3; ++w) run();
    if ((rc = hip_check(hipEventCreate(&e0), "event")) != WD_OK) break;
    if ((rc = hip_check(hipEventCreate(&e1), "event")) != WD_OK) break;
    WD_HIP(hipEventRecord(e0, 0));
    for (int r = 0; r < reps; ++r) run();
    WD_HIP(hipEventRecord(e1, 0));
    if ((rc = hip_check(hipEventSynchronize(e1), "micro timing")) != WD_OK) break;
    float ms = 0.f;
    WD_HIP(hipEventElapsedTime(&ms, e0, e1));
    *seconds = 1e-3 * ms / reps;
    rc = hip_check(hipGetLastError(), "micro launch");
  } while (0);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (void *b : buf)
    if (b) (void)hipFree(b);
  if (d_in) (void)hipFree(d_in);
  return rc;
}

extern "C" wd_status wd_micro_resident(int device, size_t bytes, int passes, int reps, double *seconds) {
  if (bytes < ((size_t)1 << 20) || bytes % ((size_t)1 << 20) || bytes > ((size_t)4 << 30))
    return set_error(WD_ERR_ARG, "micro resident: bytes = %zu (1 MiB .. 4 GiB, whole MiB)", bytes);
  if (passes < 1 || passes > 1000) return set_error(WD_ERR_ARG, "micro resident: passes = %d", passes);
  if (reps < 1 || reps > 100) return set_error(WD_ERR_ARG, "micro resident: reps = %d", reps);
  if (!seconds) return set_error(WD_ERR_ARG, "micro resident: NULL output");
  WD_HIP(hipSetDevice(device));
  int ncu = 0;
  WD_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device));
  const long n = (long)(bytes / 16);
  const unsigned grid = (unsigned)std::max(8, ncu * 8);
  void *buf = nullptr, *sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  wd_status rc = WD_OK;
  do {
    if ((rc = hip_check(hipMalloc(&buf, bytes), "micro alloc")) != WD_OK) break;
    if ((rc = hip_check(hipMalloc(&sink, 256), "micro alloc")) != WD_OK) break;
    if ((rc = hip_check(hipMemset(buf, 0, bytes), "micro fill")) != WD_OK) break;
    // one launch warms the caches
    hipLaunchKernelGGL(k_resident, dim3(grid), dim3(256), 0, 0, (const mv2d *)buf, n, 2, (mv2d *)sink);
    if ((rc = hip_check(hipEventCreate(&e0), "event")) != WD_OK) break;
    if ((rc = hip_check(hipEventCreate(&e1), "event")) != WD_OK) break;
    WD_HIP(hipEventRecord(e0, 0));
    for (int r = 0; r < reps; ++r)
      hipLaunchKernelGGL(k_resident, dim3(grid), dim3(256), 0, 0, (const mv2d *)buf, n, passes, (mv2d *)sink);
    WD_HIP(hipEventRecord(e1, 0));
    if ((rc = hip_check(hipEventSynchronize(e1), "micro timing")) != WD_OK) break;
    float ms = 0.f;
    WD_HIP(hipEventElapsedTime(&ms, e0, e1));
    *seconds = 1e-3 * ms / ((double)reps * passes);
    rc = hip_check(hipGetLastError(), "micro launch");
  } while (0);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (buf) (void)hipFree(buf);
  if (sink) (void)hipFree(sink);
  return rc;
}

extern "C" wd_status wd_micro_lds_copy(int device, int bytes, int offset, int reps, const void *src_host,
                                       unsigned long long *cycles, unsigned *sums) {
  if (bytes < 16 || bytes > MC_MAX_BYTES || bytes % 16)
    return set_error(WD_ERR_ARG, "micro copy: bytes = %d (16..%d, multiple of 16)", bytes, MC_MAX_BYTES);
  if (offset < 0 || offset >= 256 || offset % 4) return set_error(WD_ERR_ARG, "micro copy: offset = %d", offset);
  if (reps < 1 || reps > 1024) return set_error(WD_ERR_ARG, "micro copy: reps = %d (1..1024)", reps);
  if (!cycles || !sums) return set_error(WD_ERR_ARG, "micro copy: NULL output");
  WD_HIP(hipSetDevice(device));
  const size_t total = (size_t)reps * MC_STRIDE;
  char *src = nullptr;
  unsigned long long *d_cyc = nullptr;
  uint32_t *d_sum = nullptr;
  wd_status rc = WD_OK;
  do {
    if ((rc = hip_check(hipMalloc(&src, total), "micro alloc")) != WD_OK) break;
    if ((rc = hip_check(hipMalloc(&d_cyc, reps * sizeof(unsigned long long)), "micro alloc")) != WD_OK) break;
    if ((rc = hip_check(hipMalloc(&d_sum, reps * sizeof(uint32_t)), "micro alloc")) != WD_OK) break;
    // each source block r holds the caller's pattern (MC_STRIDE bytes, or zeros)
    for (int r = 0; r < reps; ++r) {
      if (src_host) {
        if ((rc = hip_check(hipMemcpy(src + (size_t)r * MC_STRIDE, src_host, MC_STRIDE, hipMemcpyHostToDevice),
                            "micro upload")) != WD_OK)
          break;
      } else if ((rc = hip_check(hipMemset(src + (size_t)r * MC_STRIDE, 0, MC_STRIDE), "micro fill")) != WD_OK) {
        break;
      }
    }
    if (rc != WD_OK) break;
    // push the source blocks out of the 256 MB Infinity Cache: write 512 MB elsewhere
    {
      void *flush = nullptr;
      if ((rc = hip_check(hipMalloc(&flush, (size_t)512 << 20), "micro alloc")) != WD_OK) break;
      rc = hip_check(hipMemset(flush, 1, (size_t)512 << 20), "micro flush");
      (void)hipDeviceSynchronize();
      (void)hipFree(flush);
      if (rc != WD_OK) break;
    }
    hipLaunchKernelGGL(k_lds_copy, dim3(1), dim3(MC_BS), (size_t)bytes, 0, (const char *)src, bytes, offset, reps,
                       d_cyc, d_sum);
    if ((rc = hip_check(hipGetLastError(), "micro launch")) != WD_OK) break;
    if ((rc = hip_check(hipMemcpy(cycles, d_cyc, reps * sizeof(unsigned long long), hipMemcpyDeviceToHost),
                        "micro read")) != WD_OK)
      break;
    rc = hip_check(hipMemcpy(sums, d_sum, reps * sizeof(uint32_t), hipMemcpyDeviceToHost), "micro read");
  } while (0);
  if (src) (void)hipFree(src);
  if (d_cyc) (void)hipFree(d_cyc);
  if (d_sum) (void)hipFree(d_sum);
  return rc;
}
