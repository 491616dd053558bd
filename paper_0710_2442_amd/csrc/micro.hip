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

}  // namespace

}  // namespace wd

using namespace wd;

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
