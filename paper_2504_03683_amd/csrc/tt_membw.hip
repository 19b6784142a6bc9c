// tt_membw.hip -- streaming-read bandwidth of the device, measured by a plain
// read kernel: the ceiling the tally pipeline's HBM fraction is compared with,
// next to the published peak.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "thapi_tally.h"

namespace {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) v4u gv4;

// Every lane reads 16-byte words in a grid-stride loop, four loads in flight
// per lane, and folds them into one word per workgroup (so the loads cannot
// be dropped).  `n` is the number of 16-byte words (a multiple of 4 x grid).
__global__ __launch_bounds__(256) void k_read(const uint4 *__restrict__ src, uint64_t n, uint32_t *__restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  gv4 *p = (gv4 *)src;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const v4u a = __builtin_nontemporal_load(p + i), b = __builtin_nontemporal_load(p + i + stride),
              c = __builtin_nontemporal_load(p + i + 2 * stride), d = __builtin_nontemporal_load(p + i + 3 * stride);
    const v4u x = a ^ b ^ c ^ d;
    acc ^= x.x ^ x.y ^ x.z ^ x.w;
  }
  for (; i < n; i += stride) {
    const v4u a = __builtin_nontemporal_load(p + i);
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  __shared__ uint32_t s;
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  atomicXor(&s, acc);
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void k_fill(uint4 *dst, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = make_uint4((uint32_t)i, (uint32_t)(i >> 32), 0x9E3779B9u, 1u);
}

}  // namespace

extern "C" int thapi_tally_read_bandwidth(int32_t device, uint64_t bytes, uint32_t reps, double *gbs) {
  if (!gbs || bytes < (1u << 20) || reps == 0) return THAPI_E_INVAL;
  if (hipSetDevice(device) != hipSuccess) return THAPI_E_DEVICE;
  int n_cu = 256;
  hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
  const uint32_t grid = (uint32_t)n_cu * 16, block = 256;
  const uint64_t quantum = 16ull * 4 * grid * block;
  const uint64_t n = bytes / quantum * quantum / 16;
  if (!n) return THAPI_E_INVAL;
  uint4 *buf = nullptr;
  uint32_t *out = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = THAPI_OK;
  float best = -1;
  if (hipMalloc(&buf, n * 16) != hipSuccess || hipMalloc(&out, 4ull * grid) != hipSuccess) {
    hipGetLastError();
    rc = THAPI_E_NOMEM;
    goto done;
  }
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    rc = THAPI_E_DEVICE;
    goto done;
  }
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(block), 0, st, buf, n);
  for (uint32_t r = 0; r <= reps; r++) {   // the first pass warms up
    hipEventRecord(e0, st);
    hipLaunchKernelGGL(k_read, dim3(grid), dim3(block), 0, st, buf, n, out);
    hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) { rc = THAPI_E_DEVICE; goto done; }
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    if (r && (best < 0 || ms < best)) best = ms;
  }
  if (hipGetLastError() != hipSuccess || best <= 0) { rc = THAPI_E_DEVICE; goto done; }
  *gbs = (double)n * 16 / (best * 1e-3) / 1e9;
done:
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (st) hipStreamDestroy(st);
  if (buf) hipFree(buf);
  if (out) hipFree(out);
  return rc;
}
