// Bare streaming read: the measured read ceiling of the device memory that the streaming kernels are
// compared with (lsq_read_bandwidth).  Every workgroup sums the 16-byte vectors of a contiguous slice of
// the buffer with the same non-temporal vector loads as the fused pass, two loads in flight per lane,
// and writes its sum, so that no load is dropped.  Only whole 16-byte vectors are read.
#include "internal.h"

namespace lsq {

typedef float probe_f4 __attribute__((ext_vector_type(4)));
constexpr int READ_NT = 256;

__global__ __launch_bounds__(READ_NT) void k_stream_read(const probe_f4* __restrict__ buf, int64_t nvec,
                                                         float* __restrict__ out) {
  const int64_t per = (nvec + gridDim.x - 1) / gridDim.x;
  const int64_t v0 = (int64_t)blockIdx.x * per, v1 = min(nvec, v0 + per);
  probe_f4 acc0 = (probe_f4){0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
  int64_t i = v0 + threadIdx.x;
  for (; i + READ_NT < v1; i += 2 * READ_NT) {
    acc0 += __builtin_nontemporal_load(buf + i);
    acc1 += __builtin_nontemporal_load(buf + i + READ_NT);
  }
  if (i < v1) acc0 += __builtin_nontemporal_load(buf + i);
  const probe_f4 a = acc0 + acc1;
  float sum = ((a[0] + a[1]) + a[2]) + a[3];
  for (int off = 32; off >= 1; off >>= 1) sum += __shfl_xor(sum, off, 64);
  __shared__ float sh[READ_NT / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// Bare streaming copy: the measured ceiling of a kernel that reads one buffer and writes another of the
// same size (the SRHT's first pass reads A and writes its intermediate).  Each workgroup copies the
// 16-byte vectors of a contiguous slice with non-temporal loads and stores, two vectors in flight per lane.
__global__ __launch_bounds__(READ_NT) void k_stream_copy(const probe_f4* __restrict__ src, probe_f4* __restrict__ dst,
                                                         int64_t nvec) {
  const int64_t per = (nvec + gridDim.x - 1) / gridDim.x;
  const int64_t v0 = (int64_t)blockIdx.x * per, v1 = min(nvec, v0 + per);
  int64_t i = v0 + threadIdx.x;
  for (; i + READ_NT < v1; i += 2 * READ_NT) {
    const probe_f4 a = __builtin_nontemporal_load(src + i);
    const probe_f4 b = __builtin_nontemporal_load(src + i + READ_NT);
    __builtin_nontemporal_store(a, dst + i);
    __builtin_nontemporal_store(b, dst + i + READ_NT);
  }
  if (i < v1) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

void stream_copy(hipStream_t st, const void* src, void* dst, int64_t bytes, int groups) {
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)groups), dim3(READ_NT), 0, st, (const probe_f4*)src,
                     (probe_f4*)dst, bytes / 16);
}

void stream_read(hipStream_t st, const void* buf, int64_t bytes, int groups, float* out) {
  hipLaunchKernelGGL(k_stream_read, dim3((unsigned)groups), dim3(READ_NT), 0, st, (const probe_f4*)buf, bytes / 16,
                     out);
}

}  // namespace lsq
