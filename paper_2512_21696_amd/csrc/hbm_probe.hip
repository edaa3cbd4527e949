// Bandwidth yardsticks for the measurement of the step kernels (not part of
// the method): plain copies of a known number of bytes with one 4-byte or one
// 16-byte access per lane, and a read and a write of many equally long arrays
// at the same voxel index (the access pattern of a structure-of-arrays
// population set).  They convert hardware traffic counters into bytes and
// give the practical HBM ceiling the step kernels are compared with.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace {

__global__ __launch_bounds__(256) void k_probe_copy_b32(const float *__restrict__ a,
                                                        float *__restrict__ b, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

__global__ __launch_bounds__(256) void k_probe_copy_b128(const float4 *__restrict__ a,
                                                         float4 *__restrict__ b, size_t n4) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += stride) b[i] = a[i];
}

// Sum of NA arrays of n floats at each index, one thread per index with all
// NA loads in flight (the pattern of a voxel reading its populations); the
// per-index sum is written so the loads cannot be dropped.
template <int NA>
__global__ __launch_bounds__(256) void k_probe_read_arrays(const float *__restrict__ a,
                                                           float *__restrict__ out, uint32_t n) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < NA; ++k) acc += a[(size_t)k * n + i];
  out[i] = acc;
}

template <int NA>
__global__ __launch_bounds__(256) void k_probe_write_arrays(float *__restrict__ b, uint32_t n) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int k = 0; k < NA; ++k) b[(size_t)k * n + i] = (float)(i + k);
}

constexpr int kArrays = 38;  // two components of 19 populations
constexpr unsigned kGrid = 8192;  // 32 blocks of 256 threads per compute unit

}  // namespace

// kind 0: copy bytes/4 floats src -> dst, 4-byte accesses
// kind 1: the same copy with 16-byte accesses (bytes a multiple of 16)
// kind 2: read 38 arrays of bytes/(4*38) floats each from src; dst receives
//         one float per index (bytes/38 bytes)
// kind 3: write 38 arrays of bytes/(4*38) floats each to dst
// narr must be 38 for kinds 2 and 3; per-array length below 2^32.
// Enqueued on the given stream; returns the launch status (hipError_t).
extern "C" int hbm_probe(int kind, const void *src, void *dst, size_t bytes, int narr,
                         void *stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t n = bytes / 4;
  const size_t per = n / kArrays;
  if ((kind == 2 || kind == 3) && (narr != kArrays || per >= 0xffffffffull))
    return (int)hipErrorInvalidValue;
  const unsigned blocks = (unsigned)((per + 255) / 256);
  switch (kind) {
    case 0:
      hipLaunchKernelGGL(k_probe_copy_b32, dim3(kGrid), dim3(256), 0, st,
                         static_cast<const float *>(src), static_cast<float *>(dst), n);
      break;
    case 1:
      hipLaunchKernelGGL(k_probe_copy_b128, dim3(kGrid), dim3(256), 0, st,
                         static_cast<const float4 *>(src), static_cast<float4 *>(dst), n / 4);
      break;
    case 2:
      hipLaunchKernelGGL(k_probe_read_arrays<kArrays>, dim3(blocks), dim3(256), 0, st,
                         static_cast<const float *>(src), static_cast<float *>(dst), (uint32_t)per);
      break;
    case 3:
      hipLaunchKernelGGL(k_probe_write_arrays<kArrays>, dim3(blocks), dim3(256), 0, st,
                         static_cast<float *>(dst), (uint32_t)per);
      break;
    default:
      return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}
