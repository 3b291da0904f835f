// Element-wise kernels: Sim(3) Exp / Log over arrays of tangents and poses (Sec. III-D), and the
// keyframe packing into the xyzc arena (float32 or bfloat16 with round-to-nearest-even).
#include "common.hpp"
#include "internal.hpp"
#include "sim3.hpp"

namespace ds3 {

__global__ void k_sim3_exp(const double* __restrict__ tau, double* __restrict__ poses, int n) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  sim3_store(sim3_exp(tau + 7 * int64_t(k)), poses + 8 * int64_t(k));
}

__global__ void k_sim3_log(const double* __restrict__ poses, double* __restrict__ tau, int n) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  sim3_log(sim3_load(poses + 8 * int64_t(k)), tau + 7 * int64_t(k));
}

int launch_sim3_exp(const double* tau, double* poses, int n, hipStream_t s) {
  if (n <= 0) return DS3_OK;
  hipLaunchKernelGGL(k_sim3_exp, dim3((n + 63) / 64), dim3(64), 0, s, tau, poses, n);
  return check_hip(hipGetLastError(), "k_sim3_exp");
}

int launch_sim3_log(const double* poses, double* tau, int n, hipStream_t s) {
  if (n <= 0) return DS3_OK;
  hipLaunchKernelGGL(k_sim3_log, dim3((n + 63) / 64), dim3(64), 0, s, poses, tau, n);
  return check_hip(hipGetLastError(), "k_sim3_log");
}

// xyz (3 float per px) + conf -> 16 B float4 or 8 B of four bfloat16 per pixel.
__global__ void k_pack_f32(const float* __restrict__ xyz, const float* __restrict__ conf, int64_t n,
                           float4* __restrict__ out) {
  int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (; k < n; k += stride) out[k] = make_float4(xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2], conf[k]);
}

__global__ void k_pack_bf16(const float* __restrict__ xyz, const float* __restrict__ conf, int64_t n,
                            uint2* __restrict__ out) {
  int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (; k < n; k += stride) {
    uint32_t x = f32_to_bf16(xyz[3 * k]), y = f32_to_bf16(xyz[3 * k + 1]);
    uint32_t z = f32_to_bf16(xyz[3 * k + 2]), c = f32_to_bf16(conf[k]);
    out[k] = make_uint2(x | (y << 16), z | (c << 16));
  }
}

int launch_pack(const float* xyz, const float* conf, int64_t n, ds3_dtype dt, void* out, hipStream_t s) {
  if (n <= 0) return DS3_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (dt == DS3_F32)
    hipLaunchKernelGGL(k_pack_f32, dim3(blocks), dim3(256), 0, s, xyz, conf, n, static_cast<float4*>(out));
  else
    hipLaunchKernelGGL(k_pack_bf16, dim3(blocks), dim3(256), 0, s, xyz, conf, n, static_cast<uint2*>(out));
  return check_hip(hipGetLastError(), "k_pack");
}

}  // namespace ds3
