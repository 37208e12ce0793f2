// Filtered back-projection (Methods, "Reconstruction procedure"): ramp
// filtering of every detector row of every projection, then back-projection
// of each slice over the angles in [0, pi).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pwf_device.h"
#include "pwf_kernels.h"

namespace pwf {

// Rows of the projections, zero-padded: dst[(j ny + y) n_pad + i] = psi_j[y][i]
// for i < nx, 0 up to n_pad.
__global__ void fbp_pad_kernel(const float2* const* __restrict__ psi, int nx, int ny, int n_pad,
                               float2* __restrict__ dst, size_t total) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const size_t row = i / n_pad;
    const int col = (int)(i - row * n_pad);
    const int j = (int)(row / ny), y = (int)(row - (size_t)j * ny);
    dst[i] = col < nx ? psi[j][(size_t)y * nx + col] : make_float2(0.f, 0.f);
  }
}

// Multiply every padded row spectrum by the real ramp response (already
// divided by n_pad, the normalisation of the inverse transform).
__global__ void fbp_ramp_kernel(float2* __restrict__ a, const float* __restrict__ h, int n_pad, size_t total) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const float w = h[i % n_pad];
    a[i] = make_float2(a[i].x * w, a[i].y * w);
  }
}

// One 16 x 16 tile of voxels of one slice per workgroup; each thread sums the
// linearly interpolated filtered rows over all angles.  Voxel centres X, Z =
// k + 1/2 - n_out/2; detector index u + nx/2 - 1/2 with u = X cos - Z sin.
__global__ void __launch_bounds__(256) fbp_backproject_kernel(const float2* __restrict__ q, int n_proj, int nx,
                                                              int ny, int n_pad, const float2* __restrict__ cs,
                                                              int n_out, float scale, float2* __restrict__ vol) {
  extern __shared__ float2 cs_lds[];
  for (int j = threadIdx.x; j < n_proj; j += blockDim.x) cs_lds[j] = cs[j];
  __syncthreads();
  const int tiles = n_out / 16;
  const int y = blockIdx.x / (tiles * tiles);
  const int tile = blockIdx.x - y * tiles * tiles;
  const int ix = (tile % tiles) * 16 + (threadIdx.x & 15);
  const int iz = (tile / tiles) * 16 + (threadIdx.x >> 4);
  const float X = (float)ix + 0.5f - 0.5f * (float)n_out;
  const float Z = (float)iz + 0.5f - 0.5f * (float)n_out;
  const float off = 0.5f * (float)nx - 0.5f;
  float2 acc = make_float2(0.f, 0.f);
  const float2* row = q + (size_t)y * n_pad;
  const size_t proj_stride = (size_t)ny * n_pad;
  for (int j = 0; j < n_proj; ++j, row += proj_stride) {
    const float2 c = cs_lds[j];
    const float t = X * c.x - Z * c.y + off;
    const float f = floorf(t);
    const int i0 = (int)f;
    const float w = t - f;
    if (i0 >= -1 && i0 < nx) {
      const float2 lo = i0 >= 0 ? row[i0] : make_float2(0.f, 0.f);
      const float2 hi = i0 + 1 < nx ? row[i0 + 1] : make_float2(0.f, 0.f);
      acc.x += lo.x + w * (hi.x - lo.x);
      acc.y += lo.y + w * (hi.y - lo.y);
    }
  }
  vol[((size_t)y * n_out + iz) * n_out + ix] = make_float2(acc.x * scale, acc.y * scale);
}

hipError_t launch_fbp_pad(const float2* const* psi, int n_proj, int nx, int ny, int n_pad, float2* dst,
                          hipStream_t st) {
  const size_t total = (size_t)n_proj * ny * n_pad;
  hipLaunchKernelGGL(fbp_pad_kernel, dim3(4096), dim3(256), 0, st, psi, nx, ny, n_pad, dst, total);
  return hipGetLastError();
}

hipError_t launch_fbp_ramp(float2* a, const float* h, int n_pad, size_t rows, hipStream_t st) {
  hipLaunchKernelGGL(fbp_ramp_kernel, dim3(4096), dim3(256), 0, st, a, h, n_pad, rows * n_pad);
  return hipGetLastError();
}

hipError_t launch_fbp_backproject(const float2* q, int n_proj, int nx, int ny, int n_pad, const float2* cs, int n_out,
                                  float scale, float2* vol, hipStream_t st) {
  const int tiles = n_out / 16;
  const size_t blocks = (size_t)ny * tiles * tiles;
  hipLaunchKernelGGL(fbp_backproject_kernel, dim3((unsigned)blocks), dim3(256), sizeof(float2) * n_proj, st, q,
                     n_proj, nx, ny, n_pad, cs, n_out, scale, vol);
  return hipGetLastError();
}

}  // namespace pwf
