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

// One 16 x 16 tile of voxels of one slice per workgroup.  Voxel centres X, Z =
// k + 1/2 - n_out/2; detector index u + nx/2 - 1/2 with u = X cos - Z sin,
// linear interpolation, 0 outside the detector.  For a chunk of angles the
// detector samples the tile can reach are staged in LDS first: over the tile u
// spans 15 (|cos| + |sin|) < 22 pixels, so kFbpSeg samples from one below the
// smallest corner value cover every voxel's pair (zeros stand for samples
// outside the detector).  Every voxel then reads its pair from LDS instead of
// gathering it through the vector-memory path once per angle.
constexpr int kFbpSeg = 32;     // staged samples per angle
constexpr int kFbpChunk = 64;   // angles per staged chunk
constexpr int kFbpThreads = 256;

__global__ void __launch_bounds__(kFbpThreads) fbp_backproject_kernel(const float2* __restrict__ q, int n_proj, int nx,
                                                                      int ny, int n_pad, const float2* __restrict__ cs,
                                                                      int n_out, float scale, float2* __restrict__ vol) {
  __shared__ float2 seg[kFbpChunk * kFbpSeg];
  __shared__ float2 csl[kFbpChunk];
  __shared__ int base[kFbpChunk];
  const int tiles = n_out / 16;
  const int y = blockIdx.x / (tiles * tiles);
  const int tile = blockIdx.x - y * tiles * tiles;
  const int tx = tile % tiles, tz = tile / tiles;
  const float h = 0.5f * (float)n_out;
  const float X = (float)(tx * 16 + (threadIdx.x & 15)) + 0.5f - h;
  const float Z = (float)(tz * 16 + (threadIdx.x >> 4)) + 0.5f - h;
  const float X0 = (float)(tx * 16) + 0.5f - h, Z0 = (float)(tz * 16) + 0.5f - h;
  const float off = 0.5f * (float)nx - 0.5f;
  float2 acc = make_float2(0.f, 0.f);
  for (int j0 = 0; j0 < n_proj; j0 += kFbpChunk) {
    const int na = min(kFbpChunk, n_proj - j0);
    __syncthreads();  // the previous chunk's reads are done
    if ((int)threadIdx.x < na) {
      const float2 c = cs[j0 + threadIdx.x];
      const float ta = X0 * c.x - Z0 * c.y, tb = (X0 + 15.f) * c.x - Z0 * c.y;
      const float tc = X0 * c.x - (Z0 + 15.f) * c.y, td = (X0 + 15.f) * c.x - (Z0 + 15.f) * c.y;
      base[threadIdx.x] = (int)floorf(fminf(fminf(ta, tb), fminf(tc, td)) + off) - 1;
      csl[threadIdx.x] = c;
    }
    __syncthreads();
    // every load of the chunk is issued before the first LDS write
    constexpr int kPer = kFbpChunk * kFbpSeg / kFbpThreads;
    float2 r[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = (int)threadIdx.x + u * kFbpThreads;
      const int a = e / kFbpSeg, i = base[a] + e % kFbpSeg;
      r[u] = (a < na && i >= 0 && i < nx) ? q[((size_t)(j0 + a) * ny + y) * n_pad + i] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) seg[threadIdx.x + u * kFbpThreads] = r[u];
    __syncthreads();
    for (int a = 0; a < na; ++a) {
      const float2 c = csl[a];
      const float t = X * c.x - Z * c.y + off;
      const float f = floorf(t);
      const float w = t - f;
      const int k = min(max((int)f - base[a], 0), kFbpSeg - 2);
      const float2 lo = seg[a * kFbpSeg + k], hi = seg[a * kFbpSeg + k + 1];
      acc.x += lo.x + w * (hi.x - lo.x);
      acc.y += lo.y + w * (hi.y - lo.y);
    }
  }
  const int ix = tx * 16 + (threadIdx.x & 15), iz = tz * 16 + (threadIdx.x >> 4);
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
  hipLaunchKernelGGL(fbp_backproject_kernel, dim3((unsigned)blocks), dim3(kFbpThreads), 0, st, q, n_proj, nx, ny, n_pad,
                     cs, n_out, scale, vol);
  return hipGetLastError();
}

}  // namespace pwf

namespace pwf {

// Fourier shell correlation (Methods, Eq. 16): the chosen part (0 real, 1
// imaginary) of a complex volume, as a complex field for the transforms.
__global__ void fsc_part_kernel(const float2* __restrict__ src, int part, float2* __restrict__ dst, size_t m) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = make_float2(part ? src[i].y : src[i].x, 0.f);
}

// Shell sums of Re(G1* G2), |G1|^2, |G2|^2 over kappa = round(|k|) (signed
// index frequencies of an n^dims grid), kappa <= n/2.  Each workgroup sums its
// grid-stride share into LDS (FP64 atomics: summation order within a
// workgroup is not fixed) and writes one row of partials.
__global__ void __launch_bounds__(256) fsc_shell_kernel(const float2* __restrict__ g1, const float2* __restrict__ g2,
                                                        int n, int dims, double* __restrict__ partial) {
  extern __shared__ double sh[];
  const int nsh = n / 2 + 1;
  for (int i = threadIdx.x; i < 3 * nsh; i += blockDim.x) sh[i] = 0.0;
  __syncthreads();
  const size_t m = dims == 3 ? (size_t)n * n * n : (size_t)n * n;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x) {
    const int kx = (int)(i % n);
    const int ky = (int)((i / n) % n);
    const int kz = dims == 3 ? (int)(i / ((size_t)n * n)) : 0;
    const float fx = (float)(kx < n / 2 ? kx : kx - n);
    const float fy = (float)(ky < n / 2 ? ky : ky - n);
    const float fz = (float)(kz < n / 2 ? kz : kz - n);
    const int s = (int)rintf(sqrtf(fx * fx + fy * fy + fz * fz));
    if (s >= nsh) continue;
    const float2 a = g1[i], b = g2[i];
    atomicAdd(&sh[s], (double)a.x * b.x + (double)a.y * b.y);
    atomicAdd(&sh[nsh + s], (double)a.x * a.x + (double)a.y * a.y);
    atomicAdd(&sh[2 * nsh + s], (double)b.x * b.x + (double)b.y * b.y);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * nsh; i += blockDim.x) partial[(size_t)blockIdx.x * 3 * nsh + i] = sh[i];
}

__global__ void fsc_final_kernel(const double* __restrict__ partial, int blocks, int len, double* __restrict__ out) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < len; j += gridDim.x * blockDim.x) {
    double t = 0.0;
    for (int b = 0; b < blocks; ++b) t += partial[(size_t)b * len + j];
    out[j] = t;
  }
}

int fsc_blocks() { return 1024; }

hipError_t launch_fsc_part(const float2* src, int part, float2* dst, size_t m, hipStream_t st) {
  hipLaunchKernelGGL(fsc_part_kernel, dim3(4096), dim3(256), 0, st, src, part, dst, m);
  return hipGetLastError();
}

hipError_t launch_fsc_shells(const float2* g1, const float2* g2, int n, int dims, double* partial, double* out,
                             hipStream_t st) {
  const int nsh = n / 2 + 1;
  hipLaunchKernelGGL(fsc_shell_kernel, dim3(fsc_blocks()), dim3(256), sizeof(double) * 3 * nsh, st, g1, g2, n, dims,
                     partial);
  hipLaunchKernelGGL(fsc_final_kernel, dim3((3 * nsh + 255) / 256), dim3(256), 0, st, partial, fsc_blocks(),
                     3 * nsh, out);
  return hipGetLastError();
}

}  // namespace pwf
