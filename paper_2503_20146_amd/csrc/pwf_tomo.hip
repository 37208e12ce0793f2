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

// One 16 (x) by 32 (z) tile of voxels of one slice per workgroup, two voxels
// per lane (rows z and z + 16).  Voxel centres X, Z = k + 1/2 - n_out/2;
// detector index u + nx/2 - 1/2 with u = X cos - Z sin, linear interpolation,
// 0 outside the detector.  For a chunk of angles the detector samples the tile
// can reach are staged in LDS first: over the tile u spans 15 |cos| + 31 |sin|
// < 35 pixels, so kFbpSeg samples from one below the smallest corner value
// cover every voxel's pair (zeros stand for samples outside the detector).
// Each staged entry holds a sample and the step to the next one, so that a
// voxel's interpolation is one LDS read and two FMAs per part, instead of a
// gather through the vector-memory path once per angle; the lane's second
// voxel shares the per-angle reads and sits 16 sin below the first.
constexpr int kFbpSeg = 40;     // staged samples per angle
constexpr int kFbpChunk = 32;   // angles per staged chunk
constexpr int kFbpThreads = 256;
constexpr int kFbpTileZ = 32;

__global__ void __launch_bounds__(kFbpThreads) fbp_backproject_kernel(const float2* __restrict__ q, int n_proj, int nx,
                                                                      int ny, int n_pad, const float2* __restrict__ cs,
                                                                      int n_out, float scale, float2* __restrict__ vol) {
  __shared__ float4 seg[kFbpChunk * kFbpSeg];  // sample k, then sample k + 1 minus sample k
  __shared__ float2 csl[kFbpChunk];  // cos, sin
  __shared__ float t0l[kFbpChunk];   // detector index of the tile's first voxel minus base
  __shared__ int base[kFbpChunk];
  const int tiles_x = n_out / 16, tiles_z = (n_out + kFbpTileZ - 1) / kFbpTileZ;
  const int y = blockIdx.x / (tiles_x * tiles_z);
  const int tile = blockIdx.x - y * tiles_x * tiles_z;
  const int tx = tile % tiles_x, tz = tile / tiles_x;
  const float h = 0.5f * (float)n_out;
  const float dx = (float)(threadIdx.x & 15), dz = (float)(threadIdx.x >> 4);  // first voxel within the tile
  const float X0 = (float)(tx * 16) + 0.5f - h, Z0 = (float)(tz * kFbpTileZ) + 0.5f - h;
  const float off = 0.5f * (float)nx - 0.5f;
  float2 acc0 = make_float2(0.f, 0.f), acc1 = make_float2(0.f, 0.f);
  for (int j0 = 0; j0 < n_proj; j0 += kFbpChunk) {
    const int na = min(kFbpChunk, n_proj - j0);
    __syncthreads();  // the previous chunk's reads are done
    if ((int)threadIdx.x < na) {
      const float2 c = cs[j0 + threadIdx.x];
      const float xe = X0 + 15.f, ze = Z0 + (float)(kFbpTileZ - 1);
      const float ta = X0 * c.x - Z0 * c.y, tb = xe * c.x - Z0 * c.y;
      const float tc = X0 * c.x - ze * c.y, td = xe * c.x - ze * c.y;
      const int b0 = (int)floorf(fminf(fminf(ta, tb), fminf(tc, td)) + off) - 1;
      base[threadIdx.x] = b0;
      // u + nx/2 - 1/2 - base = (ta + off - base) + dx cos - dz sin: small numbers,
      // so the index and the weight keep more bits than from u itself
      csl[threadIdx.x] = c;
      t0l[threadIdx.x] = (ta + off) - (float)b0;
    }
    __syncthreads();
    // every load of the chunk is issued before the first LDS write
    constexpr int kPer = (kFbpChunk * kFbpSeg + kFbpThreads - 1) / kFbpThreads;
    float2 r0[kPer], r1[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = (int)threadIdx.x + u * kFbpThreads;
      const int a = e / kFbpSeg, i = base[a < kFbpChunk ? a : 0] + e % kFbpSeg;
      const float2* row = q + ((size_t)(j0 + a) * ny + y) * n_pad;
      const bool ok = e < kFbpChunk * kFbpSeg && a < na;
      r0[u] = (ok && i >= 0 && i < nx) ? row[i] : make_float2(0.f, 0.f);
      r1[u] = (ok && i + 1 >= 0 && i + 1 < nx) ? row[i + 1] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = (int)threadIdx.x + u * kFbpThreads;
      if (e < kFbpChunk * kFbpSeg)
        seg[e] = make_float4(r0[u].x, r0[u].y, r1[u].x - r0[u].x, r1[u].y - r0[u].y);
    }
    __syncthreads();
    for (int a = 0; a < na; ++a) {
      const float2 c = csl[a];
      const float t = fmaf(dx, c.x, fmaf(-dz, c.y, t0l[a]));
      const float t2 = fmaf(-16.f, c.y, t);
      // t, t2 >= 1 by the choice of base (up to rounding), so truncation is the floor
      const float w = __builtin_amdgcn_fractf(t), w2 = __builtin_amdgcn_fractf(t2);
      const int k = min(max((int)t, 0), kFbpSeg - 1), k2 = min(max((int)t2, 0), kFbpSeg - 1);
      const float4 p = seg[a * kFbpSeg + k], p2 = seg[a * kFbpSeg + k2];
      acc0.x = fmaf(w, p.z, acc0.x + p.x);
      acc0.y = fmaf(w, p.w, acc0.y + p.y);
      acc1.x = fmaf(w2, p2.z, acc1.x + p2.x);
      acc1.y = fmaf(w2, p2.w, acc1.y + p2.y);
    }
  }
  const int ix = tx * 16 + (threadIdx.x & 15), iz = tz * kFbpTileZ + (threadIdx.x >> 4);
  if (iz < n_out) vol[((size_t)y * n_out + iz) * n_out + ix] = make_float2(acc0.x * scale, acc0.y * scale);
  if (iz + 16 < n_out)
    vol[((size_t)y * n_out + iz + 16) * n_out + ix] = make_float2(acc1.x * scale, acc1.y * scale);
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
  const size_t blocks = (size_t)ny * (n_out / 16) * ((n_out + kFbpTileZ - 1) / kFbpTileZ);
  hipLaunchKernelGGL(fbp_backproject_kernel, dim3((unsigned)blocks), dim3(kFbpThreads), 0, st, q, n_proj, nx, ny, n_pad,
                     cs, n_out, scale, vol);
  return hipGetLastError();
}

}  // namespace pwf

namespace pwf {

// Fourier shell correlation (Methods, Eq. 16) of the chosen parts (0 real,
// 1 imaginary) of two complex volumes.  Both real fields go into one complex
// field c = a + i b, whose single DFT C holds both spectra:
//   A(k) = (C(k) + conj C(-k)) / 2,   B(k) = (C(k) - conj C(-k)) / (2 i),
// one transform instead of two.  The rounding of each spectrum is then
// relative to the larger of the two at that frequency, so a and b are first
// scaled to unit RMS: the correlation does not change under positive scaling
// of either input, and inputs of any relative size keep FP32 accuracy.
constexpr int kFscThreads = 256;

// FP64 sums of a^2 and b^2 per workgroup, in a fixed order.
__global__ void __launch_bounds__(kFscThreads) fsc_norm_kernel(const float2* __restrict__ g1,
                                                               const float2* __restrict__ g2, int part, size_t m,
                                                               double* __restrict__ partial) {
  double sa = 0.0, sb = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x) {
    const float2 u = g1[i], v = g2[i];
    const double a = part ? u.y : u.x, b = part ? v.y : v.x;
    sa = fma(a, a, sa);
    sb = fma(b, b, sb);
  }
  __shared__ double red[kFscThreads / 64][2];
  for (int off = 32; off > 0; off >>= 1) {
    sa += __shfl_xor(sa, off, 64);
    sb += __shfl_xor(sb, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = sa;
    red[threadIdx.x >> 6][1] = sb;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int w = 0; w < kFscThreads / 64; ++w) t += red[w][threadIdx.x];
    partial[2 * (size_t)blockIdx.x + threadIdx.x] = t;
  }
}

// scale[p] = 1 / RMS of field p (1 for a field of zeros), the partials summed in order
__global__ void fsc_scale_kernel(const double* __restrict__ partial, int blocks, size_t m, float* __restrict__ scale) {
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int b = 0; b < blocks; ++b) t += partial[2 * (size_t)b + threadIdx.x];
    scale[threadIdx.x] = t > 0.0 ? (float)(1.0 / sqrt(t / (double)m)) : 1.f;
  }
}

__global__ void fsc_pack_kernel(const float2* __restrict__ g1, const float2* __restrict__ g2, int part,
                                const float* __restrict__ scale, float2* __restrict__ dst, size_t m) {
  const float sa = scale[0], sb = scale[1];
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x) {
    const float2 a = g1[i], b = g2[i];
    dst[i] = part ? make_float2(a.y * sa, b.y * sb) : make_float2(a.x * sa, b.x * sb);
  }
}

// Shell sums of Re(G1* G2), |G1|^2, |G2|^2 over kappa = round(|k|) (signed
// index frequencies of an n^dims grid), kappa <= n/2, in a fixed order (the
// result is bit-reproducible).  Every wave owns a private histogram of the
// three sums in LDS and walks its share of the grid in chunks of 64 K
// consecutive elements, K per lane.  A chunk lies in one half of one x row
// (64 K divides n/2), where kappa is monotone in kx, so equal kappa form runs
// of consecutive elements:
//  * each lane sums its own K elements run by run; a run that starts and ends
//    inside the lane is complete and goes to the histogram at once (no other
//    lane holds that kappa);
//  * the lane's first and last runs may continue runs of its neighbours.  A
//    lane whose K elements are one run passes the sum arriving from the left
//    on (when kappa matches) plus its own; any other lane starts afresh with
//    its last run.  That is the map x -> A x + B per lane (A = 1 for a
//    continuing single-run lane, else 0), composed over the wave by an
//    inclusive scan in a fixed butterfly order;
//  * a lane with several runs adds the sum arriving from the left to its first
//    run and writes that; a lane whose last run the next lane does not
//    continue writes its scan value.
// The kappa written by the lanes of one store are distinct, so no two lanes
// of a wave touch one entry at once, and the stores follow program order.
// The workgroup then adds its waves' histograms in wave order and writes one
// row of partials.  Four waves per workgroup up to n = 1024 and two at 2048
// keep the histograms at 49 KB of LDS.

template <int K>
__global__ void __launch_bounds__(kFscThreads) fsc_shell_kernel(const float2* __restrict__ spec, int n, int dims,
                                                                double* __restrict__ partial) {
  extern __shared__ double sh[];
  const int nsh = n / 2 + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  for (int i = threadIdx.x; i < waves * 3 * nsh; i += blockDim.x) sh[i] = 0.0;
  __syncthreads();
  double* h = sh + wave * 3 * nsh;
  const size_t m = dims == 3 ? (size_t)n * n * n : (size_t)n * n;
  const size_t chunks = m / (64 * K);
  const size_t stride = (size_t)gridDim.x * waves;
  const int lg = 31 - __clz(n);  // n is a power of two
  auto put = [&](int k, double x0, double x1, double x2) {
    if (k < nsh) {
      h[k] += x0;
      h[nsh + k] += x1;
      h[2 * nsh + k] += x2;
    }
  };
  for (size_t c = (size_t)blockIdx.x * waves + wave; c < chunks; c += stride) {
    const size_t e0 = c * (64 * K) + (size_t)lane * K;  // this lane's first element
    const size_t row = e0 >> lg;
    const int kx0 = (int)(e0 & (size_t)(n - 1));
    const int ky = (int)(row & (size_t)(n - 1));
    const int kz = (int)(row >> lg);  // 0 in 2-D
    const float fy = (float)(ky < n / 2 ? ky : ky - n);
    const float fz = (float)(kz < n / 2 ? kz : kz - n);
    const float r2 = fy * fy + fz * fz;
    int sk[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int kx = kx0 + j;
      const float fx = (float)(kx < n / 2 ? kx : kx - n);
      const int k = (int)rintf(sqrtf(fx * fx + r2));
      sk[j] = k < nsh ? k : nsh;  // nsh: outside the last shell
    }
    // kappa is monotone over the lane's elements: one inside means an end is.
    // C(k) and C(-k) (same shell): -k is (n - kx, n - ky, n - kz) mod n.
    float2 ck[K], cm[K];
    const bool any_in = sk[0] < nsh || sk[K - 1] < nsh;
    const size_t mrow = (((size_t)((n - kz) & (n - 1)) * n + (size_t)((n - ky) & (n - 1)))) * n;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      ck[j] = any_in ? spec[e0 + j] : make_float2(0.f, 0.f);
      cm[j] = any_in ? spec[mrow + ((n - kx0 - j) & (n - 1))] : make_float2(0.f, 0.f);
    }
    // runs inside the lane: f = first run, q = current run
    double f0 = 0.0, f1 = 0.0, f2 = 0.0, q0 = 0.0, q1 = 0.0, q2 = 0.0;
    int sf = sk[0], sq = sk[0];
    bool multi = false;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      // A = ((Cr + Cmr) + i (Ci - Cmi)) / 2,  B = ((Ci + Cmi) + i (Cmr - Cr)) / 2
      const double ax = 0.5 * ((double)ck[j].x + cm[j].x), ay = 0.5 * ((double)ck[j].y - cm[j].y);
      const double bx = 0.5 * ((double)ck[j].y + cm[j].y), by = 0.5 * ((double)cm[j].x - ck[j].x);
      double v0 = ax * bx + ay * by;
      double v1 = ax * ax + ay * ay;
      double v2 = bx * bx + by * by;
      if (sk[j] == nsh) v0 = v1 = v2 = 0.0;
      if (j == 0) {
        f0 = v0;
        f1 = v1;
        f2 = v2;
      } else if (sk[j] == sq) {
        if (multi) {
          q0 += v0;
          q1 += v1;
          q2 += v2;
        } else {
          f0 += v0;
          f1 += v1;
          f2 += v2;
        }
      } else {
        if (multi) put(sq, q0, q1, q2);  // a run inside the lane is complete
        multi = true;
        sq = sk[j];
        q0 = v0;
        q1 = v1;
        q2 = v2;
      }
    }
    const int sl = multi ? sq : sf;  // kappa of the lane's last run
    const int sl_prev = __shfl_up(sl, 1, 64);
    const bool join = lane > 0 && sl_prev == sf;
    int A = !multi && join ? 1 : 0;
    double B0 = multi ? q0 : f0, B1 = multi ? q1 : f1, B2 = multi ? q2 : f2;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int Ap = __shfl_up(A, d, 64);
      const double P0 = __shfl_up(B0, d, 64);
      const double P1 = __shfl_up(B1, d, 64);
      const double P2 = __shfl_up(B2, d, 64);
      if (lane >= d) {
        if (A) {
          B0 += P0;
          B1 += P1;
          B2 += P2;
        }
        A &= Ap;
      }
    }
    // B is now the sum of this lane's last run and the run it continues
    const double in0 = __shfl_up(B0, 1, 64), in1 = __shfl_up(B1, 1, 64), in2 = __shfl_up(B2, 1, 64);
    if (multi) put(sf, join ? f0 + in0 : f0, join ? f1 + in1 : f1, join ? f2 + in2 : f2);
    const int sf_next = __shfl_down(sf, 1, 64);
    if (!(lane < 63 && sf_next == sl)) put(sl, B0, B1, B2);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * nsh; i += blockDim.x) {
    double t = sh[i];
    for (int w = 1; w < waves; ++w) t += sh[w * 3 * nsh + i];
    partial[(size_t)blockIdx.x * 3 * nsh + i] = t;
  }
}

__global__ void fsc_final_kernel(const double* __restrict__ partial, int blocks, int len, double* __restrict__ out) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < len; j += gridDim.x * blockDim.x) {
    double t = 0.0;
    for (int b = 0; b < blocks; ++b) t += partial[(size_t)b * len + j];
    out[j] = t;
  }
}

// three 49 KB workgroups per CU: one round over the 256 CUs
int fsc_blocks() { return 768; }

hipError_t launch_fsc_pack(const float2* g1, const float2* g2, int part, float2* dst, size_t m, double* partial,
                           float* scale, hipStream_t st) {
  hipLaunchKernelGGL(fsc_norm_kernel, dim3(fsc_blocks()), dim3(kFscThreads), 0, st, g1, g2, part, m, partial);
  hipLaunchKernelGGL(fsc_scale_kernel, dim3(1), dim3(64), 0, st, partial, fsc_blocks(), m, scale);
  hipLaunchKernelGGL(fsc_pack_kernel, dim3(4096), dim3(256), 0, st, g1, g2, part, scale, dst, m);
  return hipGetLastError();
}

hipError_t launch_fsc_shells(const float2* spec, int n, int dims, double* partial, double* out, hipStream_t st) {
  const int nsh = n / 2 + 1;
  const int threads = n > 1024 ? kFscThreads / 2 : kFscThreads;
  const size_t lds = sizeof(double) * (threads / 64) * 3 * nsh;
  // four elements per lane where 256 divides n/2, else one (64 divides n/2 from n = 128)
  if (n >= 512)
    hipLaunchKernelGGL(fsc_shell_kernel<4>, dim3(fsc_blocks()), dim3(threads), lds, st, spec, n, dims, partial);
  else
    hipLaunchKernelGGL(fsc_shell_kernel<1>, dim3(fsc_blocks()), dim3(threads), lds, st, spec, n, dims, partial);
  hipLaunchKernelGGL(fsc_final_kernel, dim3((3 * nsh + 255) / 256), dim3(256), 0, st, partial, fsc_blocks(),
                     3 * nsh, out);
  return hipGetLastError();
}

}  // namespace pwf

namespace pwf {

// Quadratic background removal after tomography (Methods, "Reconstruction
// procedure"): per slice, the least-squares quadratic in x, z (voxel-centre
// coordinates over n/2) fitted separately to the real and imaginary parts of
// the voxels at radius >= r_bg, subtracted from the whole slice.  The normal
// matrix depends only on the grid and the radius; the host inverts it once.
// Each slice is split into kBgRows-row bands, one workgroup per band.
constexpr int kBgThreads = 256;

__device__ __forceinline__ void bg_monomials(double x, double z, double (&m)[6]) {
  m[0] = 1.0;
  m[1] = x;
  m[2] = z;
  m[3] = x * x;
  m[4] = x * z;
  m[5] = z * z;
}

// partial[(slice * bands + band) * 12 + p * 6 + k] = sum over the band's
// background voxels of monomial k times part p (0 real, 1 imaginary).
__global__ void __launch_bounds__(kBgThreads) bg_moments_kernel(const float2* __restrict__ vol, int n, int rows,
                                                               double r2_bg, double* __restrict__ partial) {
  const int bands = n / rows;
  const int slice = blockIdx.x / bands, band = blockIdx.x - slice * bands;
  const double h = 0.5 * n, inv_h = 1.0 / h;
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  // kBgCols columns per lane at a time, their loads issued before the sums
  constexpr int kBgCols = 4;
  for (int r = 0; r < rows; ++r) {
    const int iz = band * rows + r;
    const double Z = (double)iz + 0.5 - h;
    const float2* row = vol + ((size_t)slice * n + iz) * n;
    for (int ix0 = threadIdx.x; ix0 < n; ix0 += kBgCols * kBgThreads) {
      float2 v[kBgCols];
      bool bg[kBgCols];
#pragma unroll
      for (int u = 0; u < kBgCols; ++u) {
        const int ix = ix0 + u * kBgThreads;
        const double X = (double)ix + 0.5 - h;
        bg[u] = ix < n && X * X + Z * Z >= r2_bg;
        v[u] = bg[u] ? row[ix] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < kBgCols; ++u) {
        if (!bg[u]) continue;
        double m[6];
        bg_monomials(((double)(ix0 + u * kBgThreads) + 0.5 - h) * inv_h, Z * inv_h, m);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          acc[k] = fma(m[k], (double)v[u].x, acc[k]);
          acc[6 + k] = fma(m[k], (double)v[u].y, acc[6 + k]);
        }
      }
    }
  }
  // fixed-order reduction: wave butterflies, then the waves in order
  __shared__ double red[kBgThreads / 64][12];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    double a = acc[k];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = a;
  }
  __syncthreads();
  if (threadIdx.x < 12) {
    double a = 0.0;
    for (int w = 0; w < kBgThreads / 64; ++w) a += red[w][threadIdx.x];
    partial[(size_t)blockIdx.x * 12 + threadIdx.x] = a;
  }
}

// Coefficients of every slice (band sums in order, times the inverse normal
// matrix), then the surface subtracted over the band.  coef[slice * 12 + p * 6
// + k]: coefficient k of part p, written by the slice's first band.
__global__ void __launch_bounds__(kBgThreads) bg_subtract_kernel(float2* __restrict__ vol, int n, int rows,
                                                                const double* __restrict__ partial,
                                                                const double* __restrict__ minv,
                                                                double* __restrict__ coef) {
  const int bands = n / rows;
  const int slice = blockIdx.x / bands, band = blockIdx.x - slice * bands;
  __shared__ double mom[12], c[12];
  if (threadIdx.x < 12) {
    double a = 0.0;
    for (int b = 0; b < bands; ++b) a += partial[((size_t)slice * bands + b) * 12 + threadIdx.x];
    mom[threadIdx.x] = a;
  }
  __syncthreads();
  if (threadIdx.x < 12) {
    const int p = threadIdx.x / 6, k = threadIdx.x % 6;
    double a = 0.0;
    for (int j = 0; j < 6; ++j) a = fma(minv[k * 6 + j], mom[p * 6 + j], a);
    c[threadIdx.x] = a;
    if (band == 0) coef[(size_t)slice * 12 + threadIdx.x] = a;
  }
  __syncthreads();
  const double h = 0.5 * n, inv_h = 1.0 / h;
  for (int r = 0; r < rows; ++r) {
    const int iz = band * rows + r;
    const double z = ((double)iz + 0.5 - h) * inv_h;
    float2* row = vol + ((size_t)slice * n + iz) * n;
    for (int ix = threadIdx.x; ix < n; ix += kBgThreads) {
      double m[6];
      bg_monomials(((double)ix + 0.5 - h) * inv_h, z, m);
      double bre = 0.0, bim = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        bre = fma(c[k], m[k], bre);
        bim = fma(c[6 + k], m[k], bim);
      }
      const float2 v = row[ix];
      row[ix] = make_float2((float)((double)v.x - bre), (float)((double)v.y - bim));
    }
  }
}

int bg_rows_per_band(int n) { return n % 64 == 0 ? 64 : 16; }

hipError_t launch_bg_moments(const float2* vol, int n_slices, int n, double r_bg, double* partial, hipStream_t st) {
  const int rows = bg_rows_per_band(n);
  const size_t blocks = (size_t)n_slices * (n / rows);
  hipLaunchKernelGGL(bg_moments_kernel, dim3((unsigned)blocks), dim3(kBgThreads), 0, st, vol, n, rows, r_bg * r_bg,
                     partial);
  return hipGetLastError();
}

hipError_t launch_bg_subtract(float2* vol, int n_slices, int n, const double* partial, const double* minv,
                              double* coef, hipStream_t st) {
  const int rows = bg_rows_per_band(n);
  const size_t blocks = (size_t)n_slices * (n / rows);
  hipLaunchKernelGGL(bg_subtract_kernel, dim3((unsigned)blocks), dim3(kBgThreads), 0, st, vol, n, rows, partial,
                     minv, coef);
  return hipGetLastError();
}

}  // namespace pwf
