// Element-wise, reduction and utility kernels of libpwf, and the host-side
// dispatch of the per-side sweep instantiations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "pwf_device.h"
#include "pwf_kernels.h"

namespace pwf {

__device__ __forceinline__ float2 cexp_c(float2 p) {
  float s, c;
  sincosf(p.y, &s, &c);
  const float a = expf(p.x);
  return make_float2(a * c, a * s);
}

// Multiply a natural-order spectrum by one of the Algorithm S2 windows and 1/m.
__global__ void plain_window(float2* __restrict__ a, const Inst* __restrict__ ip, int which) {
  const Inst& I = *ip;
  const int nx = I.nx, ny = I.ny;
  const size_t m = (size_t)nx * ny;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x) {
    const int ky = (int)(i / nx), kx = (int)(i - (size_t)ky * nx);
    const float fx = freq_of(kx, nx), fy = freq_of(ky, ny);
    float2 val = a[i];
    switch (which) {
      case PLAIN_W_Q1: val = cmul(val, transfer(I.chirp1_rev, I.s_coef, I.series, fx, fy, false)); break;
      case PLAIN_W_Q2: val = cmul(val, transfer(I.chirp2_rev, I.s_coef, I.series, fx, fy, false)); break;
      case PLAIN_W_Q2C: val = cmul(val, transfer(I.chirp2_rev, I.s_coef, I.series, fx, fy, true)); break;
      case PLAIN_W_Q1C: val = cmul(val, transfer(I.chirp1_rev, I.s_coef, I.series, fx, fy, true)); break;
      case PLAIN_W_IOTF: val = cscale(val, iotf_at(I, kx, ky)); break;
      case PLAIN_W_PINV: val = cscale(val, pinv_of(I, fx, fy)); break;
      case PLAIN_W_GAMMA2: val = cscale(val, gamma2_at(I, kx, ky)); break;
      case PLAIN_W_WIENER: {
        const float h = iotf_at(I, kx, ky);
        val = cscale(val, h / (h * h + I.wiener_eps));
        break;
      }
      default: break;
    }
    a[i] = cscale(val, I.inv_m);
  }
}

// Element-wise steps of Algorithm S2 in natural layout.
__global__ void plain_elementwise(int op, size_t m, const float2* __restrict__ a, const float2* __restrict__ b,
                                  float2* __restrict__ c, float2* __restrict__ out,
                                  const Inst* __restrict__ ip, const double* beta, int iter,
                                  double* __restrict__ partial) {
  const Inst& I = *ip;
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x) {
    switch (op) {
      case PLAIN_EXP: out[i] = cexp_c(a[i]); break;
      case PLAIN_MUL_T: out[i] = cmul(a[i], I.t[i]); break;
      case PLAIN_MUL_CONJ_T: out[i] = cmulc(a[i], I.t[i]); break;
      case PLAIN_ABS2: out[i] = make_float2(a[i].x * a[i].x + a[i].y * a[i].y, 0.f); break;
      case PLAIN_REAL: out[i] = make_float2(a[i].x, 0.f); break;
      case PLAIN_NEG_ERR: {  // -e = f - y, and the loss sum of e^2
        const float e = I.y[i] - a[i].x;
        acc += (double)e * (double)e;
        out[i] = make_float2(-e, 0.f);
        break;
      }
      case PLAIN_MUL: out[i] = cmul(a[i], make_float2(b[i].x, 0.f)); break;  // v * Re(h)
      case PLAIN_GRAD: out[i] = cscale(cmulc(a[i], b[i]), 1.0f / *I.maxt2); break;  // b * conj(x) / max|t|^2
      case PLAIN_IMAG: out[i] = make_float2(a[i].y, 0.f); break;
      case PLAIN_DIRECTION: {  // d = Re g + i Re(Filter(Im g, P)) + Re a Re(rho) + i Im a Im(rho)
        out[i] = make_float2(a[i].x + (I.alpha_c1 + I.alpha_c2) * c[i].x,
                             b[i].x + (I.alpha_c1 - I.alpha_c2) * c[i].y);
        break;
      }
      case PLAIN_FROM_REAL: out[i] = make_float2(I.y[i], 0.f); break;
      case PLAIN_SQRT_POS: out[i] = make_float2(sqrtf(fmaxf(a[i].x, 0.f)), 0.f); break;
      case PLAIN_NESTEROV: {  // a = psi (in/out via out), b = d, c = z (updated in place)
        const float bf = (float)beta[iter];
        const float2 zp = c[i];
        const float2 z = make_float2(a[i].x - I.eta * b[i].x, a[i].y - I.eta * b[i].y);
        c[i] = z;
        out[i] = make_float2(z.x + bf * (z.x - zp.x), z.y + bf * (z.y - zp.y));
        break;
      }
      default: break;
    }
  }
  if (op == PLAIN_NEG_ERR) {
    __shared__ double red[16];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int i = 0; i < (int)(blockDim.x >> 6); ++i) sum += red[i];
      partial[blockIdx.x] = sum;
    }
  }
}

__global__ void plain_loss_final(const double* partial, int np, double* dst, int iter, int32_t* status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < np; ++i) s += partial[i];
    if (dst) dst[iter] = s;
    if (!isfinite(s)) atomicOr(status, 1);
  }
}

// Loss of every instance from its column-tile partials (fixed order, FP64),
// when no back-blur sweep follows to sum them: one workgroup per instance.
__global__ void loss_final_kernel(const Inst* __restrict__ insts, int32_t* status) {
  const Inst& I = insts[blockIdx.x];
  if (threadIdx.x == 0 && I.loss_dst) {
    double s = 0.0;
    for (int i = 0; i < I.n_partials; ++i) s += I.loss_partial[i];
    s *= I.inv_m_d;
    I.loss_dst[0] = s;
    if (!isfinite(s)) atomicOr(status, 1);
  }
}

// ------------------------------------------------------------------ utilities

__global__ void fill_zero_kernel(float4* __restrict__ p, size_t n16) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// max_r |t_r|^2 of one diffuser: per-block maxima, then the last pass reduces them.
__global__ void maxabs2_partial(const float2* __restrict__ t, size_t m, float* __restrict__ partial) {
  float mx = 0.f;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x) {
    const float2 a = t[i];
    mx = fmaxf(mx, a.x * a.x + a.y * a.y);
  }
  __shared__ float red[16];
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) mx = fmaxf(mx, red[i]);
    partial[blockIdx.x] = fmaxf(mx, red[0]);
  }
}

__global__ void maxabs2_final(const float* __restrict__ partial, int np, float* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float mx = 0.f;
    for (int i = 0; i < np; ++i) mx = fmaxf(mx, partial[i]);
    *out = mx;
  }
}

// max |t|^2 of up to kMaxabs2Batch diffusers in one launch pair (blockIdx.y =
// diffuser): the same per-block partials and the same final reduction order
// as maxabs2_partial / maxabs2_final.
__global__ void maxabs2_partial_multi(Maxabs2Batch B, float* __restrict__ partial) {
  const int d = blockIdx.y;
  const float2* __restrict__ t = B.t[d];
  const size_t m = B.m[d];
  float mx = 0.f;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x) {
    const float2 a = t[i];
    mx = fmaxf(mx, a.x * a.x + a.y * a.y);
  }
  __shared__ float red[16];
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) mx = fmaxf(mx, red[i]);
    partial[(size_t)d * gridDim.x + blockIdx.x] = fmaxf(mx, red[0]);
  }
}

__global__ void maxabs2_final_multi(Maxabs2Batch B, const float* __restrict__ partial, int np) {
  if (threadIdx.x == 0) {
    const int d = blockIdx.x;
    float mx = 0.f;
    for (int i = 0; i < np; ++i) mx = fmaxf(mx, partial[(size_t)d * np + i]);
    *B.out[d] = mx;
  }
}

// 1-D factors of the separable windows of one instance (FP64 arguments).
__global__ void build_tables_kernel(const Inst* __restrict__ insts) {
  const Inst I = insts[blockIdx.x];
  for (int k = threadIdx.x; k < I.nx + I.ny; k += blockDim.x) {
    const bool isx = k < I.nx;
    const int kk = isx ? k : k - I.nx;
    const int n = isx ? I.nx : I.ny;
    const double f = (double)(kk < (n >> 1) ? kk : kk - n) / (double)n;
    const double f2 = f * f;
    float2 q[2];
    const double a[2] = {I.chirp1_rev, I.chirp2_rev};
    for (int j = 0; j < 2; ++j) {
      double rev = -a[j] * f2;
      rev -= rint(rev);
      float sn, cs;
      sincosf((float)(rev * 6.283185307179586476925), &sn, &cs);
      q[j] = make_float2(cs, sn);
    }
    const float cio = isx ? I.iotf_cx : I.iotf_cy;
    const float cst = isx ? I.stf_cx : I.stf_cy;
    const float ff = (float)f2;
    // IOTF factor and 1 - STF factor: Eq. 5 / Eq. 14 in closed form, or from the
    // caller's separable IOTF with STF = IOTF^(2 gamma)
    const float* src = isx ? I.src_ix : I.src_iy;
    float iotf, g2;
    if (src) {
      iotf = src[kk];
      g2 = 1.f - powf(fmaxf(iotf, 0.f), I.two_gamma);
    } else {
      iotf = expf(-cio * ff);
      g2 = -expm1f(-cst * ff);
    }
    if (isx) {
      I.qx1[kk] = q[0];
      I.qx2[kk] = q[1];
      // (y factors below carry the 1/m of the inverse 2-D transform: exact, m = 2^k)
      I.ix[kk] = iotf;
      I.gx[kk] = g2;
    } else {
      I.qy1[kk] = make_float2(q[0].x * I.inv_m, q[0].y * I.inv_m);
      I.qy2[kk] = make_float2(q[1].x * I.inv_m, q[1].y * I.inv_m);
      I.iy[kk] = iotf;
      I.gy[kk] = g2;
    }
  }
}

hipError_t launch_build_tables(const Inst* insts, int n, hipStream_t st) {
  hipLaunchKernelGGL(build_tables_kernel, dim3(n), dim3(256), 0, st, insts);
  return hipGetLastError();
}

// ------------------------------------------------------------------ host dispatch

#define PWF_DECLARE_SIDE(N)                                                                              \
  template <int M> hipError_t launch_row_n(int op, int plan, int nblocks, const Sweep& S, hipStream_t st); \
  template <int M> hipError_t launch_col_n(int w, int op, int nblocks, const Sweep& S, hipStream_t st); \
  template <int M> hipError_t plain_rows_n(int dir, const float2* src, float2* dst, int ny,             \
                                           const float2* tw, hipStream_t st);                          \
  template <int M> hipError_t plain_cols_n(int dir, float2* a, int nx, const float2* tw, int planes,   \
                                           size_t plane_stride, hipStream_t st);                       \
  template <int M> int plan_twiddles_n(int which, float2* out);                                       \
  extern template hipError_t launch_row_n<N>(int, int, int, const Sweep&, hipStream_t);                \
  extern template hipError_t launch_col_n<N>(int, int, int, const Sweep&, hipStream_t);                \
  extern template hipError_t plain_rows_n<N>(int, const float2*, float2*, int, const float2*, hipStream_t); \
  extern template hipError_t plain_cols_n<N>(int, float2*, int, const float2*, int, size_t, hipStream_t); \
  extern template int plan_twiddles_n<N>(int, float2*);
PWF_DECLARE_SIDE(128)
PWF_DECLARE_SIDE(256)
PWF_DECLARE_SIDE(512)
PWF_DECLARE_SIDE(1024)
PWF_DECLARE_SIDE(2048)
#undef PWF_DECLARE_SIDE

bool row_alt_default_n(int n, int op) {
  switch (n) {
    case 128: return row_alt_default<128>(op);
    case 256: return row_alt_default<256>(op);
    case 512: return row_alt_default<512>(op);
    case 1024: return row_alt_default<1024>(op);
    case 2048: return row_alt_default<2048>(op);
    default: return false;
  }
}

int row_plan_count_n(int n) {
  switch (n) {
    case 128: return row_plan_count<128>();
    case 256: return row_plan_count<256>();
    case 512: return row_plan_count<512>();
    case 1024: return row_plan_count<1024>();
    case 2048: return row_plan_count<2048>();
    default: return 0;
  }
}

template <int N> int rows_per_block_of(int plan) {
  return plan == 2 ? RowCfgAlt2<N>::RW : plan == 1 ? RowCfgAlt<N>::RW : RowCfg<N>::RW;
}

int row_rows_per_block(int n, int plan) {
  switch (n) {
    case 128: return rows_per_block_of<128>(plan);
    case 256: return rows_per_block_of<256>(plan);
    case 512: return rows_per_block_of<512>(plan);
    case 1024: return rows_per_block_of<1024>(plan);
    case 2048: return rows_per_block_of<2048>(plan);
    default: return 0;
  }
}

int col_default_width(int n) {
  switch (n) {
    case 128: return ColSweepCfg<128>::WA;
    case 256: return ColSweepCfg<256>::WA;
    case 512: return ColSweepCfg<512>::WA;
    case 1024: return ColSweepCfg<1024>::WA;
    case 2048: return ColSweepCfg<2048>::WA;
    default: return 0;
  }
}

bool col_width_supported(int n, int w) {
  switch (n) {
    case 128: return w == ColSweepCfg<128>::WA || w == ColSweepCfg<128>::WB;
    case 256: return w == ColSweepCfg<256>::WA || w == ColSweepCfg<256>::WB;
    case 512: return w == ColSweepCfg<512>::WA || w == ColSweepCfg<512>::WB;
    case 1024: return w == ColSweepCfg<1024>::WA || w == ColSweepCfg<1024>::WB;
    case 2048: return w == ColSweepCfg<2048>::WA || w == ColSweepCfg<2048>::WB;
    default: return false;
  }
}

int col_alt_width(int n) {
  switch (n) {
    case 128: return ColSweepCfg<128>::WB;
    case 256: return ColSweepCfg<256>::WB;
    case 512: return ColSweepCfg<512>::WB;
    case 1024: return ColSweepCfg<1024>::WB;
    case 2048: return ColSweepCfg<2048>::WB;
    default: return 0;
  }
}

hipError_t launch_row(int nx, int op, int plan, int nblocks, const Sweep& S, hipStream_t st) {
  switch (nx) {
    case 128: return launch_row_n<128>(op, plan, nblocks, S, st);
    case 256: return launch_row_n<256>(op, plan, nblocks, S, st);
    case 512: return launch_row_n<512>(op, plan, nblocks, S, st);
    case 1024: return launch_row_n<1024>(op, plan, nblocks, S, st);
    case 2048: return launch_row_n<2048>(op, plan, nblocks, S, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_col(int ny, int width, int op, int nblocks, const Sweep& S, hipStream_t st) {
  switch (ny) {
    case 128: return launch_col_n<128>(width, op, nblocks, S, st);
    case 256: return launch_col_n<256>(width, op, nblocks, S, st);
    case 512: return launch_col_n<512>(width, op, nblocks, S, st);
    case 1024: return launch_col_n<1024>(width, op, nblocks, S, st);
    case 2048: return launch_col_n<2048>(width, op, nblocks, S, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_plain_rows(int nx, int dir, const float2* src, float2* dst, int ny, const float2* tw,
                             hipStream_t st) {
  switch (nx) {
    case 128: return plain_rows_n<128>(dir, src, dst, ny, tw, st);
    case 256: return plain_rows_n<256>(dir, src, dst, ny, tw, st);
    case 512: return plain_rows_n<512>(dir, src, dst, ny, tw, st);
    case 1024: return plain_rows_n<1024>(dir, src, dst, ny, tw, st);
    case 2048: return plain_rows_n<2048>(dir, src, dst, ny, tw, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_plain_cols(int ny, int dir, float2* a, int nx, const float2* tw, hipStream_t st, int planes,
                             size_t plane_stride) {
  if (planes < 1 || planes > 65535) return hipErrorInvalidValue;
  switch (ny) {
    case 128: return plain_cols_n<128>(dir, a, nx, tw, planes, plane_stride, st);
    case 256: return plain_cols_n<256>(dir, a, nx, tw, planes, plane_stride, st);
    case 512: return plain_cols_n<512>(dir, a, nx, tw, planes, plane_stride, st);
    case 1024: return plain_cols_n<1024>(dir, a, nx, tw, planes, plane_stride, st);
    case 2048: return plain_cols_n<2048>(dir, a, nx, tw, planes, plane_stride, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_plain_window(float2* a, const Inst* inst, int which, size_t m, hipStream_t st) {
  const int blocks = (int)((m + 255) / 256 < 4096 ? (m + 255) / 256 : 4096);
  hipLaunchKernelGGL(plain_window, dim3(blocks), dim3(256), 0, st, a, inst, which);
  return hipGetLastError();
}

int plain_elementwise_blocks() { return 1024; }

hipError_t launch_plain_elementwise(int op, size_t m, const float2* a, const float2* b, float2* c, float2* out,
                                    const Inst* inst, const double* beta, int iter, double* partial,
                                    hipStream_t st) {
  hipLaunchKernelGGL(plain_elementwise, dim3(plain_elementwise_blocks()), dim3(256), 0, st, op, m, a, b, c, out,
                     inst, beta, iter, partial);
  return hipGetLastError();
}

hipError_t launch_plain_loss_final(const double* partial, int np, double* dst, int iter, int32_t* status,
                                   hipStream_t st) {
  hipLaunchKernelGGL(plain_loss_final, dim3(1), dim3(64), 0, st, partial, np, dst, iter, status);
  return hipGetLastError();
}

hipError_t launch_loss_final(const Inst* insts, int n, int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(loss_final_kernel, dim3(n), dim3(64), 0, st, insts, status);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  const size_t want = (n16 + 255) / 256;
  const int blocks = (int)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, st, (float4*)p, n16);
  return hipGetLastError();
}

int maxabs2_blocks() { return 256; }

// Joint diffuser refinement: normalisation sum_j max|u1_j|^2 from the S2
// workgroup maxima (n instances, `count` maxima each, `stride` floats apart).
// One workgroup per instance takes its maximum (order-free, so deterministic)
// and leaves it in the instance's first entry, which the next S2 rewrites;
// one thread then sums the n maxima in instance order in FP64.
__global__ void __launch_bounds__(256) joint_max_kernel(float* __restrict__ u1max, int count, size_t stride) {
  float* p = u1max + (size_t)blockIdx.x * stride;
  __shared__ float red[4];
  float mx = 0.f;
  for (int b = threadIdx.x; b < count; b += blockDim.x) mx = fmaxf(mx, p[b]);
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) p[0] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__global__ void __launch_bounds__(256) joint_norm_kernel(const float* __restrict__ u1max, int n, size_t stride,
                                                         double* __restrict__ dsum) {
  __shared__ float v[256];
  double acc = 0.0;
  for (int j0 = 0; j0 < n; j0 += 256) {  // maxima gathered in parallel, summed in order
    const int m = min(256, n - j0);
    if ((int)threadIdx.x < m) v[threadIdx.x] = u1max[(size_t)(j0 + threadIdx.x) * stride];
    __syncthreads();
    if (threadIdx.x == 0)
      for (int j = 0; j < m; ++j) acc += (double)v[j];
    __syncthreads();
  }
  if (threadIdx.x == 0) *dsum = acc;
}

// t <- t - eta_t sum_j G_j / dsum, G_j = conj(u1_j) a2_j of instance j (fields
// `stride` elements apart); the sum over instances runs in order, in FP64.
__global__ void joint_update_kernel(const float2* __restrict__ g, int n, size_t stride, size_t m,
                                    float2* __restrict__ t, double eta_t, const double* __restrict__ dsum) {
  const double scale = eta_t / *dsum;
  for (size_t r = blockIdx.x * (size_t)blockDim.x + threadIdx.x; r < m; r += (size_t)gridDim.x * blockDim.x) {
    double gx = 0.0, gy = 0.0;
    for (int j = 0; j < n; ++j) {
      const float2 a = g[(size_t)j * stride + r];
      gx += a.x;
      gy += a.y;
    }
    const float2 tv = t[r];
    t[r] = make_float2((float)((double)tv.x - scale * gx), (float)((double)tv.y - scale * gy));
  }
}

hipError_t launch_joint_update(float* u1max, int n, int count, size_t max_stride, const float2* g,
                               size_t field_stride, size_t m, float2* t, double eta_t, double* dsum,
                               hipStream_t st) {
  hipLaunchKernelGGL(joint_max_kernel, dim3(n), dim3(256), 0, st, u1max, count, max_stride);
  hipLaunchKernelGGL(joint_norm_kernel, dim3(1), dim3(256), 0, st, u1max, n, max_stride, dsum);
  const int blocks = (int)std::min<size_t>((m + 255) / 256, 4096);
  hipLaunchKernelGGL(joint_update_kernel, dim3(blocks), dim3(256), 0, st, g, n, field_stride, m, t, eta_t, dsum);
  return hipGetLastError();
}

// Speckle autocorrelation sums (Siegert calibration).  Each thread takes
// pixels in a grid-stride loop and accumulates, for every shift d, the
// products with the pixels d to the right and d below (circular), in FP64.
__global__ void __launch_bounds__(256) speckle_sums_kernel(const float* __restrict__ img, int nx, int ny, int max_shift,
                                    double* __restrict__ partial) {
  constexpr int K = kMaxShift + 1;
  constexpr int NV = 1 + 2 * K;
  double acc[NV];  // [0]: sum I; [1 + d]: x shift d; [1 + K + d]: y shift d
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  const size_t m = (size_t)nx * ny;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / nx), x = (int)(i - (size_t)y * nx);
    const float v = img[i];
    acc[0] += v;
#pragma unroll
    for (int d = 0; d < K; ++d) {
      if (d <= max_shift) {
        const int xd = x + d < nx ? x + d : x + d - nx;
        const int yd = y + d < ny ? y + d : y + d - ny;
        acc[1 + d] += (double)(v * img[(size_t)y * nx + xd]);
        acc[1 + K + d] += (double)(v * img[(size_t)yd * nx + x]);
      }
    }
  }
  // block reduction, one value at a time (wave butterflies, then waves in order)
  __shared__ double red[16];
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    double a = acc[j];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
      partial[(size_t)blockIdx.x * NV + j] = t;
    }
    __syncthreads();
  }
}

__global__ void speckle_sums_final(const double* __restrict__ partial, int blocks, int nv, double* __restrict__ out) {
  for (int j = threadIdx.x; j < nv; j += blockDim.x) {
    double t = 0.0;
    for (int b = 0; b < blocks; ++b) t += partial[(size_t)b * nv + j];
    out[j] = t;
  }
}

int speckle_sum_blocks() { return 512; }

hipError_t launch_speckle_sums(const float* img, int nx, int ny, int max_shift, double* partial, double* out,
                               hipStream_t st) {
  if (max_shift < 0 || max_shift > kMaxShift) return hipErrorInvalidValue;
  hipLaunchKernelGGL(speckle_sums_kernel, dim3(speckle_sum_blocks()), dim3(256), 0, st, img, nx, ny, max_shift,
                     partial);
  hipLaunchKernelGGL(speckle_sums_final, dim3(1), dim3(128), 0, st, partial, speckle_sum_blocks(),
                     1 + 2 * (kMaxShift + 1), out);
  return hipGetLastError();
}

hipError_t launch_maxabs2_batch(const Maxabs2Batch& B, float* partial, hipStream_t st) {
  if (B.n < 1 || B.n > kMaxabs2Batch) return hipErrorInvalidValue;
  hipLaunchKernelGGL(maxabs2_partial_multi, dim3(maxabs2_blocks(), B.n), dim3(256), 0, st, B, partial);
  hipLaunchKernelGGL(maxabs2_final_multi, dim3(B.n), dim3(64), 0, st, B, partial, maxabs2_blocks());
  return hipGetLastError();
}

hipError_t launch_maxabs2(const float2* t, size_t m, float* partial, float* out, hipStream_t st) {
  hipLaunchKernelGGL(maxabs2_partial, dim3(maxabs2_blocks()), dim3(256), 0, st, t, m, partial);
  hipLaunchKernelGGL(maxabs2_final, dim3(1), dim3(64), 0, st, partial, maxabs2_blocks(), out);
  return hipGetLastError();
}

int plan_twiddles(int n, int which, float2* out) {
  switch (n) {
    case 128: return plan_twiddles_n<128>(which, out);
    case 256: return plan_twiddles_n<256>(which, out);
    case 512: return plan_twiddles_n<512>(which, out);
    case 1024: return plan_twiddles_n<1024>(which, out);
    case 2048: return plan_twiddles_n<2048>(which, out);
    default: return -1;
  }
}

}  // namespace pwf
