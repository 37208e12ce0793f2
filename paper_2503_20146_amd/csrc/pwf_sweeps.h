// Sweep kernel templates of the PWF hot path (instantiated once per grid side
// in pwf_sweeps_<N>.hip so that the sides compile in parallel).
#pragma once


#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "pwf_device.h"
#include "pwf_kernels.h"

namespace pwf {

// ------------------------------------------------------------------ row sweeps

template <int OP> struct RowOpTraits;
#define PWF_ROW_TRAIT(op, in_freq, out_freq) \
  template <> struct RowOpTraits<op> { static constexpr bool kInFreq = in_freq, kOutFreq = out_freq; };
PWF_ROW_TRAIT(ROW_PSI_UPDATE, true, true)
PWF_ROW_TRAIT(ROW_START, false, true)
PWF_ROW_TRAIT(ROW_MUL_T, true, true)
PWF_ROW_TRAIT(ROW_MUL_CONJ_T, true, true)
PWF_ROW_TRAIT(ROW_INTENSITY, true, true)
PWF_ROW_TRAIT(ROW_BACKBLUR, true, true)
PWF_ROW_TRAIT(ROW_GRAD, true, true)
PWF_ROW_TRAIT(ROW_FORWARD_OUT, true, false)
PWF_ROW_TRAIT(ROW_REAL_FFT, false, true)
PWF_ROW_TRAIT(ROW_CPLX_FFT, false, true)
PWF_ROW_TRAIT(ROW_IFFT_OUT, true, false)
#undef PWF_ROW_TRAIT

__device__ __forceinline__ float2 cexp_f(float2 p) {
  float s, c;
  sincosf(p.y, &s, &c);
  const float a = expf(p.x);
  return make_float2(a * c, a * s);
}

template <int NX, int OP>
__global__ void __launch_bounds__(RowCfg<NX>::T * RowCfg<NX>::RW) row_sweep(Sweep S) {
  using C = RowCfg<NX>;
  using Plan = typename C::Plan;
  constexpr int T = C::T, RW = C::RW, E = NX / T;
  constexpr int R1 = Plan::radix[0], RL = Plan::radix[Plan::NPASS - 1];
  constexpr int M1 = NX / R1, ML = NX / RL;
  constexpr bool IN_FREQ = RowOpTraits<OP>::kInFreq, OUT_FREQ = RowOpTraits<OP>::kOutFreq;
  __shared__ float2 lds[RW * lds_len(NX)];

  const int inst = blockIdx.x / S.blocks_per_inst;
  const int blk = blockIdx.x - inst * S.blocks_per_inst;
  const Inst& I = S.inst[inst];
  const int t = threadIdx.x % T, rw = threadIdx.x / T;
  const int row = blk * RW + rw;
  const LdsView lv{lds + rw * lds_len(NX), 1};
  const float2* tw = S.tw_row;
  const float2* twr = S.tw_row + Plan::tw_total();
  const size_t rbase = (size_t)row * NX;

  float2 v[E];
  if constexpr (IN_FREQ) {
    const float2* __restrict__ src = I.W + rbase;
    static_for<0, E / RL>([&](auto cc) {
      static_for<0, RL>([&](auto rr) {
        constexpr int c = decltype(cc)::value, r = decltype(rr)::value;
        v[c * RL + r] = src[col_of_kx(t + T * c + r * ML, NX)];
      });
    });
    fft_inverse<Plan, T>(v, t, twr, lv);
  } else if constexpr (OP == ROW_REAL_FFT) {
    const float* __restrict__ src = I.y + rbase;
    static_for<0, E / R1>([&](auto cc) {
      static_for<0, R1>([&](auto qq) {
        constexpr int c = decltype(cc)::value, q = decltype(qq)::value;
        v[c * R1 + q] = make_float2(src[t + T * c + q * M1], 0.f);
      });
    });
  } else {  // ROW_START / ROW_CPLX_FFT: complex real-space input (null = zeros)
    const float2* __restrict__ src = I.psi_src;
    static_for<0, E / R1>([&](auto cc) {
      static_for<0, R1>([&](auto qq) {
        constexpr int c = decltype(cc)::value, q = decltype(qq)::value;
        v[c * R1 + q] = src ? src[rbase + t + T * c + q * M1] : make_float2(0.f, 0.f);
      });
    });
  }

  // real-space step; element e = c*R1 + q sits at x = t + T c + q M1
  static_for<0, E / R1>([&](auto cc) {
    static_for<0, R1>([&](auto qq) {
      constexpr int c = decltype(cc)::value, q = decltype(qq)::value;
      constexpr int e = c * R1 + q;
      const size_t idx = rbase + t + T * c + q * M1;
      if constexpr (OP == ROW_PSI_UPDATE) {
        I.psi[idx] = v[e];
        v[e] = cexp_f(v[e]);
      } else if constexpr (OP == ROW_START) {
        v[e] = cexp_f(v[e]);
      } else if constexpr (OP == ROW_MUL_T) {
        v[e] = cmul(v[e], I.t[idx]);
      } else if constexpr (OP == ROW_MUL_CONJ_T) {
        v[e] = cmulc(v[e], I.t[idx]);
      } else if constexpr (OP == ROW_INTENSITY) {
        if (I.v) I.v[idx] = v[e];
        v[e] = make_float2(v[e].x * v[e].x + v[e].y * v[e].y, 0.f);
      } else if constexpr (OP == ROW_BACKBLUR) {
        const float h = v[e].x;
        const float2 vv = I.v[idx];
        v[e] = make_float2(vv.x * h, vv.y * h);
      } else if constexpr (OP == ROW_GRAD) {
        const float inv = 1.0f / *I.maxt2;
        const float2 x = cexp_f(I.psi[idx]);
        v[e] = cscale(cmulc(v[e], x), inv);
        if (I.g_out) I.g_out[idx] = v[e];
      } else if constexpr (OP == ROW_FORWARD_OUT) {
        I.f_out[idx] = v[e].x;
      } else if constexpr (OP == ROW_CPLX_FFT) {
        if (I.psi && I.psi != I.psi_src) I.psi[idx] = v[e];
      } else if constexpr (OP == ROW_IFFT_OUT) {
        if (I.out) I.out[idx] = v[e];
      }
    });
  });

  if constexpr (OUT_FREQ) {
    fft_forward<Plan, T>(v, t, tw, lv);
    float2* __restrict__ dst = I.W + rbase;
    static_for<0, E / RL>([&](auto cc) {
      static_for<0, RL>([&](auto rr) {
        constexpr int c = decltype(cc)::value, r = decltype(rr)::value;
        dst[col_of_kx(t + T * c + r * ML, NX)] = v[c * RL + r];
      });
    });
  }

  if constexpr (OP == ROW_BACKBLUR) {
    // Final FP64 sum of the column-tile partials of the loss (fixed order).
    if (blk == 0 && threadIdx.x == 0 && I.loss_dst) {
      double acc = 0.0;
      for (int i = 0; i < I.n_partials; ++i) acc += I.loss_partial[i];
      acc *= I.inv_m_d;
      I.loss_dst[S.iter] = acc;
      if (!isfinite(acc)) atomicOr(S.status, 1);
    }
  }
}

// ------------------------------------------------------------------ column sweeps

template <int OP> struct ColOpTraits;
#define PWF_COL_TRAIT(op, inv) \
  template <> struct ColOpTraits<op> { static constexpr bool kInverse = inv; };
PWF_COL_TRAIT(COL_CHIRP1, true)
PWF_COL_TRAIT(COL_CHIRP2, true)
PWF_COL_TRAIT(COL_CHIRP2_CONJ, true)
PWF_COL_TRAIT(COL_CHIRP1_CONJ, true)
PWF_COL_TRAIT(COL_BLUR_LOSS, true)
PWF_COL_TRAIT(COL_BLUR, true)
PWF_COL_TRAIT(COL_NESTEROV, true)
PWF_COL_TRAIT(COL_DIRECTION, true)
PWF_COL_TRAIT(COL_SPEC_YHAT, false)
PWF_COL_TRAIT(COL_SPEC_PSIHAT, false)
#undef PWF_COL_TRAIT

template <int NY, int OP>
__global__ void __launch_bounds__(ColCfg<NY>::T * ColCfg<NY>::W) col_sweep(Sweep S) {
  using C = ColCfg<NY>;
  using Plan = typename C::Plan;
  constexpr int T = C::T, W = C::W, E = NY / T;
  constexpr int R1 = Plan::radix[0], RL = Plan::radix[Plan::NPASS - 1];
  constexpr int M1 = NY / R1, ML = NY / RL;
  constexpr int NT = T * W;
  __shared__ float2 lds[W * lds_len(NY)];
  __shared__ double red[NT / 64];

  const int inst = blockIdx.x / S.blocks_per_inst;
  const int tile = blockIdx.x - inst * S.blocks_per_inst;
  const Inst& I = S.inst[inst];
  const int nx = I.nx;
  const int w = threadIdx.x % W, t = threadIdx.x / W;
  const int s = tile * W + w;
  const LdsView lv{lds + w, W};
  const float2* tw = S.tw_col;
  const float2* twr = S.tw_col + Plan::tw_total();

  float2 v[E];
  {
    const float2* __restrict__ src = I.W + s;
    static_for<0, E / R1>([&](auto cc) {
      static_for<0, R1>([&](auto qq) {
        constexpr int c = decltype(cc)::value, q = decltype(qq)::value;
        v[c * R1 + q] = src[(size_t)(t + T * c + q * M1) * nx];
      });
    });
  }
  fft_forward<Plan, T>(v, t, tw, lv);

  // Fourier-domain step; element e = c*RL + r holds ky = t + T c + r ML.
  const int kx = kx_of_col(s, nx);
  const float fx = freq_of(kx, nx);
  double acc = 0.0;

  if constexpr (OP == COL_NESTEROV || OP == COL_DIRECTION) {
    // Needs G(-k) and Psi(-k): exchange through LDS.  Column -kx is the
    // neighbour position mirror_col(s), inside this tile.
    const int wm = mirror_col(s) - tile * W;
    const LdsView lm{lds + wm, W};
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      constexpr int c = e / RL, r = e % RL;
      lv.at(t + T * c + r * ML) = v[e];
    });
    __syncthreads();
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      constexpr int c = e / RL, r = e % RL;
      const int ky = t + T * c + r * ML;
      const int kym = (NY - ky) & (NY - 1);
      const float2 gm = lm.at(kym);
      const float P = pinv_of(I, fx, freq_of(ky, NY));
      const float a = 0.5f * (1.f + P), b = 0.5f * (1.f - P);
      // (1+P)/2 G + (1-P)/2 conj(G(-k)) = F{Re g} + i P F{Im g}
      v[e] = make_float2(a * v[e].x + b * gm.x, a * v[e].y - b * gm.y);
    });
    __syncthreads();
    float2 ps[E];
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      constexpr int c = e / RL, r = e % RL;
      const int ky = t + T * c + r * ML;
      ps[e] = I.psi_hat[(size_t)ky * nx + s];
      lv.at(ky) = ps[e];
    });
    __syncthreads();
    const double beta = (OP == COL_NESTEROV) ? S.beta[I.k0 + S.iter] : 0.0;
    const float bf = (float)beta;
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      constexpr int c = e / RL, r = e % RL;
      const int ky = t + T * c + r * ML;
      const int kym = (NY - ky) & (NY - 1);
      const float2 pm = lm.at(kym);
      const float g2 = gamma2_of(I, fx, freq_of(ky, NY));
      // Re(a) F{Re psi} + i Im(a) F{Im psi} = c1 Psi + c2 conj(Psi(-k))
      const float2 reg = make_float2(I.alpha_c1 * ps[e].x + I.alpha_c2 * pm.x,
                                     I.alpha_c1 * ps[e].y - I.alpha_c2 * pm.y);
      const float2 d = make_float2(v[e].x + g2 * reg.x, v[e].y + g2 * reg.y);
      if constexpr (OP == COL_NESTEROV) {
        const size_t gi = (size_t)ky * nx + s;
        const float2 zp = I.z_hat[gi];
        const float2 z = make_float2(ps[e].x - I.eta * d.x, ps[e].y - I.eta * d.y);
        const float2 pn = make_float2(z.x + bf * (z.x - zp.x), z.y + bf * (z.y - zp.y));
        I.z_hat[gi] = z;
        I.psi_hat[gi] = pn;
        v[e] = cscale(pn, I.inv_m);
      } else {
        v[e] = cscale(d, I.inv_m);
      }
    });
    __syncthreads();
  } else {
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      constexpr int c = e / RL, r = e % RL;
      const int ky = t + T * c + r * ML;
      const float fy = freq_of(ky, NY);
      if constexpr (OP == COL_CHIRP1 || OP == COL_CHIRP1_CONJ) {
        const float2 q = transfer(I.chirp1_rev, I.s_coef, I.series, fx, fy, OP == COL_CHIRP1_CONJ);
        v[e] = cscale(cmul(v[e], q), I.inv_m);
      } else if constexpr (OP == COL_CHIRP2 || OP == COL_CHIRP2_CONJ) {
        const float2 q = transfer(I.chirp2_rev, I.s_coef, I.series, fx, fy, OP == COL_CHIRP2_CONJ);
        v[e] = cscale(cmul(v[e], q), I.inv_m);
      } else if constexpr (OP == COL_BLUR) {
        v[e] = cscale(v[e], iotf_of(I, fx, fy) * I.inv_m);
      } else if constexpr (OP == COL_BLUR_LOSS) {
        const float h = iotf_of(I, fx, fy);
        const float2 yh = I.y_hat[(size_t)ky * nx + s];
        const float2 rr = make_float2(h * v[e].x - yh.x, h * v[e].y - yh.y);
        acc += (double)rr.x * (double)rr.x + (double)rr.y * (double)rr.y;
        v[e] = cscale(rr, h * I.inv_m);
      } else if constexpr (OP == COL_SPEC_YHAT) {
        I.y_hat[(size_t)ky * nx + s] = v[e];
      } else if constexpr (OP == COL_SPEC_PSIHAT) {
        I.psi_hat[(size_t)ky * nx + s] = v[e];
        if (I.z_hat) I.z_hat[(size_t)ky * nx + s] = make_float2(0.f, 0.f);
      }
    });
  }

  if constexpr (ColOpTraits<OP>::kInverse) {
    fft_inverse<Plan, T>(v, t, twr, lv);
    float2* __restrict__ dst = I.W + s;
    static_for<0, E / R1>([&](auto cc) {
      static_for<0, R1>([&](auto qq) {
        constexpr int c = decltype(cc)::value, q = decltype(qq)::value;
        dst[(size_t)(t + T * c + q * M1) * nx] = v[c * R1 + q];
      });
    });
  }

  if constexpr (OP == COL_BLUR_LOSS) {
    // deterministic block reduction: wave butterflies, then waves in order
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int i = 0; i < NT / 64; ++i) sum += red[i];
      I.loss_partial[tile] = sum;
    }
  }
}

// ------------------------------------------------------------------ plain path kernels

// Out-of-place FFT of every row (natural order in and out).
template <int NX, int DIR>
__global__ void __launch_bounds__(RowCfg<NX>::T * RowCfg<NX>::RW)
plain_fft_rows(const float2* __restrict__ src, float2* __restrict__ dst, const float2* tw) {
  using C = RowCfg<NX>;
  using Plan = typename C::Plan;
  constexpr int T = C::T, RW = C::RW, E = NX / T;
  constexpr int R1 = Plan::radix[0], RL = Plan::radix[Plan::NPASS - 1];
  constexpr int M1 = NX / R1, ML = NX / RL;
  __shared__ float2 lds[RW * lds_len(NX)];
  const int t = threadIdx.x % T, rw = threadIdx.x / T;
  const size_t rbase = (size_t)(blockIdx.x * RW + rw) * NX;
  const LdsView lv{lds + rw * lds_len(NX), 1};
  float2 v[E];
  if constexpr (DIR < 0) {
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      v[e] = src[rbase + t + T * (e / R1) + (e % R1) * M1];
    });
    fft_forward<Plan, T>(v, t, tw, lv);
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      dst[rbase + t + T * (e / RL) + (e % RL) * ML] = v[e];
    });
  } else {
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      v[e] = src[rbase + t + T * (e / RL) + (e % RL) * ML];
    });
    fft_inverse<Plan, T>(v, t, tw + Plan::tw_total(), lv);
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      dst[rbase + t + T * (e / R1) + (e % R1) * M1] = v[e];
    });
  }
}

// In-place FFT of every column (natural order).
template <int NY, int DIR>
__global__ void __launch_bounds__(ColCfg<NY>::T * ColCfg<NY>::W)
plain_fft_cols(float2* __restrict__ a, int nx, const float2* tw) {
  using C = ColCfg<NY>;
  using Plan = typename C::Plan;
  constexpr int T = C::T, W = C::W, E = NY / T;
  constexpr int R1 = Plan::radix[0], RL = Plan::radix[Plan::NPASS - 1];
  constexpr int M1 = NY / R1, ML = NY / RL;
  __shared__ float2 lds[W * lds_len(NY)];
  const int w = threadIdx.x % W, t = threadIdx.x / W;
  const int s = blockIdx.x * W + w;
  const LdsView lv{lds + w, W};
  float2 v[E];
  if constexpr (DIR < 0) {
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      v[e] = a[(size_t)(t + T * (e / R1) + (e % R1) * M1) * nx + s];
    });
    fft_forward<Plan, T>(v, t, tw, lv);
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      a[(size_t)(t + T * (e / RL) + (e % RL) * ML) * nx + s] = v[e];
    });
  } else {
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      v[e] = a[(size_t)(t + T * (e / RL) + (e % RL) * ML) * nx + s];
    });
    fft_inverse<Plan, T>(v, t, tw + Plan::tw_total(), lv);
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      a[(size_t)(t + T * (e / R1) + (e % R1) * M1) * nx + s] = v[e];
    });
  }
}

template <int N>
hipError_t launch_row_n(int op, int nblocks, const Sweep& S, hipStream_t st) {
  using C = RowCfg<N>;
  const dim3 grid(nblocks), block(C::T * C::RW);
  switch (op) {
#define PWF_CASE(o) case o: hipLaunchKernelGGL((row_sweep<N, o>), grid, block, 0, st, S); break;
    PWF_CASE(ROW_PSI_UPDATE) PWF_CASE(ROW_START) PWF_CASE(ROW_MUL_T) PWF_CASE(ROW_MUL_CONJ_T)
    PWF_CASE(ROW_INTENSITY) PWF_CASE(ROW_BACKBLUR) PWF_CASE(ROW_GRAD) PWF_CASE(ROW_FORWARD_OUT)
    PWF_CASE(ROW_REAL_FFT) PWF_CASE(ROW_CPLX_FFT) PWF_CASE(ROW_IFFT_OUT)
#undef PWF_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int N>
hipError_t launch_col_n(int op, int nblocks, const Sweep& S, hipStream_t st) {
  using C = ColCfg<N>;
  const dim3 grid(nblocks), block(C::T * C::W);
  switch (op) {
#define PWF_CASE(o) case o: hipLaunchKernelGGL((col_sweep<N, o>), grid, block, 0, st, S); break;
    PWF_CASE(COL_CHIRP1) PWF_CASE(COL_CHIRP2) PWF_CASE(COL_CHIRP2_CONJ) PWF_CASE(COL_CHIRP1_CONJ)
    PWF_CASE(COL_BLUR_LOSS) PWF_CASE(COL_BLUR) PWF_CASE(COL_NESTEROV) PWF_CASE(COL_DIRECTION)
    PWF_CASE(COL_SPEC_YHAT) PWF_CASE(COL_SPEC_PSIHAT)
#undef PWF_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int N>
hipError_t plain_rows_n(int dir, const float2* src, float2* dst, int ny, const float2* tw, hipStream_t st) {
  using C = RowCfg<N>;
  const dim3 grid(ny / C::RW), block(C::T * C::RW);
  if (dir < 0) hipLaunchKernelGGL((plain_fft_rows<N, -1>), grid, block, 0, st, src, dst, tw);
  else hipLaunchKernelGGL((plain_fft_rows<N, 1>), grid, block, 0, st, src, dst, tw);
  return hipGetLastError();
}

template <int N>
hipError_t plain_cols_n(int dir, float2* a, int nx, const float2* tw, hipStream_t st) {
  using C = ColCfg<N>;
  const dim3 grid(nx / C::W), block(C::T * C::W);
  if (dir < 0) hipLaunchKernelGGL((plain_fft_cols<N, -1>), grid, block, 0, st, a, nx, tw);
  else hipLaunchKernelGGL((plain_fft_cols<N, 1>), grid, block, 0, st, a, nx, tw);
  return hipGetLastError();
}

template <class PP>
static void fill_twiddles(float2* out) {
  for (int p = 1; p < PP::NPASS; ++p) {
    const int L = PP::stride_before(p), R = PP::radix[p];
    for (int q = 0; q < R; ++q)
      for (int k = 0; k < L; ++k) {
        const double ang = -2.0 * M_PI * (double)(q * k) / (double)(L * R);
        out[PP::tw_offset(p) + q * L + k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
      }
  }
}

// Twiddle tables of the N-point plan followed by those of its reversed plan.
template <int N>
int plan_twiddles_n(float2* out) {
  using Plan = typename RowCfg<N>::Plan;
  using RPlan = typename Reverse<Plan>::type;
  static_assert(Plan::valid(), "radices must multiply to N");
  static_assert(std::is_same<Plan, typename ColCfg<N>::Plan>::value, "row and column plans share tables");
  if (out) {
    fill_twiddles<Plan>(out);
    fill_twiddles<RPlan>(out + Plan::tw_total());
  }
  return Plan::tw_total() + RPlan::tw_total();
}

}  // namespace pwf
