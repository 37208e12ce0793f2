// Sweep kernel templates of the PWF hot path (instantiated once per grid side
// in pwf_sweeps_<N>.hip so that the sides compile in parallel).
//
// Fused path: every iteration of Algorithm S1 is twelve sweeps over each
// instance's fields.  A row sweep finishes the inverse 2-D FFT of the
// previous Filter along x, applies the real-space step of the algorithm and
// starts the next forward 2-D FFT along x; a column sweep does the y
// transforms with the Fourier-domain window in between.  Sweeps S0..S11:
//   S0 R  psi = IFFT(.); x = exp(psi) (saved); FFT      (Algorithm S1 loop head)
//   S1 C  x Q_L1                                          (FreePropagation L1)
//   S2 R  x t                                             (diffuser)
//   S3 C  x Q_L2                                          (FreePropagation L2)
//   S4 R  v saved; I = |v|^2                              (PhysicalModel)
//   S5 C  R = IOTF I^ - Y^ (= F{-e}); loss += |R|^2/m; x IOTF   (Eq. 2, Filter(-e, IOTF))
//   S6 R  h = Re(.); a = v h                              (WirtingerDerivative)
//   S7 C  x conj Q_L2                                     (FreePropagation -L2)
//   S8 R  x conj t
//   S9 C  x conj Q_L1                                     (FreePropagation -L1)
//   S10 R g = x* b / max|t|^2
//   S11 C direction d (Preconditioner + Regularizer) and the Nesterov step on
//         the spectra of z_k, z_{k-1}; IFFT of psi_{k+1} towards the next S0.
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
PWF_ROW_TRAIT(ROW_PSI_UPDATE_CORR, true, true)
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

// exp(p) for complex p.  The phase is reduced to a quadrant index n and a
// remainder f in [-pi/4, pi/4] in units of revolutions (r = p.y / 2 pi; r - n/4
// is exact), and cos f, sin f come from their Taylor series, truncated where
// the next term is below 2e-9 on that interval.  The only error beyond the
// polynomials' rounding is that of r itself, |p.y| 2^-24 rad, the same as
// one rounding of p.y.
__device__ __forceinline__ float2 cexp_f(float2 p) {
  const float r = p.y * 0.159154943091895336f;
  const float n = rintf(4.f * r);
  const float f = fmaf(-0.25f, n, r) * 6.28318530717958648f;
  const float f2 = f * f;
  // sin f = f (1 - f^2/3! + f^4/5! - f^6/7! + f^8/9!)
  float sp = fmaf(f2, 2.75573192e-6f, -1.98412698e-4f);
  sp = fmaf(f2, sp, 8.33333333e-3f);
  sp = fmaf(f2, sp, -1.66666667e-1f);
  const float sn = fmaf(f * f2, sp, f);
  // cos f = 1 - f^2/2! + f^4/4! - f^6/6! + f^8/8! - f^10/10!
  float cp = fmaf(f2, -2.75573192e-7f, 2.48015873e-5f);
  cp = fmaf(f2, cp, -1.38888889e-3f);
  cp = fmaf(f2, cp, 4.16666667e-2f);
  cp = fmaf(f2, cp, -0.5f);
  const float cs = fmaf(f2, cp, 1.f);
  // rotate by n quarter turns: n = 1 -> (-sin, cos), 2 -> (-cos, -sin), 3 -> (sin, -cos)
  const int q = (int)n;
  const bool swap = q & 1;
  const float c1 = swap ? sn : cs, s1 = swap ? cs : sn;
  const uint32_t flip_c = (uint32_t)((q + 1) & 2) << 30, flip_s = (uint32_t)(q & 2) << 30;
  const float a = expf(p.x);
  return make_float2(a * __uint_as_float(__float_as_uint(c1) ^ flip_c),
                     a * __uint_as_float(__float_as_uint(s1) ^ flip_s));
}

// Butterflies of the column transform's radix-2 split (col_split) in the row
// sweeps.  The two rows n and n + H of a pair sit PD lanes apart in one wave
// (pb = 1 for row n + H) and hold the same x positions.  w = w_ny^n.
//   reading W after a column sweep: row n holds A[n], row n + H holds B[n];
//     x[n] = A + w^-n B, x[n + H] = A - w^-n B;
//   writing W for a column sweep: rows n, n + H hold X[n], X[n + H];
//     a[n] = X[n] + X[n + H] (row n), b[n] = (X[n] - X[n + H]) w^n (row n + H).
// At PD = 32 two elements go at once: v_permlane32_swap of the registers of
// elements e1, e2 leaves the lower half-wave with both rows' values of e1 and
// the upper half with those of e2; each lane computes both outputs of its
// element and a second swap returns them to their rows.  Rows on fewer than
// 32 lanes (sides 128 and 256) exchange each value with a lane shuffle.
__device__ __forceinline__ void lane_swap32(float& p, float& q) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(p), __float_as_uint(q), false, false);
  p = __uint_as_float(r[0]);
  q = __uint_as_float(r[1]);
}
template <bool FWD>
__device__ __forceinline__ void split_butterfly(float2& a, float2& b, float2 w) {
  if constexpr (FWD) {
    const float2 d = make_float2(a.x - b.x, a.y - b.y);
    a = make_float2(a.x + b.x, a.y + b.y);
    b = cmul(d, w);
  } else {
    const float2 wb = cmulc(b, w);
    b = make_float2(a.x - wb.x, a.y - wb.y);
    a = make_float2(a.x + wb.x, a.y + wb.y);
  }
}
// elements p, q of this lane (PD = 32): both replaced by this row's outputs
template <bool FWD>
__device__ __forceinline__ void split_two(float2& p, float2& q, float2 w) {
  lane_swap32(p.x, q.x);
  lane_swap32(p.y, q.y);
  split_butterfly<FWD>(p, q, w);   // (row n, row n + H) values of one element
  lane_swap32(p.x, q.x);
  lane_swap32(p.y, q.y);
}
// one element of this lane (any PD): replaced by this row's output
template <bool FWD, int PD>
__device__ __forceinline__ void split_one(float2& v, float2 w, int pb) {
  const float2 o = make_float2(__shfl_xor(v.x, PD, 64), __shfl_xor(v.y, PD, 64));
  float2 a = pb ? o : v, b = pb ? v : o;
  split_butterfly<FWD>(a, b, w);
  v = pb ? b : a;
}
// The elements v[IDX(i)], i < COUNT, of this lane.
template <bool FWD, int PD, int COUNT, class F, int E>
__device__ __forceinline__ void split_elements(float2 (&v)[E], float2 w, int pb, F idx) {
  if constexpr (PD == 32 && COUNT % 2 == 0) {
    static_for<0, COUNT / 2>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      split_two<FWD>(v[idx(std::integral_constant<int, 2 * i>{})], v[idx(std::integral_constant<int, 2 * i + 1>{})], w);
    });
  } else {
    static_for<0, COUNT>([&](auto ii) { split_one<FWD, PD>(v[idx(ii)], w, pb); });
  }
}

// A copy of v that the compiler cannot see through.  Stores at the end of a
// sweep take their offsets from such a copy: otherwise the compiler reuses the
// 64-bit addresses of the matching loads and keeps one register pair per
// element alive across the whole FFT.
__device__ __forceinline__ uint32_t opaque(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Twiddles staged in LDS.  Every load of the table is issued ahead of the
// sweep's own loads and held in registers, and the LDS writes come after those
// loads are issued: the table's latency then hides under the data's instead of
// costing one dependent round trip per strided chunk of the table.
template <int COUNT, int NTHR>
struct TwStage {
  static constexpr int K = (COUNT + NTHR - 1) / NTHR;
  float2 r[K];
  __device__ __forceinline__ void load(const float2* src) {
    static_for<0, K>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      const int i = (int)threadIdx.x + j * NTHR;
      if (COUNT % NTHR == 0 || i < COUNT) r[j] = gld(src, (uint32_t)i);
    });
  }
  __device__ __forceinline__ void store(float2* lds) const {
    static_for<0, K>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      const int i = (int)threadIdx.x + j * NTHR;
      if (COUNT % NTHR == 0 || i < COUNT) lds[i] = r[j];
    });
  }
};

// Logical block of hardware block b in a grid of g blocks.  Workgroups are
// dispatched round-robin over the 8 XCDs: XCD x = b % 8 gets the contiguous
// range [x g/8, (x + 1) g/8), walked forwards, or backwards with REV, from a
// start rotated by x eighths of the range.  Row sweeps walk forwards and
// column sweeps backwards, so that each sweep starts on the data its
// predecessor wrote last, which the memory-side cache may still hold.  The
// rotation keeps the XCDs out of step: when each range holds whole instances
// (8 x 2048^2: one each), unrotated XCDs visit the same offsets of instances a
// power of two apart at the same time, and the column sweeps there ran 12-26%
// slower (row sweeps up to 7%; 0.3-1% at 180 x 1024^2).  (Plain reversal when
// 8 does not divide g.)
template <bool REV>
__device__ __forceinline__ int xcd_contiguous(int b, int g) {
  if (g & 7) return REV ? g - 1 - b : b;
  const int per = g >> 3, j = b >> 3, x = b & 7;
  int k = (REV ? per - 1 - j : j) + x * (per >> 3);
  if (k >= per) k -= per;
  return x * per + k;
}

// Waves per SIMD the compiler must leave room for (launch bound).
template <int NX, int OP> constexpr int row_min_waves() {
  return (OP == ROW_PSI_UPDATE || OP == ROW_PSI_UPDATE_CORR) ? 3 : OP == ROW_GRAD ? (NX >= 2048 ? 2 : 3) : 4;
}

template <int NX, int PLAN>
using RowCfgSel = typename std::conditional<PLAN == 2, RowCfgAlt2<NX>,
                                            typename std::conditional<PLAN == 1, RowCfgAlt<NX>, RowCfg<NX>>::type>::type;

template <int NX, int PLAN> constexpr int row_threads() { return RowCfgSel<NX, PLAN>::T * RowCfgSel<NX, PLAN>::RW; }

// LDS a row sweep needs: the exchange buffer and the staged twiddles, a
// fraction 1/row_tw_div of w_N^m (TwTable).  The update sweep stages half of
// it up to 1024: the 4 KB saved let a fourth workgroup of the 16x16x4 plan fit
// in a CU's LDS (its registers allow it; the other sweeps at 1024 gained
// nothing from a quarter table).  At 2048, beside the two rows' 33 KB exchange
// buffer, the half table (8 KB) leaves room for three workgroups per CU and
// the quarter table (4 KB) for four; the quarter's rotations cost registers,
// and the x t, intensity and gradient sweeps run as fast or faster with the
// half table (x t spills with the quarter).  Reading the per-pass tables from
// global memory instead cost the 2048 row sweeps 20% (23.1 against 18.7 ms
// per iteration of 180 projections).
template <int NX, int OP> constexpr int row_tw_div() {
  if constexpr (NX > 1024) return (OP == ROW_MUL_T || OP == ROW_INTENSITY || OP == ROW_GRAD) ? 2 : 4;
  else return (OP == ROW_PSI_UPDATE || OP == ROW_PSI_UPDATE_CORR) ? 2 : 1;
}
template <int NX, int OP, int PLAN>
struct RowLds {
  using C = RowCfgSel<NX, PLAN>;
  using TS = TwSel<typename C::Plan, row_tw_div<NX, OP>(), true>;
  static constexpr int kExchange = C::RW * lds_len(NX);
  static constexpr int kTwiddles = TS::kLds;
};

// Row sweep `OP` on logical block b (instance b / blocks_per_inst) with the
// caller's LDS (RowLds sizes).
template <int NX, int OP, int PLAN, bool PAIR>
__device__ __forceinline__ void row_body(const Sweep& S, int b, float2* lds, float2* twl) {
  using C = RowCfgSel<NX, PLAN>;
  using Plan = typename C::Plan;
  constexpr int T = C::T, RW = C::RW, E = NX / T;
  constexpr int R1 = Plan::radix[0], RL = Plan::radix[Plan::NPASS - 1];
  constexpr int M1 = NX / R1, ML = NX / RL;
  constexpr bool IN_FREQ = RowOpTraits<OP>::kInFreq, OUT_FREQ = RowOpTraits<OP>::kOutFreq;

  const int inst = b / S.blocks_per_inst;
  const int blk = b - inst * S.blocks_per_inst;
  const Inst I = S.inst[inst];  // by value: the fields stay in registers
  if (instance_stopped(I)) return;  // uniform over the workgroup
  // Rows of the workgroup: RW consecutive rows, or, with the column transform
  // split (PAIR, pair_half = H = ny/2), RW/2 pairs (n, n + H) whose two rows
  // sit PD lanes apart in one wave (lane t of row n + H is PD lanes after lane
  // t of row n) for the split's butterflies.  The workspace fields that only
  // the row sweeps and the split halves address (W, x, v) store the two rows
  // of a pair close together (split_row), so that a workgroup reads and
  // writes one region instead of two ny/2 rows apart (that cost the 2048 row
  // sweeps 7%); `mrow` is the stored row, `row` the row of the caller's
  // fields (t, y, psi, outputs) and of u1.
  static_assert(RW % 2 == 0, "row pairs");
  constexpr int PD = T < 32 ? T : 32;
  int t, rw, row, mrow, pb = 0, prow = 0;
  if constexpr (PAIR) {
    const int H = S.pair_half;
    const int u = (int)threadIdx.x % (2 * T);
    pb = (u / PD) & 1;
    t = (u / (2 * PD)) * PD + u % PD;
    rw = 2 * ((int)threadIdx.x / (2 * T)) + pb;
    prow = blk * (RW / 2) + (int)threadIdx.x / (2 * T);
    row = prow + pb * H;
    mrow = split_row(prow, pb);
  } else {
    t = (int)threadIdx.x % T;
    rw = (int)threadIdx.x / T;
    row = blk * RW + rw;
    mrow = row;
  }
  const float2 wp = PAIR ? gld(S.twn_pair, (uint32_t)prow) : make_float2(1.f, 0.f);
  const LdsView lv{lds + rw * lds_len(NX), 1};
  using TS = typename RowLds<NX, OP, PLAN>::TS;
  const float2* twg = PLAN == 2 ? S.tw_alt2 : PLAN == 1 ? S.tw_alt : S.tw_row;
  const auto tw = TS::forward(twl, twg);
  const auto twr = TS::inverse(twl, twg);
  const uint32_t rbase = (uint32_t)row * NX;   // caller fields, u1
  const uint32_t wbase = (uint32_t)mrow * NX;  // W, x, v
  // Twiddles to LDS; the first pass needs none, and the barrier after its
  // LDS exchange orders these writes before the first use.
  TwStage<TS::kLds, row_threads<NX, PLAN>()> tws;
  if constexpr (TS::kMode != 0) tws.load(TS::staged_from(twg, S.twn_row));
  // The transforms of a row (or of a pair of rows) whose lanes lie in one wave
  // order their LDS exchanges per wave; the staged twiddles, which every wave
  // reads, then need a workgroup barrier of their own.
  constexpr bool WAVE = PAIR ? 2 * T <= 64 : T <= 64;
  auto load_twiddles = [&]() {
    if constexpr (TS::kMode != 0) {
      tws.store(twl);
      if constexpr (WAVE) __syncthreads();
    }
  };

  // Side input of the real-space step (t, v or x at this row), loaded after
  // the row spectrum so that its latency overlaps the inverse FFT.  The
  // gradient sweep at 32 elements per lane loads it at its use instead: held
  // through the FFT it would not fit the register file.
  constexpr bool SIDE = OP == ROW_MUL_T || OP == ROW_MUL_CONJ_T || OP == ROW_BACKBLUR ||
                        (OP == ROW_GRAD && E <= 16);
  float2 side[SIDE ? E : 1];
  float2 v[E];
  if constexpr (IN_FREQ) {
    if constexpr (OP == ROW_BACKBLUR || OP == ROW_FORWARD_OUT) {
      // half-form x-spectrum (see col_op_half): kx > nx/2 from conj at nx - kx,
      // kx = 0 and nx/2 from the packed position 0 (after the residual sweep's
      // second IOTF, kx = nx/2 still lacks its second x factor)
      const uint32_t rh = wbase;
      const float s_ny = OP == ROW_BACKBLUR ? gldf(I.ix, NX / 2) : 1.f;
      static_for<0, E / RL>([&](auto cc) {
        static_for<0, RL>([&](auto rr) {
          constexpr int c = decltype(cc)::value, r = decltype(rr)::value;
          const int kx = t + T * c + r * ML;
          const int kk = kx <= NX / 2 ? kx : NX - kx;
          v[c * RL + r] = gld(I.W, rh + (uint32_t)(kk == NX / 2 ? 0 : kk));
        });
      });
      // the split's butterflies act on the stored values (the packed column
      // included), before they are unpacked
      if constexpr (PAIR) split_elements<false, PD, E>(v, wp, pb, [](auto i) { return decltype(i)::value; });
      static_for<0, E / RL>([&](auto cc) {
        static_for<0, RL>([&](auto rr) {
          constexpr int c = decltype(cc)::value, r = decltype(rr)::value;
          const int kx = t + T * c + r * ML;
          float2 a = v[c * RL + r];
          if (kx > NX / 2) a.y = -a.y;
          else if (kx == 0) a.y = 0.f;
          else if (kx == NX / 2) a = make_float2(s_ny * a.y, 0.f);
          v[c * RL + r] = a;
        });
      });
    } else {
      static_for<0, E / RL>([&](auto cc) {
        static_for<0, RL>([&](auto rr) {
          constexpr int c = decltype(cc)::value, r = decltype(rr)::value;
          v[c * RL + r] = gld(I.W, wbase + col_of_kx(t + T * c + r * ML, NX));
        });
      });
    }
    load_twiddles();
    if constexpr (SIDE) {
      constexpr bool T_SIDE = OP == ROW_MUL_T || OP == ROW_MUL_CONJ_T;
      const float2* __restrict__ sp = T_SIDE ? I.t : (OP == ROW_BACKBLUR ? I.v : I.x);
      const uint32_t sb = T_SIDE ? rbase : wbase;
      static_for<0, E / R1>([&](auto cc) {
        static_for<0, R1>([&](auto qq) {
          constexpr int c = decltype(cc)::value, q = decltype(qq)::value;
          side[c * R1 + q] = gld(sp, sb + t + T * c + q * M1);
        });
      });
    }
    if constexpr (!(OP == ROW_BACKBLUR || OP == ROW_FORWARD_OUT)) {
      // (issued after the side loads, whose latency then overlaps the wait)
      if constexpr (PAIR) split_elements<false, PD, E>(v, wp, pb, [](auto i) { return decltype(i)::value; });
    }
    fft_inverse<Plan, T, WAVE>(v, t, twr, lv);
  } else if constexpr (OP == ROW_REAL_FFT) {
    static_for<0, E / R1>([&](auto cc) {
      static_for<0, R1>([&](auto qq) {
        constexpr int c = decltype(cc)::value, q = decltype(qq)::value;
        v[c * R1 + q] = make_float2(gldf(I.y, rbase + t + T * c + q * M1), 0.f);
      });
    });
    load_twiddles();
  } else {  // ROW_START / ROW_CPLX_FFT: complex real-space input (null = zeros)
    const float2* __restrict__ src = I.psi_src;
    static_for<0, E / R1>([&](auto cc) {
      static_for<0, R1>([&](auto qq) {
        constexpr int c = decltype(cc)::value, q = decltype(qq)::value;
        v[c * R1 + q] = src ? gld(src, rbase + t + T * c + q * M1) : make_float2(0.f, 0.f);
      });
    });
    load_twiddles();
  }

  // real-space step; element e = c*R1 + q sits at x = t + T c + q M1
  float inv_maxt2 = 0.f;
  float u1max = 0.f;  // joint diffuser mode (S2): max |u1|^2 over this lane's elements
  if constexpr (OP == ROW_GRAD) inv_maxt2 = I.grad_mul > 0.f ? I.grad_mul : 1.0f / *I.maxt2;
  // stopping correlation of exp(psi) with the previous iterate (FP64 sums):
  // only the S0 variant for the stopping rule (solves with a threshold attach
  // the partials and launch that variant)
  constexpr bool PSI = OP == ROW_PSI_UPDATE || OP == ROW_PSI_UPDATE_CORR;
  const bool corr = OP == ROW_PSI_UPDATE_CORR && I.corr_partial != nullptr;
  const bool corr_sum = corr && S.iter > 0;
  double c_re = 0.0, c_im = 0.0, n_new = 0.0, n_old = 0.0;
  const uint32_t rb_rs = opaque(rbase);
  const uint32_t wb_rs = PAIR ? opaque(wbase) : rb_rs;
  if constexpr (OP == ROW_MUL_CONJ_T) {
    if (I.u1) {
      // Joint diffuser mode: u1 <- conj(u1) a2 with a2 = this back-propagated
      // field (dL/dt*).  In batches of four elements, each batch's u1 loads
      // issued before the previous batch's stores: behind the stores the
      // compiler would load one element per memory round trip.
      constexpr int NB = 4;
      static_assert(E % NB == 0, "joint batches");
      float2 ub[2][NB];
      auto load_u1 = [&](auto bb) {
        constexpr int b = decltype(bb)::value;
        static_for<0, NB>([&](auto uu) {
          constexpr int u = decltype(uu)::value, e = b * NB + u;
          ub[b & 1][u] = gld(I.u1, rb_rs + t + T * (e / R1) + (e % R1) * M1);
        });
      };
      load_u1(std::integral_constant<int, 0>{});
      static_for<0, E / NB>([&](auto bb) {
        constexpr int b = decltype(bb)::value;
        if constexpr (b + 1 < E / NB) load_u1(std::integral_constant<int, b + 1>{});
        static_for<0, NB>([&](auto uu) {
          constexpr int u = decltype(uu)::value, e = b * NB + u;
          gst(I.u1, rb_rs + t + T * (e / R1) + (e % R1) * M1, cmulc(v[e], ub[b & 1][u]));
        });
      });
    }
  }
  // With the stopping rule the previous x is read where the new one is
  // stored: the S0 variant for it loads it four elements at a time, the next
  // batch before this batch's stores (behind them the compiler would load one
  // element per memory round trip).  The fixed-iteration S0 keeps the
  // registers this costs.
  constexpr bool XB = OP == ROW_PSI_UPDATE_CORR;
  constexpr int NBX = 4;
  static_assert(!XB || E % NBX == 0, "stopping-rule batches");
  float2 xb[XB ? 2 : 1][NBX];
  auto load_x = [&](auto bb) {
    constexpr int b = decltype(bb)::value;
    static_for<0, NBX>([&](auto uu) {
      constexpr int u = decltype(uu)::value, e = b * NBX + u;
      xb[XB ? b & 1 : 0][u] = gld(I.x, wb_rs + t + T * (e / R1) + (e % R1) * M1);
    });
  };
  if constexpr (XB) {
    if (corr_sum) load_x(std::integral_constant<int, 0>{});
  }
  static_for<0, E / R1>([&](auto cc) {
    static_for<0, R1>([&](auto qq) {
      constexpr int c = decltype(cc)::value, q = decltype(qq)::value;
      constexpr int e = c * R1 + q;
      const uint32_t idx = rb_rs + t + T * c + q * M1;   // caller fields, u1
      const uint32_t midx = PAIR ? wb_rs + t + T * c + q * M1 : idx;  // x, v
      if constexpr (PSI) {
        if constexpr (XB) {
          if (corr_sum && e % NBX == 0 && e / NBX + 1 < E / NBX) load_x(std::integral_constant<int, e / NBX + 1>{});
        }
        if (corr) gst(I.out, idx, v[e]);  // psi of this iterate, kept in case the stop fires
        const float2 xn = cexp_f(v[e]);
        if (corr_sum) {
          const float2 xo = XB ? xb[XB ? (e / NBX) & 1 : 0][e % NBX] : gld(I.x, midx);
          c_re += (double)xn.x * xo.x + (double)xn.y * xo.y;
          c_im += (double)xn.x * xo.y - (double)xn.y * xo.x;
          n_new += (double)xn.x * xn.x + (double)xn.y * xn.y;
          n_old += (double)xo.x * xo.x + (double)xo.y * xo.y;
        }
        v[e] = xn;
        if (I.x) gst(I.x, midx, v[e]);
      } else if constexpr (OP == ROW_START) {
        v[e] = cexp_f(v[e]);
        if (I.x) gst(I.x, midx, v[e]);
      } else if constexpr (OP == ROW_MUL_T) {
        if (I.u1) {  // joint diffuser mode: keep u1 for the diffuser gradient of S8
          gst(I.u1, idx, v[e]);
          u1max = fmaxf(u1max, v[e].x * v[e].x + v[e].y * v[e].y);
        }
        v[e] = cmul(v[e], side[e]);
      } else if constexpr (OP == ROW_MUL_CONJ_T) {
        v[e] = cmulc(v[e], side[e]);
      } else if constexpr (OP == ROW_INTENSITY) {
        if (I.v) gst(I.v, midx, v[e]);
        v[e] = make_float2(v[e].x * v[e].x + v[e].y * v[e].y, 0.f);
      } else if constexpr (OP == ROW_BACKBLUR) {
        const float h = v[e].x;
        v[e] = make_float2(side[e].x * h, side[e].y * h);
      } else if constexpr (OP == ROW_GRAD) {
        const float2 xs = SIDE ? side[SIDE ? e : 0] : gld(I.x, midx);
        v[e] = cscale(cmulc(v[e], xs), inv_maxt2);
        if (I.g_out) gst(I.g_out, idx, v[e]);
        v[e].x *= kGradReScale;  // the direction sweeps undo this (see kGradReScale)
      } else if constexpr (OP == ROW_FORWARD_OUT) {
        const float f = v[e].x;   // RMSE image (Methods): |y - f| scaled by 100 / <reference>
        gstf(I.f_out, idx, I.rmse_scale > 0.f ? fabsf(gldf(I.y, idx) - f) * I.rmse_scale : f);
      } else if constexpr (OP == ROW_CPLX_FFT) {
        if (I.psi) gst(I.psi, idx, v[e]);
      } else if constexpr (OP == ROW_IFFT_OUT) {
        if (I.out) gst(I.out, idx, v[e]);
      }
    });
  });

  if constexpr (OUT_FREQ) {
    fft_forward<Plan, T, WAVE>(v, t, tw, lv);
    if constexpr (OP == ROW_INTENSITY || OP == ROW_REAL_FFT) {
      // spectrum of a real row in half form (see col_op_half); lane 0 holds
      // kx = 0 in v[0] and kx = nx/2 in v[RL/2].  Element (c, r) has kx < nx/2
      // exactly when r < RL/2 (t + T c < nx/RL), so only those are stored.
      static_assert(RL % 2 == 0, "half form");
      const uint32_t rh = opaque(wbase);
      const float s_ny = OP == ROW_INTENSITY ? gldf(I.ix, NX / 2) : 1.f;
      float2 packed = make_float2(v[0].x, s_ny * v[RL / 2].x);
      if constexpr (PAIR) {
        split_one<true, PD>(packed, wp, pb);
        // the stored elements (c, r < RL/2), i -> c = i / (RL/2), r = i % (RL/2)
        split_elements<true, PD, E / 2>(v, wp, pb, [](auto i) {
          constexpr int k = decltype(i)::value;
          return (k / (RL / 2)) * RL + k % (RL / 2);
        });
      }
      static_for<0, E / RL>([&](auto cc) {
        static_for<0, RL / 2>([&](auto rr) {
          constexpr int c = decltype(cc)::value, r = decltype(rr)::value;
          const int kx = t + T * c + r * ML;
          if (kx > 0) gst(I.W, rh + (uint32_t)kx, v[c * RL + r]);
        });
      });
      if (t == 0) gst(I.W, rh, packed);
    } else {
      if constexpr (PAIR) split_elements<true, PD, E>(v, wp, pb, [](auto i) { return decltype(i)::value; });
      const uint32_t rb_st = opaque(wbase);
      static_for<0, E / RL>([&](auto cc) {
        static_for<0, RL>([&](auto rr) {
          constexpr int c = decltype(cc)::value, r = decltype(rr)::value;
          gst(I.W, rb_st + col_of_kx(t + T * c + r * ML, NX), v[c * RL + r]);
        });
      });
    }
  }

  if constexpr (OP == ROW_MUL_T) {
    if (I.u1) {  // block max of |u1|^2 -> u1max[blk] (order-free, so deterministic)
      __shared__ float mred[RW * T / 64 + 1];
      for (int off = 32; off > 0; off >>= 1) u1max = fmaxf(u1max, __shfl_xor(u1max, off, 64));
      if ((threadIdx.x & 63) == 0) mred[threadIdx.x >> 6] = u1max;
      __syncthreads();
      if (threadIdx.x == 0) {
        float m = mred[0];
        for (int i = 1; i < RW * T / 64; ++i) m = fmaxf(m, mred[i]);
        gstf(I.u1max, blk, m);
      }
    }
  }

  if constexpr (PSI) {
    if (corr_sum) {
      // deterministic block reduction of the four sums -> corr_partial[blk]
      __shared__ double cred[4][RW * T / 64 + 1];
      double vals[4] = {c_re, c_im, n_new, n_old};
      for (int j = 0; j < 4; ++j) {
        double a = vals[j];
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
        if ((threadIdx.x & 63) == 0) cred[j][threadIdx.x >> 6] = a;
      }
      __syncthreads();
      if (threadIdx.x < 4) {
        double a = 0.0;
        for (int i = 0; i < RW * T / 64; ++i) a += cred[threadIdx.x][i];
        I.corr_partial[4 * blk + threadIdx.x] = a;
      }
    }
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

template <int NX, int OP, int PLAN, bool PAIR>
__global__ void __launch_bounds__((row_threads<NX, PLAN>()), (row_min_waves<NX, OP>())) row_sweep(Sweep S) {
  __shared__ float2 lds[RowLds<NX, OP, PLAN>::kExchange];
  __shared__ float2 twl[RowLds<NX, OP, PLAN>::kTwiddles];
  row_body<NX, OP, PLAN, PAIR>(S, xcd_contiguous<false>(blockIdx.x, gridDim.x), lds, twl);
}

// ------------------------------------------------------------------ column sweeps

// Column tile of the j-th workgroup of an instance with B tiles of W columns.
// The G = 128 / (8 W) tiles that share a 128-byte line stay adjacent in time;
// the groups are dealt out over the four quarters of the row (group m ->
// (m mod 4) B/(4G) + m/4), so that the workgroups in flight touch more HBM
// channels (about 1% on the column sweeps at 1024^2).  Identity when 4 does
// not divide B/G.
template <int W>
__device__ __forceinline__ int col_tile_of(int j, int B) {
  constexpr int G = W >= 16 ? 1 : 16 / W;
  const int ng = B / G, m = j / G;
  if (ng & 3) return j;
  return (((m & 3) * (ng >> 2)) + (m >> 2)) * G + j % G;
}

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

// Transfer function of FreePropagation at (fx, fy) from the 1-D factors:
// Q = Qx(fx) Qy(fy) exp(i theta_c), where the cross term theta_c = -2 pi a rho^2
// (2/(1+sqrt(1-s)) - 1) is applied as (1, theta_c).  For hard X-ray geometries
// it stays below a quarter ulp of 1 everywhere and the sweep skips it.
__device__ __forceinline__ float2 transfer_sep(float2 qx, float2 qy, float fx, float fy, float s_coef,
                                               float two_pi_a) {
  const float2 q = cmul(qx, qy);
  const float rho2 = fx * fx + fy * fy;
  const float s = s_coef * rho2;
  const float thc = -two_pi_a * rho2 * s * (0.25f + 0.125f * s);
  return make_float2(q.x - thc * q.y, q.y + thc * q.x);
}

// Geometries outside the series range use the FP64 formula per element.
__device__ __noinline__ float2 transfer_direct(double chirp_rev, double s_coef, float fx, float fy) {
  return transfer(chirp_rev, s_coef, 0, fx, fy, false);
}

// Waves per SIMD the column sweeps must leave room for: 4 (128 registers)
// for the Nesterov sweep where the LDS lets four waves per SIMD in (two
// 512-thread or four 256-thread workgroups per CU), else 3 for the update
// sweeps (168 registers; at 256 points the 16-column tile would spill), 2 for
// the others, which need fewer registers than that anyway (a 4-wave bound,
// 128 registers, makes the chirp sweeps spill).
template <int NY, int W, int OP> constexpr int col_min_waves() {
  constexpr int NF = col_fft_len<NY>();
  return OP == COL_NESTEROV && (NF == 512 || (NF > 512 && ColCfg<NF>::T * W == 512)) ? 4
         : (OP == COL_NESTEROV || OP == COL_DIRECTION) && !(NF == 256 && W == 16) ? 3 : 2;
}

// LDS a column sweep needs: the exchange buffer and the staged twiddles of
// its transform (NY points, or NY/2 when split).
template <int NY, int W>
struct ColLds {
  static constexpr int NF = col_fft_len<NY>();
  using TS = TwSel<typename ColCfg<NF>::Plan, 1, true>;
  static constexpr int kExchange = W * lds_len(NF);
  static constexpr int kTwiddles = TS::kLds;
  static constexpr int kYTable = NF / 2 + 1;  // chirp sweeps: staged y factors
};
constexpr bool col_op_chirp(int op) {
  return op == COL_CHIRP1 || op == COL_CHIRP1_CONJ || op == COL_CHIRP2 || op == COL_CHIRP2_CONJ;
}
// Sweeps that stage their per-ky factor in LDS (ColLds::kYTable entries):
// the chirp factor, the regulariser window 1 - STF_y (S11), the IOTF (S5).
constexpr bool col_op_ystage(int op) { return col_op_chirp(op) || op == COL_NESTEROV || op == COL_BLUR_LOSS; }

// Column sweep `OP` on logical block b (instance b / blocks_per_inst) with the
// caller's LDS (ColLds sizes).
// With the transform split (col_split), logical blocks [0, B/2) of an
// instance run the even-ky half (rows 0 .. NY/2 - 1) and [B/2, B) the odd
// half, over the same tiles; elements are addressed by their position j in
// the half-column (row part NY/2 + j) and the frequency is ky = 2 j + part.
template <int NY, int W, int OP>
__device__ __forceinline__ void col_body(const Sweep& S, int b, float2* lds, float2* twl, float2* qyl) {
  constexpr bool SPLIT = col_split<NY>();
  constexpr int NF = col_fft_len<NY>();
  using C = ColCfg<NF>;
  using Plan = typename C::Plan;
  constexpr int T = C::T, E = NF / T;
  constexpr int R1 = Plan::radix[0], RL = Plan::radix[Plan::NPASS - 1];
  constexpr int M1 = NF / R1, ML = NF / RL;
  constexpr int NT = T * W;
  __shared__ double red[(NT + 63) / 64];

  const int inst = b / S.blocks_per_inst;
  const int jb = b - inst * S.blocks_per_inst;
  const int ntile = SPLIT ? S.blocks_per_inst / 2 : S.blocks_per_inst;
  const int part = SPLIT && jb >= ntile ? 1 : 0;
  const int tile = col_tile_of<W>(jb - part * ntile, ntile);
  const Inst I = S.inst[inst];  // by value: the fields stay in registers
  if (instance_stopped(I)) return;  // uniform over the workgroup
  // frequency of position j, and the position of -ky within the half
  auto ky_of = [&](int j) { return SPLIT ? 2 * j + part : j; };
  auto mirror_pos = [&](int j) { return SPLIT && part ? NF - 1 - j : (NF - j) & (NF - 1); };
  // x-spectra in half form (col_op_half) use columns 0 .. nx/2 - 1 only
  constexpr bool HALF = col_op_half(OP);
  const int nx = I.nx;
  if constexpr (OP == COL_CHIRP1) {
    // Stopping rule (Methods, "Reconstruction procedure"): |<x_k, x_k-1>| /
    // (|x_k| |x_k-1|) above the threshold, from the FP64 partials of S0.
    if (I.corr_partial && S.iter > 0 && tile == 0 && part == 0 && threadIdx.x == 0) {
      double a[4] = {0.0, 0.0, 0.0, 0.0};
      for (int i = 0; i < I.n_corr_partials; ++i)
        for (int j = 0; j < 4; ++j) a[j] += I.corr_partial[4 * i + j];
      const double c = sqrt(a[0] * a[0] + a[1] * a[1]) / sqrt(a[2] * a[3]);
      if (c > S.corr_tol) *I.stop_iter = S.iter;
    }
  }
  const int w = threadIdx.x % W, t = threadIdx.x / W;
  const int s = tile * W + w;
  // spectra: row part NF + j; W (split): stored row split_row(j, part), which
  // for the positions t + T c + q M1 of a lane (T, M1 multiples of the block)
  // is split_row(t, part) + 2 (T c + q M1)
  const uint32_t o_ld = (uint32_t)((part * NF + t) * nx + s);  // element (t, s) of the half; position j adds (j - t) nx
  constexpr int WS = SPLIT ? 2 : 1;  // W row stride of consecutive positions
  static_assert(!SPLIT || (T % kSplitBlock == 0 && M1 % kSplitBlock == 0), "split row blocks");
  const uint32_t o_w = SPLIT ? (uint32_t)(split_row(t, part) * nx + s) : o_ld;
  const LdsView lv{lds + w, W};
  using TS = typename ColLds<NY, W>::TS;
  const auto tw = TS::forward(twl, S.tw_col);
  const auto twr = TS::inverse(twl, S.tw_col);

  TwStage<TS::kLds, NT> tws;
  if constexpr (TS::kMode != 0) tws.load(TS::staged_from(S.tw_col, S.twn_col));
  // The per-ky factor of the Fourier-domain step (chirp y factor; 1 - STF_y
  // in S11; IOTF_y in S5) staged in LDS like the twiddles, instead of one
  // global load per element (the 16-column chirp sweeps at 1024: 0.636 ->
  // 0.591 ms).  The factors depend on fy^2, so positions j and mirror_pos(j)
  // (ky and -ky) share them: the table (the caller's LDS, ColLds::kYTable
  // entries; float factors in .x) holds positions 0 .. NF/2 (4 KB at 1024
  // points, which still lets two workgroups share a CU).
  constexpr bool YSTAGE = col_op_ystage(OP);
  constexpr int NQ = YSTAGE ? ColLds<NY, W>::kYTable : 1;
  constexpr int KQ = (NQ + NT - 1) / NT;
  float2 qys[YSTAGE ? KQ : 1];
  if constexpr (YSTAGE) {
    static_for<0, KQ>([&](auto jj) {
      constexpr int k = decltype(jj)::value;
      const int j = (int)threadIdx.x + k * NT;
      // (half 1 uses positions below NF/2 only: its entry NF/2 would be ky = ny + 1)
      if (j < NQ && !(part == 1 && j == NF / 2)) {
        const uint32_t ky = (uint32_t)ky_of(j);
        if constexpr (OP == COL_CHIRP1 || OP == COL_CHIRP1_CONJ) qys[k] = gld(I.qy1, ky);
        else if constexpr (OP == COL_CHIRP2 || OP == COL_CHIRP2_CONJ) qys[k] = gld(I.qy2, ky);
        else qys[k] = make_float2(gldf(OP == COL_NESTEROV ? I.gy : I.iy, ky), 0.f);
      }
    });
  }
  // staged factor of position j: that of min(j, mirror_pos(j))
  auto ytab = [&](int j) { return qyl[j <= NF / 2 - part ? j : mirror_pos(j)]; };
  float2 v[E];
  static_for<0, E / R1>([&](auto cc) {
    static_for<0, R1>([&](auto qq) {
      constexpr int c = decltype(cc)::value, q = decltype(qq)::value;
      v[c * R1 + q] = gld(I.W, o_w + (uint32_t)((T * c + q * M1) * WS * nx));
    });
  });
  // Twiddles (and y factors) to LDS; the first pass needs none, and the
  // barrier after its LDS exchange orders these writes before the first use.
  if constexpr (TS::kMode != 0) tws.store(twl);
  if constexpr (YSTAGE) {
    static_for<0, KQ>([&](auto jj) {
      constexpr int k = decltype(jj)::value;
      const int j = (int)threadIdx.x + k * NT;
      if (j < NQ && !(part == 1 && j == NF / 2)) qyl[j] = qys[k];
    });
  }
  fft_forward<Plan, T>(v, t, tw, lv);

  // Fourier-domain step; element e = c*RL + r holds position j = t + T c + r ML.
  const int kx = HALF ? s : kx_of_col(s, nx);
  const float fx = freq_of(kx, nx);
  double acc = 0.0;

  if constexpr (OP == COL_NESTEROV) {
    // d = F{Re g} + i P F{Im g} + STF-weighted regulariser; with
    // F{Re a}_k = (A_k + conj A_{-k})/2 and P, 1 - STF even in k, its terms in
    // G(-k) and Psi(-k) are conj(h(-k)) with h = (1-P)/2 G + g2 c2 Psi: each
    // lane hands h of its elements to their mirror lanes through LDS (column
    // -kx is the neighbour position mirror_col(s), inside this tile) and keeps
    // the rest of the step in registers.
    //
    // The Nesterov state is the last two gradient-step spectra Z_k and Z_{k-1},
    // in psi_hat and z_hat with roles alternating on the parity of k, so one
    // field is written per iteration (Z_{k+1} over Z_{k-1}); the extrapolated
    // Psi_k = Z_k + beta_{k-1} (Z_k - Z_{k-1}) is rebuilt here, the same
    // expression that formed it at the end of the previous iteration.
    const int wm = mirror_col(s) - tile * W;
    const LdsView lm{lds + wm, W};
    const int kg = I.k0 + S.iter;
    float2* const z_cur = (kg & 1) ? I.z_hat : I.psi_hat;
    float2* const z_old = (kg & 1) ? I.psi_hat : I.z_hat;
    const float bp = kg > 0 ? (float)S.beta[kg - 1] : 0.f;
    const float bf = (float)S.beta[kg];
    const float gxv = gldf(I.gx, kx);
    // State and STF loads in batches of NA, the next batch in flight while
    // this one is combined; the scheduling barriers keep the compiler from
    // hoisting every load, which would not fit in 128 registers.  Z_k stays
    // in registers for the momentum term.
    constexpr int NA = 4;
    static_assert(E % NA == 0, "state batches");
    float2 zk[E], zp[2][NA];
    float gb[2][NA];
    const uint32_t o_a = opaque(o_ld);
    auto load_state = [&](auto bb, int slot) {
      static_for<0, NA>([&](auto uu) {
        constexpr int u = decltype(uu)::value, e = decltype(bb)::value * NA + u;
        const int j = t + T * (e / RL) + (e % RL) * ML;
        zk[e] = gld(z_cur, o_a + (uint32_t)((j - t) * nx));
        zp[slot][u] = gld(z_old, o_a + (uint32_t)((j - t) * nx));
        gb[slot][u] = ytab(j).x;
      });
    };
    load_state(std::integral_constant<int, 0>{}, 0);
    static_for<0, E / NA>([&](auto bb) {
      constexpr int b = decltype(bb)::value;
      if constexpr (b + 1 < E / NA) load_state(std::integral_constant<int, b + 1>{}, (b + 1) & 1);
      __builtin_amdgcn_sched_barrier(0);
      static_for<0, NA>([&](auto uu) {
        constexpr int u = decltype(uu)::value, e = b * NA + u;
        const int j = t + T * (e / RL) + (e % RL) * ML;
        const float2 z0 = zk[e], z1 = zp[b & 1][u];
        const float2 ps = make_float2(z0.x + bp * (z0.x - z1.x), z0.y + bp * (z0.y - z1.y));
        const float P = pinv_of(I, fx, freq_of(ky_of(j), NY));
        // G = F{s Re g} + i F{Im g} with s = kGradReScale: the Hermitian split
        // with Re g unscaled gives a = (1/s + P)/2, c = (1/s - P)/2
        const float a = 0.5f * (kGradReUnscale + P), c = 0.5f * (kGradReUnscale - P);
        const float g2 = gxv + (1.f - gxv) * gb[b & 1][u];  // 1 - STFx STFy without cancellation
        const float r1 = g2 * I.alpha_c1, r2 = g2 * I.alpha_c2;
        lv.at(j) = make_float2(c * v[e].x + r2 * ps.x, c * v[e].y + r2 * ps.y);
        // Psi - eta (a G + g2 c1 Psi); the mirror's share follows the exchange
        v[e] = make_float2(ps.x - I.eta * (a * v[e].x + r1 * ps.x), ps.y - I.eta * (a * v[e].y + r1 * ps.y));
      });
      __builtin_amdgcn_sched_barrier(0);
    });
    __syncthreads();
    const uint32_t o_up = opaque(o_ld);
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      const int j = t + T * (e / RL) + (e % RL) * ML;
      const int kl = (int)opaque((uint32_t)t) + T * (e / RL) + (e % RL) * ML;
      const float2 hm = lm.at(mirror_pos(kl));
      const float2 z = make_float2(v[e].x - I.eta * hm.x, v[e].y + I.eta * hm.y);  // - eta conj(h(-k))
      const float2 pn = make_float2(z.x + bf * (z.x - zk[e].x), z.y + bf * (z.y - zk[e].y));
      gst(z_old, o_up + (uint32_t)((j - t) * nx), z);  // Z_{k+1}; this lane read Z_{k-1} here above
      v[e] = cscale(pn, I.inv_m);
    });
    __syncthreads();
  } else if constexpr (OP == COL_DIRECTION) {
    // Needs G(-k) and Psi(-k): exchange through LDS.  Column -kx is the
    // neighbour position mirror_col(s), inside this tile.
    const int wm = mirror_col(s) - tile * W;
    const LdsView lm{lds + wm, W};
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      lv.at(t + T * (e / RL) + (e % RL) * ML) = v[e];
    });
    __syncthreads();
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      const int j = t + T * (e / RL) + (e % RL) * ML;
      const float2 gm = lm.at(mirror_pos(j));
      const float P = pinv_of(I, fx, freq_of(ky_of(j), NY));
      const float a = 0.5f * (kGradReUnscale + P), b = 0.5f * (kGradReUnscale - P);
      // G = F{s Re g} + i F{Im g} (s = kGradReScale):
      // (1/s+P)/2 G + (1/s-P)/2 conj(G(-k)) = F{Re g} + i P F{Im g}
      v[e] = make_float2(a * v[e].x + b * gm.x, a * v[e].y - b * gm.y);
    });
    __syncthreads();
    static_for<0, E>([&](auto ee) {  // Psi to LDS: each lane needs Psi(k) and Psi(-k)
      constexpr int e = decltype(ee)::value;
      const int j = t + T * (e / RL) + (e % RL) * ML;
      lv.at(j) = gld(I.psi_hat, o_ld + (uint32_t)((j - t) * nx));
    });
    __syncthreads();
    const float gxv = gldf(I.gx, kx);
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      const int j = t + T * (e / RL) + (e % RL) * ML;
      const float2 pk = lv.at(j);
      const float2 pm = lm.at(mirror_pos(j));
      const float g2 = gxv + (1.f - gxv) * gldf(I.gy, ky_of(j));   // 1 - STFx STFy without cancellation
      // Re(a) F{Re psi} + i Im(a) F{Im psi} = c1 Psi + c2 conj(Psi(-k))
      const float2 reg = make_float2(I.alpha_c1 * pk.x + I.alpha_c2 * pm.x, I.alpha_c1 * pk.y - I.alpha_c2 * pm.y);
      v[e] = cscale(make_float2(v[e].x + g2 * reg.x, v[e].y + g2 * reg.y), I.inv_m);
    });
    __syncthreads();
  } else {
    float2 qx = make_float2(1.f, 0.f);
    float ixv = 1.f;
    if constexpr (OP == COL_CHIRP1 || OP == COL_CHIRP1_CONJ) qx = gld(I.qx1, kx);
    if constexpr (OP == COL_CHIRP2 || OP == COL_CHIRP2_CONJ) qx = gld(I.qx2, kx);
    // (half form: the packed column 0 carries its x factors from the row sweeps)
    if constexpr (OP == COL_BLUR || OP == COL_BLUR_LOSS) ixv = (HALF && s == 0) ? 1.f : gldf(I.ix, kx);
    // half form: columns s > 0 stand for kx and -kx in the loss
    const double wgt = (HALF && s > 0) ? 2.0 : 1.0;
    constexpr bool CHIRP = OP == COL_CHIRP1 || OP == COL_CHIRP1_CONJ || OP == COL_CHIRP2 || OP == COL_CHIRP2_CONJ;
    constexpr bool CONJ = OP == COL_CHIRP1_CONJ || OP == COL_CHIRP2_CONJ;
    constexpr bool L1 = OP == COL_CHIRP1 || OP == COL_CHIRP1_CONJ;
    if constexpr (CHIRP) {
      const float two_pi_a = L1 ? I.two_pi_a1 : I.two_pi_a2;
      // the y factors carry the 1/m of the inverse transform
      // y factor of position j (staged: that of min(j, mirror_pos(j)); else from the table)
      auto qy_at = [&](int j) { return ytab(j); };
      if (I.series && I.cross) {
        static_for<0, E>([&](auto ee) {
          constexpr int e = decltype(ee)::value;
          const int j = t + T * (e / RL) + (e % RL) * ML;
          const int ky = ky_of(j);
          float2 q = transfer_sep(qx, qy_at(j), fx, freq_of(ky, NY), I.s_coef_f, two_pi_a);
          if (CONJ) q = cconj(q);
          v[e] = cmul(v[e], q);
        });
      } else if (I.series) {
        static_for<0, E>([&](auto ee) {
          constexpr int e = decltype(ee)::value;
          const int j = t + T * (e / RL) + (e % RL) * ML;
          float2 q = cmul(qx, qy_at(j));
          if (CONJ) q = cconj(q);
          v[e] = cmul(v[e], q);
        });
      } else {
        const double a = L1 ? I.chirp1_rev : I.chirp2_rev;
        static_for<0, E>([&](auto ee) {  // rare path: one out-of-line FP64 call per element
          constexpr int e = decltype(ee)::value;
          const int ky = ky_of(t + T * (e / RL) + (e % RL) * ML);
          float2 q = transfer_direct(a, I.s_coef, fx, freq_of(ky, NY));
          if (CONJ) q = cconj(q);
          v[e] = cscale(cmul(v[e], q), I.inv_m);
        });
      }
    } else {
      static_for<0, E>([&](auto ee) {
        constexpr int e = decltype(ee)::value;
        const int j = t + T * (e / RL) + (e % RL) * ML;
        const int ky = ky_of(j);
        const uint32_t o_e = (uint32_t)((part * NF + j) * nx + s);  // this element's place in the spectra
        if constexpr (OP == COL_BLUR) {
          v[e] = cscale(v[e], ixv * gldf(I.iy, ky) * I.inv_m);
        } else if constexpr (OP == COL_BLUR_LOSS) {
          const float h = ixv * ytab(j).x;
          const float2 yh = gld(I.y_hat, o_e);
          const float2 rr = make_float2(h * v[e].x - yh.x, h * v[e].y - yh.y);
          acc += wgt * ((double)rr.x * (double)rr.x + (double)rr.y * (double)rr.y);
          v[e] = cscale(rr, h * I.inv_m);
        } else if constexpr (OP == COL_SPEC_YHAT) {
          gst(I.y_hat, o_e, v[e]);
        } else if constexpr (OP == COL_SPEC_PSIHAT) {
          gst(I.psi_hat, o_e, v[e]);
          if (I.z_hat) gst(I.z_hat, o_e, v[e]);  // Z_{-1} = Z_0 = Psi_0
        }
      });
    }
  }

  if constexpr (ColOpTraits<OP>::kInverse) {
    fft_inverse<Plan, T>(v, t, twr, lv);
    const uint32_t o_st = opaque(o_w);
    static_for<0, E / R1>([&](auto cc) {
      static_for<0, R1>([&](auto qq) {
        constexpr int c = decltype(cc)::value, q = decltype(qq)::value;
        gst(I.W, o_st + (uint32_t)((T * c + q * M1) * WS * nx), v[c * R1 + q]);
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
      I.loss_partial[part * ntile + tile] = sum;
    }
  }
}

template <int NY, int W, int OP>
__global__ void __launch_bounds__(ColSweepCfg<NY>::T * W, (col_min_waves<NY, W, OP>())) col_sweep(Sweep S) {
  __shared__ float2 lds[ColLds<NY, W>::kExchange];
  __shared__ float2 twl[ColLds<NY, W>::kTwiddles];
  __shared__ float2 qyl[col_op_ystage(OP) ? ColLds<NY, W>::kYTable : 1];
  // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous range of tiles so that tiles sharing 128-byte lines meet in
  // the same L2.
  col_body<NY, W, OP>(S, xcd_contiguous<true>(blockIdx.x, gridDim.x), lds, twl, qyl);
}

// ------------------------------------------------------------------ plain path kernels

// Out-of-place FFT of every row (natural order in and out).
template <int NX, int DIR>
__global__ void __launch_bounds__(RowCfg<NX>::T * RowCfg<NX>::RW, 2)
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
    fft_forward<Plan, T>(v, t, TwPass{tw}, lv);
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      dst[rbase + t + T * (e / RL) + (e % RL) * ML] = v[e];
    });
  } else {
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      v[e] = src[rbase + t + T * (e / RL) + (e % RL) * ML];
    });
    fft_inverse<Plan, T>(v, t, TwPass{tw + Plan::tw_total()}, lv);
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      dst[rbase + t + T * (e / R1) + (e % R1) * M1] = v[e];
    });
  }
}

// In-place FFT of every column (natural order) of gridDim.y planes
// plane_stride elements apart.
template <int NY, int DIR>
__global__ void __launch_bounds__(ColCfg<NY>::T * ColCfg<NY>::WA, 2)
plain_fft_cols(float2* __restrict__ a, int nx, const float2* tw, size_t plane_stride) {
  a += blockIdx.y * plane_stride;
  using C = ColCfg<NY>;
  using Plan = typename C::Plan;
  constexpr int T = C::T, W = C::WA, E = NY / T;
  static_assert(T * W <= 1024, "workgroup too large");
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
    fft_forward<Plan, T>(v, t, TwPass{tw}, lv);
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      a[(size_t)(t + T * (e / RL) + (e % RL) * ML) * nx + s] = v[e];
    });
  } else {
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      v[e] = a[(size_t)(t + T * (e / RL) + (e % RL) * ML) * nx + s];
    });
    fft_inverse<Plan, T>(v, t, TwPass{tw + Plan::tw_total()}, lv);
    static_for<0, E>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      a[(size_t)(t + T * (e / R1) + (e % R1) * M1) * nx + s] = v[e];
    });
  }
}

template <int N, int OP, int PLAN, bool PAIR>
hipError_t launch_row_one(int nblocks, const Sweep& S, hipStream_t st) {
  hipLaunchKernelGGL((row_sweep<N, OP, PLAN, PAIR>), dim3(nblocks), dim3(row_threads<N, PLAN>()), 0, st, S);
  return hipGetLastError();
}

// Row sweep `op` with radix plan `plan` (tunable sweeps only; the others
// always run with their default plan).
template <int N, int OP, bool PAIR>
hipError_t launch_row_plan(int plan, int nblocks, const Sweep& S, hipStream_t st) {
  if (plan == 1) return launch_row_one<N, OP, 1, PAIR>(nblocks, S, st);
  if constexpr (row_plan_count<N>() > 2) {
    if (plan == 2) return launch_row_one<N, OP, 2, PAIR>(nblocks, S, st);
  }
  if (plan == 0) return launch_row_one<N, OP, 0, PAIR>(nblocks, S, st);
  return hipErrorInvalidValue;
}

template <int N, bool PAIR>
hipError_t launch_row_np(int op, int plan, int nblocks, const Sweep& S, hipStream_t st) {
  switch (op) {
#define PWF_TUNABLE(o) case o: return launch_row_plan<N, o, PAIR>(plan, nblocks, S, st);
#define PWF_FIXED(o) case o: return launch_row_one<N, o, row_alt_default<N>(o) ? 1 : 0, PAIR>(nblocks, S, st);
    PWF_TUNABLE(ROW_PSI_UPDATE) PWF_TUNABLE(ROW_PSI_UPDATE_CORR) PWF_TUNABLE(ROW_MUL_T) PWF_TUNABLE(ROW_MUL_CONJ_T) PWF_TUNABLE(ROW_INTENSITY)
    PWF_TUNABLE(ROW_BACKBLUR) PWF_TUNABLE(ROW_GRAD)
    PWF_FIXED(ROW_START) PWF_FIXED(ROW_FORWARD_OUT) PWF_FIXED(ROW_REAL_FFT) PWF_FIXED(ROW_CPLX_FFT)
    PWF_FIXED(ROW_IFFT_OUT)
#undef PWF_TUNABLE
#undef PWF_FIXED
    default: return hipErrorInvalidValue;
  }
}

// Row sweep on side N; rows are paired (PAIR) when the launch's column
// transform is split (Sweep::pair_half > 0).
template <int N>
hipError_t launch_row_n(int op, int plan, int nblocks, const Sweep& S, hipStream_t st) {
  return S.pair_half > 0 ? launch_row_np<N, true>(op, plan, nblocks, S, st)
                         : launch_row_np<N, false>(op, plan, nblocks, S, st);
}

template <int N, int W>
hipError_t launch_col_nw(int op, int nblocks, const Sweep& S, hipStream_t st) {
  using C = ColSweepCfg<N>;
  const dim3 grid(nblocks), block(C::T * W);
  switch (op) {
#define PWF_CASE(o) case o: hipLaunchKernelGGL((col_sweep<N, W, o>), grid, block, 0, st, S); break;
    PWF_CASE(COL_CHIRP1) PWF_CASE(COL_CHIRP2) PWF_CASE(COL_CHIRP2_CONJ) PWF_CASE(COL_CHIRP1_CONJ)
    PWF_CASE(COL_BLUR_LOSS) PWF_CASE(COL_BLUR) PWF_CASE(COL_NESTEROV) PWF_CASE(COL_DIRECTION)
    PWF_CASE(COL_SPEC_YHAT) PWF_CASE(COL_SPEC_PSIHAT)
#undef PWF_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int N>
hipError_t launch_col_n(int width, int op, int nblocks, const Sweep& S, hipStream_t st) {
  using C = ColSweepCfg<N>;
  if (width == C::WA) return launch_col_nw<N, C::WA>(op, nblocks, S, st);
  if (width == C::WB) return launch_col_nw<N, C::WB>(op, nblocks, S, st);
  return hipErrorInvalidValue;
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
hipError_t plain_cols_n(int dir, float2* a, int nx, const float2* tw, int planes, size_t plane_stride,
                        hipStream_t st) {
  using C = ColCfg<N>;
  const dim3 grid(nx / C::WA, planes), block(C::T * C::WA);
  if (dir < 0) hipLaunchKernelGGL((plain_fft_cols<N, -1>), grid, block, 0, st, a, nx, tw, plane_stride);
  else hipLaunchKernelGGL((plain_fft_cols<N, 1>), grid, block, 0, st, a, nx, tw, plane_stride);
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

// Twiddle tables of an N-point plan followed by those of its reversed plan:
// which = 0 for the row plan, 1 for the column plan, 2 for the alternative row
// plan, 3 for the third row plan.
template <int N>
int plan_twiddles_n(int which, float2* out) {
  auto emit = [&](auto tag) {
    using Plan = decltype(tag);
    using RPlan = typename Reverse<Plan>::type;
    static_assert(Plan::valid(), "radices must multiply to N");
    if (out) {
      fill_twiddles<Plan>(out);
      fill_twiddles<RPlan>(out + Plan::tw_total());
    }
    return Plan::tw_total() + RPlan::tw_total();
  };
  return which == 0   ? emit(typename RowCfg<N>::Plan{})
         : which == 1 ? emit(typename ColCfg<N>::Plan{})
         : which == 2 ? emit(typename RowCfgAlt<N>::Plan{})
                      : emit(typename RowCfgAlt2<N>::Plan{});
}

}  // namespace pwf
