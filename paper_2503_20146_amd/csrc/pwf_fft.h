// Device-side FFT engine for gfx950: register-resident radix-R butterflies
// with compile-time twiddles, joined by Stockham auto-sort passes through LDS.
//
// A transform of length N is shared by T lanes; each lane holds E = N / T
// complex values in registers.  Pass p (radix R, stride L = product of the
// earlier radices, m = N / R) computes, for butterfly j in [0, m):
//     k = j mod L,  a_q = x[j + q m] * w_{L R}^{q k},  b_r = sum_q a_q w_R^{q r},
//     y[(j / L) L R + k + r L] = b_r,
// with w_n = exp(-2 pi i / n) forward and its conjugate inverse.  Lane t owns
// butterflies j = t + T c.  The first pass reads a_q from registers that the
// caller loaded at positions t + T c + q m (coalesced along t); the last pass
// (L = m) leaves b_r in registers at frequency t + T c + r m, which is also
// the input layout of an inverse transform whose first radix is the same.
// Between passes the data goes through LDS.  Inverse transforms are
// unnormalised.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace pwf {

// ------------------------------------------------------------------ helpers

template <int I, int END, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < END) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, END>(static_cast<F&&>(f));
  }
}

__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n >> 1); }
__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }

__host__ __device__ constexpr int bitrev(int x, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1) << (bits - 1 - i);
  return r;
}

// cos and sin of 2 pi num / den evaluated at compile time (Taylor series after
// an exact reduction to the first octant).
__host__ __device__ constexpr double cx_taylor_sin(double x) {
  double term = x, sum = x;
  for (int i = 1; i < 14; ++i) {
    term *= -x * x / ((2 * i) * (2 * i + 1));
    sum += term;
  }
  return sum;
}
__host__ __device__ constexpr double cx_taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < 14; ++i) {
    term *= -x * x / ((2 * i - 1) * (2 * i));
    sum += term;
  }
  return sum;
}
// angle = 2 pi num / den, returns cos (which=0) or sin (which=1)
__host__ __device__ constexpr double cx_trig(long num, long den, int which) {
  num %= den;
  if (num < 0) num += den;
  // reduce to [0, den/8] using exact symmetries: work with octant index
  long n8 = num * 8;
  int oct = (int)(n8 / den);        // 0..7
  long rem = n8 - (long)oct * den;  // angle within octant = 2 pi rem / (8 den)
  const double quarter_pi = 0.78539816339744830961566084581987572;
  double a = quarter_pi * (double)rem / (double)den;  // [0, pi/4)
  double b = quarter_pi - a;                           // (0, pi/4]
  double c = 0, s = 0;
  switch (oct) {
    case 0: c = cx_taylor_cos(a); s = cx_taylor_sin(a); break;
    case 1: c = cx_taylor_sin(b); s = cx_taylor_cos(b); break;
    case 2: c = -cx_taylor_sin(a); s = cx_taylor_cos(a); break;
    case 3: c = -cx_taylor_cos(b); s = cx_taylor_sin(b); break;
    case 4: c = -cx_taylor_cos(a); s = -cx_taylor_sin(a); break;
    case 5: c = -cx_taylor_sin(b); s = -cx_taylor_cos(b); break;
    case 6: c = cx_taylor_sin(a); s = -cx_taylor_cos(a); break;
    default: c = cx_taylor_cos(b); s = -cx_taylor_sin(b); break;
  }
  return which == 0 ? c : s;
}

// ------------------------------------------------------------------ complex helpers

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// Multiply by w_n^k (DIR = -1 forward, +1 inverse) with n, k compile-time.
template <int DIR, int K, int NN>
__device__ __forceinline__ float2 twiddle_const(float2 a) {
  constexpr int k = ((K % NN) + NN) % NN;
  if constexpr (k == 0) {
    return a;
  } else if constexpr (4 * k == NN) {  // w = -i (fwd) / +i (inv)
    return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
  } else if constexpr (2 * k == NN) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (4 * k == 3 * NN) {  // w = +i (fwd) / -i (inv)
    return DIR < 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
  } else if constexpr ((8 * k) % NN == 0) {  // odd multiple of 45 degrees: |cos| = |sin|
    constexpr float c = (float)cx_trig(k, NN, 0);
    constexpr float s = (float)(DIR * cx_trig(k, NN, 1));
    if constexpr ((c > 0) == (s > 0)) {  // s = c
      return make_float2(c * (a.x - a.y), c * (a.x + a.y));
    } else {  // s = -c
      return make_float2(c * (a.x + a.y), c * (a.y - a.x));
    }
  } else {
    constexpr float c = (float)cx_trig(k, NN, 0);
    constexpr float s = (float)(DIR * cx_trig(k, NN, 1));  // exp(DIR i 2 pi k / n)
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

// Register position of output r of the in-register R-point DFT below.
__host__ __device__ constexpr int dft_pos(int R, int r) {
  return R == 4 ? r : R == 8 ? 4 * (r % 2) + r / 2 : R == 16 ? 4 * (r % 4) + r / 4 : bitrev(r, ilog2(R));
}

// 4-point DFT on the registers at compile-time positions P0..P3; outputs in
// natural order at the same positions.
template <int DIR, int P0, int P1, int P2, int P3, int E>
__device__ __forceinline__ void dft4_at(float2 (&a)[E]) {
  const float2 t0 = cadd(a[P0], a[P2]), t1 = csub(a[P0], a[P2]);
  const float2 t2 = cadd(a[P1], a[P3]), t3 = csub(a[P1], a[P3]);
  a[P0] = cadd(t0, t2);
  a[P2] = csub(t0, t2);
  // forward: X1 = t1 - i t3, X3 = t1 + i t3 (inverse: signs swapped)
  const float2 it3 = DIR < 0 ? make_float2(t3.y, -t3.x) : make_float2(-t3.y, t3.x);
  a[P1] = cadd(t1, it3);
  a[P3] = csub(t1, it3);
}

// Generic radix-2 decimation-in-frequency network (outputs bit-reversed).
template <int R, int DIR, int OFF, int E>
__device__ __forceinline__ void dft_radix2(float2 (&a)[E]) {
  constexpr int LOGR = ilog2(R);
  static_for<0, LOGR>([&](auto st) {
    constexpr int half = R >> (decltype(st)::value + 1);
    static_for<0, R / (2 * half)>([&](auto bb) {
      constexpr int blk = decltype(bb)::value * 2 * half;
      static_for<0, half>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        float2 x = a[OFF + blk + i];
        float2 y = a[OFF + blk + i + half];
        a[OFF + blk + i] = cadd(x, y);
        a[OFF + blk + i + half] = twiddle_const<DIR, i, 2 * half>(csub(x, y));
      });
    });
  });
}

// In-register radix-R DFT.  On entry a[OFF + q] holds input q; on exit
// a[OFF + dft_pos(R, r)] holds output r.  R = 4, 8, 16 use radix-4 codelets
// (8 = 2 x 4, 16 = 4 x 4, decimation in frequency); other R the radix-2 network.
template <int R, int DIR, int OFF, int E>
__device__ __forceinline__ void dft_reg(float2 (&a)[E]) {
  if constexpr (R == 4) {
    dft4_at<DIR, OFF, OFF + 1, OFF + 2, OFF + 3>(a);
  } else if constexpr (R == 8) {
    // stage 1: 2-point DFTs over n1 for each n2, twiddle w8^(n2 k1)
    static_for<0, 4>([&](auto nn) {
      constexpr int n2 = decltype(nn)::value;
      const float2 u = a[OFF + n2], w = a[OFF + n2 + 4];
      a[OFF + n2] = cadd(u, w);
      a[OFF + n2 + 4] = twiddle_const<DIR, n2, 8>(csub(u, w));
    });
    // stage 2: 4-point DFTs over n2 for each k1; X[k1 + 2 k2] lands at 4 k1 + k2
    dft4_at<DIR, OFF + 0, OFF + 1, OFF + 2, OFF + 3>(a);
    dft4_at<DIR, OFF + 4, OFF + 5, OFF + 6, OFF + 7>(a);
  } else if constexpr (R == 16) {
    // stage 1: 4-point DFTs over n1 (stride 4) for each n2, twiddle w16^(n2 k1)
    static_for<0, 4>([&](auto nn) {
      constexpr int n2 = decltype(nn)::value;
      dft4_at<DIR, OFF + n2, OFF + n2 + 4, OFF + n2 + 8, OFF + n2 + 12>(a);
      a[OFF + n2 + 4] = twiddle_const<DIR, n2 * 1, 16>(a[OFF + n2 + 4]);
      a[OFF + n2 + 8] = twiddle_const<DIR, n2 * 2, 16>(a[OFF + n2 + 8]);
      a[OFF + n2 + 12] = twiddle_const<DIR, n2 * 3, 16>(a[OFF + n2 + 12]);
    });
    // stage 2: 4-point DFTs over n2 for each k1; X[k1 + 4 k2] lands at 4 k1 + k2
    static_for<0, 4>([&](auto kk) {
      constexpr int b = 4 * decltype(kk)::value;
      dft4_at<DIR, OFF + b, OFF + b + 1, OFF + b + 2, OFF + b + 3>(a);
    });
  } else {
    dft_radix2<R, DIR, OFF>(a);
  }
}

// ------------------------------------------------------------------ Stockham passes

// LDS index with one pad element every 32 (breaks power-of-two bank strides).
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 5); }
__host__ __device__ constexpr int lds_len(int n) { return n + (n >> 5); }

// Where a transform's elements live in LDS: element i -> base[(pad(i)) * stride].
struct LdsView {
  float2* base;
  int stride;
  __device__ __forceinline__ float2& at(int i) const { return base[lds_pad(i) * stride]; }
};

// Twiddles of pass p of an N-point transform: table[q * L + k] = w_{L R}^{q k}
// (forward sign; the inverse uses the conjugate).  Tables for all passes of a
// plan are concatenated; offsets are compile-time.
template <int N, int... RS>
struct FftPlan {
  static constexpr int kN = N;
  static constexpr int NPASS = sizeof...(RS);
  static constexpr int radix[NPASS] = {RS...};
  static constexpr int stride_before(int p) {
    int l = 1;
    for (int i = 0; i < p; ++i) l *= radix[i];
    return l;
  }
  static constexpr int tw_offset(int p) {
    int off = 0;
    for (int i = 1; i < p; ++i) off += stride_before(i) * radix[i];
    return off;
  }
  static constexpr int tw_total() { return tw_offset(NPASS); }
  static constexpr bool valid() {
    int prod = 1;
    for (int i = 0; i < NPASS; ++i) prod *= radix[i];
    return prod == N;
  }
};

// Twiddle sources.  A pass with stride L and radix R needs w_{LR}^{qk} for
// 0 < q < R, 0 <= k < L (forward sign; the inverse conjugates).
//
// TwPass: per-pass tables in global memory, table[tw_offset(P) + q L + k]
// (the layout plan_twiddles writes).
struct TwPass {
  const float2* tw;
  template <class Plan, int P, int q>
  __device__ __forceinline__ float2 get(int k) const {
    return tw[Plan::tw_offset(P) + q * Plan::stride_before(P) + k];
  }
};

// TwTable: one table of w_N^m (m = 0..N-1) for every pass of both
// directions: w_{LR}^{qk} = w_N^{qk N/(LR)}, and qk N/(LR) < N.
// DIV = 2 keeps only m < N/2 and uses w_N^(m + N/2) = -w_N^m (a sign flip of
// both parts); DIV = 4 keeps m < N/4 and uses w_N^(m + a N/4) = (-i)^a w_N^m
// (a swap of the parts and sign flips).  Both cut the staged table at the
// cost of a few integer ops per twiddle; the rotations are exact.
template <int N, int DIV = 1>
struct TwTable {
  static_assert(DIV == 1 || DIV == 2 || DIV == 4, "table fraction");
  const float2* tab;
  template <class Plan, int P, int q>
  __device__ __forceinline__ float2 get(int k) const {
    const int i = q * (N / (Plan::stride_before(P) * Plan::radix[P])) * k;
    if constexpr (DIV == 1) {
      return tab[i];
    } else if constexpr (DIV == 2) {
      const float2 w = tab[i & (N / 2 - 1)];
      const uint32_t sg = (uint32_t)(i & (N / 2)) << (31 - ilog2(N / 2));
      return make_float2(__uint_as_float(__float_as_uint(w.x) ^ sg), __uint_as_float(__float_as_uint(w.y) ^ sg));
    } else {
      const float2 w = tab[i & (N / 4 - 1)];
      const int a = (i >> ilog2(N / 4)) & 3;   // quarter turns: (-i)^a
      const float x = (a & 1) ? w.y : w.x, y = (a & 1) ? w.x : w.y;
      const uint32_t sx = (uint32_t)(a & 2) << 30, sy = (uint32_t)((a ^ (a >> 1)) & 1) << 31;
      return make_float2(__uint_as_float(__float_as_uint(x) ^ sx), __uint_as_float(__float_as_uint(y) ^ sy));
    }
  }
};

// One pass over registers.  v holds B = E/R butterflies' inputs at v[c*R + q].
// Applies the inter-pass twiddle and the radix-R DFT; leaves outputs at
// v[c*R + dft_pos(R, r)].
template <class Plan, int P, int T, int DIR, int E, class TW>
__device__ __forceinline__ void pass_compute(float2 (&v)[E], int t, const TW& tw) {
  constexpr int N = E * T;
  constexpr int R = Plan::radix[P];
  constexpr int L = Plan::stride_before(P);
  constexpr int B = E / R;
  static_assert(B * R == E, "radix must divide elements per lane");
  static_assert((N / R) % T == 0, "lanes must divide butterflies");
  static_for<0, B>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    if constexpr (L > 1) {
      const int j = t + T * c;
      const int k = j & (L - 1);
      static_for<1, R>([&](auto qq) {
        constexpr int q = decltype(qq)::value;
        float2 w = tw.template get<Plan, P, q>(k);
        if constexpr (DIR > 0) w.y = -w.y;
        v[c * R + q] = cmul(v[c * R + q], w);
      });
    }
    dft_reg<R, DIR, c * R>(v);
  });
}

// Write pass-P outputs (permuted in registers, see dft_pos) to LDS at Stockham positions.
template <class Plan, int P, int T, int E>
__device__ __forceinline__ void pass_store_lds(const float2 (&v)[E], int t, LdsView lds) {
  constexpr int R = Plan::radix[P];
  constexpr int L = Plan::stride_before(P);
  constexpr int B = E / R;
  static_for<0, B>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    const int j = t + T * c;
    const int k = j & (L - 1);
    const int base = (j / L) * L * R + k;
    static_for<0, R>([&](auto rr) {
      constexpr int r = decltype(rr)::value;
      lds.at(base + r * L) = v[c * R + dft_pos(R, r)];
    });
  });
}

// Read pass-P inputs from LDS: v[c*R + q] = x[j + q m].
template <class Plan, int P, int T, int E>
__device__ __forceinline__ void pass_load_lds(float2 (&v)[E], int t, LdsView lds) {
  constexpr int N = E * T;
  constexpr int R = Plan::radix[P];
  constexpr int M = N / R;
  constexpr int B = E / R;
  static_for<0, B>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    const int j = t + T * c;
    static_for<0, R>([&](auto qq) {
      constexpr int q = decltype(qq)::value;
      v[c * R + q] = lds.at(j + q * M);
    });
  });
}

// Put the last pass's permuted outputs back in natural register order so
// that v[c*R + r] holds frequency t + T c + r m.
template <int R, int E>
__device__ __forceinline__ void unscramble(float2 (&v)[E]) {
  constexpr int B = E / R;
  float2 tmp[R];
  static_for<0, B>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    static_for<0, R>([&](auto rr) { tmp[decltype(rr)::value] = v[c * R + decltype(rr)::value]; });
    static_for<0, R>([&](auto rr) {
      constexpr int r = decltype(rr)::value;
      v[c * R + r] = tmp[dft_pos(R, r)];
    });
  });
}

// Order a pass's LDS stores before the next pass's loads.  WAVE: the
// transform's lanes (and the LDS region they exchange through) belong to one
// wave, whose LDS operations complete in issue order, so a compiler fence at
// wavefront scope suffices; otherwise a workgroup barrier.
template <bool WAVE>
__device__ __forceinline__ void exchange_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Forward transform: registers in "first-radix layout" (v[c*R0 + q] = x[t + T c
// + q N/R0]) -> registers in "last-radix layout" (v[c*RL + r] = X[t + T c + r
// N/RL]).  The LDS region must be free on entry; it is free again on exit
// (a trailing barrier is issued only between passes).
template <class Plan, int T, bool WAVE = false, int E, class TW>
__device__ __forceinline__ void fft_forward(float2 (&v)[E], int t, const TW& tw, LdsView lds) {
  static_for<0, Plan::NPASS>([&](auto pp) {
    constexpr int P = decltype(pp)::value;
    if constexpr (P > 0) {
      pass_load_lds<Plan, P, T>(v, t, lds);
      exchange_sync<WAVE>();
    }
    pass_compute<Plan, P, T, -1>(v, t, tw);
    if constexpr (P + 1 < Plan::NPASS) {
      pass_store_lds<Plan, P, T>(v, t, lds);
      exchange_sync<WAVE>();
    }
  });
  unscramble<Plan::radix[Plan::NPASS - 1]>(v);
}

// Inverse plan: the same radices in reverse order.
template <class Plan>
struct Reverse;
template <int N, int... RS>
struct Reverse<FftPlan<N, RS...>> {
  template <int... IS>
  static auto make(std::integer_sequence<int, IS...>)
      -> FftPlan<N, FftPlan<N, RS...>::radix[sizeof...(RS) - 1 - IS]...>;
  using type = decltype(make(std::make_integer_sequence<int, sizeof...(RS)>{}));
};

// Per-pass twiddle tables of a plan followed by those of its reversed plan,
// as plan_twiddles lays them out.  A palindromic plan (e.g. 32 x 32) is its
// own reverse, and the inverse then reads the forward tables (conjugated).
template <class Plan>
struct TwLayout {
  using RP = typename Reverse<Plan>::type;
  static constexpr bool kSelfReverse = std::is_same<Plan, RP>::value;
  static constexpr int kInverseAt = kSelfReverse ? 0 : Plan::tw_total();   // offset of the inverse tables
  static constexpr int kUsed = kSelfReverse ? Plan::tw_total() : Plan::tw_total() + RP::tw_total();
};

// Where a sweep kernel reads its twiddles from.  Mode 1: the per-pass tables
// of a palindromic plan staged in LDS (conflict-free reads; the inverse shares
// them).  Mode 2: the single table w_N^m staged in LDS (N entries, fewer than
// the per-pass tables of both directions), or the fraction 1/DIV of it (see
// TwTable).  Mode 0: per-pass tables read from global memory.  Above 1024
// points the full table (16 KB at 2048) would leave room for only one
// workgroup per CU beside the exchange buffer: kernels that pass STAGE_LARGE
// stage at least the half table there, the others use mode 0.
template <class Plan, int DIV = 1, bool STAGE_LARGE = false>
struct TwSel {
  static constexpr int N = Plan::kN;
  static constexpr int kDiv = N > 1024 && DIV < 2 ? 2 : DIV;
  static constexpr int kMode = N > 1024 ? (STAGE_LARGE ? 2 : 0) : (TwLayout<Plan>::kSelfReverse ? 1 : 2);
  static constexpr int kLds = kMode == 1 ? TwLayout<Plan>::kUsed : kMode == 2 ? N / kDiv : 1;
  using View = typename std::conditional<kMode == 2, TwTable<N, kDiv>, TwPass>::type;
  // pass: per-pass tables in global memory (forward, then reversed plan);
  // full: w_N^m in global memory; lds: the staged copy.
  __device__ static const float2* staged_from(const float2* pass, const float2* full) {
    return kMode == 1 ? pass : full;
  }
  __device__ static View forward(const float2* lds, const float2* pass) { return View{kMode == 0 ? pass : lds}; }
  __device__ static View inverse(const float2* lds, const float2* pass) {
    return View{kMode == 0 ? pass + Plan::tw_total() : kMode == 1 ? lds + TwLayout<Plan>::kInverseAt : lds};
  }
};

// Inverse transform: registers in last-radix layout of Plan -> registers in
// first-radix layout of Plan.  `twr` gives the twiddles of the reversed plan.
template <class Plan, int T, bool WAVE = false, int E, class TW>
__device__ __forceinline__ void fft_inverse(float2 (&v)[E], int t, const TW& twr, LdsView lds) {
  using RP = typename Reverse<Plan>::type;
  static_for<0, RP::NPASS>([&](auto pp) {
    constexpr int P = decltype(pp)::value;
    if constexpr (P > 0) {
      pass_load_lds<RP, P, T>(v, t, lds);
      exchange_sync<WAVE>();
    }
    pass_compute<RP, P, T, +1>(v, t, twr);
    if constexpr (P + 1 < RP::NPASS) {
      pass_store_lds<RP, P, T>(v, t, lds);
      exchange_sync<WAVE>();
    }
  });
  unscramble<RP::radix[RP::NPASS - 1]>(v);
}

}  // namespace pwf
