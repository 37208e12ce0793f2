// Per-instance descriptors, FFT configurations and the Fourier-domain windows
// of the PWF hot path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pwf_fft.h"

namespace pwf {

// Per-instance descriptor, uploaded to device memory once per call.  Field
// buffers are complex64 [ny][nx] unless noted.  Spectra (psi_hat, z_hat,
// y_hat and the x-transformed work field W) store column kx at the paired
// position s(kx) (see col_of_kx) so that kx and -kx are neighbours.
struct Inst {
  int32_t nx, ny;
  int32_t k0;           // iterations already done (momentum table offset)
  int32_t n_partials;   // number of loss partials (column tiles)
  float2* W;            // work field between sweeps
  float2* v;            // detector field v, saved by the forward for the gradient
  float2* u1;           // joint diffuser mode: field incident on the diffuser (S2), then
                        // conj(u1) a2 (S8); null otherwise
  float* u1max;         // joint diffuser mode: per-workgroup max |u1|^2 of S2
  float2* x;            // sample transmission x = exp(psi), saved for the gradient
  const float2* psi_src;// real-space psi that a forward pass starts from
  float2* psi;          // real-space psi written by a state initialisation
  float2* psi_hat;      // spectrum of psi (one-shot calls), or of z_k / z_{k-1} (iterations, k even / odd)
  float2* z_hat;        // spectrum of z_{k-1} / z_k (iterations, k even / odd)
  float2* y_hat;        // spectrum of the measured speckle
  const float* y;       // measured speckle (real space, float32)
  const float2* t;      // diffuser transmission
  const float* maxt2;   // device scalar max_r |t_r|^2
  float* f_out;         // forward-model output (float32), may be null
  float2* g_out;        // Wirtinger derivative output, may be null
  float2* out;          // real-space complex output of a final inverse pass
  double* loss_partial; // one FP64 partial per column tile
  double* loss_dst;     // loss destination (indexed by iteration), may be null
  double* corr_partial; // 4 FP64 partials per row block for the stopping correlation, or null
  int32_t* stop_iter;   // device: iteration at which the correlation stop fired (0 = running), or null
  int32_t n_corr_partials;
  float grad_mul;       // > 0: S10 scales by this instead of 1/max|t|^2
  // 1-D factors of the separable windows, indexed by DFT bin (built per call)
  float2* qx1; float2* qy1;  // exp(i theta_x), exp(i theta_y) of FreePropagation over L1
  float2* qx2; float2* qy2;  // same over L2
  float* ix; float* iy;      // IOTF factors exp(-c f^2)
  float* gx; float* gy;      // 1 - STF factors, 1 - exp(-c f^2)
  // Fourier-domain constants (frequencies f in cycles/pixel)
  double chirp1_rev;    // L1 lambda / (2 p^2): revolutions per f^2 (paraxial part)
  double chirp2_rev;    // L2 lambda / (2 p^2)
  double s_coef;        // (lambda / p)^2: lambda^2 rho^2 = s_coef f^2
  int32_t series;       // 1: separable chirp + power-series cross term; 0: direct FP64 chirp
  int32_t cross;        // 1: the cross term can change an FP32 result and is applied
  float two_pi_a1, two_pi_a2;  // 2 pi chirp_rev (radians per f^2), FP32 copy for the cross term
  float s_coef_f;
  float iotf_cx, iotf_cy;  // IOTF = exp(-(cx fx^2 + cy fy^2)), c = (pi/2) (x_coh/p)^2
  float stf_cx, stf_cy;    // STF  = exp(-(cx fx^2 + cy fy^2)), c = pi gamma (x_coh/p)^2
  const float* src_ix;     // caller's separable IOTF (PWF_SRC_IOTF) by DFT bin, or null
  const float* src_iy;
  float two_gamma;         // STF = IOTF^(2 gamma) for a caller's IOTF
  float pinv_scale;        // s_P; negative: preconditioner off
  float alpha_c1, alpha_c2;// (Re a + Im a)/2, (Re a - Im a)/2
  float eta;
  float inv_m;             // 1/(nx ny)
  double inv_m_d;
  float wiener_eps;     // calibration: Wiener regulariser of the IOTF deconvolution
  float rmse_scale;     // > 0: the forward output is the RMSE image |y - f| rmse_scale
};

// Loads and stores through the global address space, element i of a field
// at a 32-bit byte offset from its base.  Descriptor fields are generic
// pointers; without the cast the compiler emits flat instructions, which count
// against both the memory and the LDS wait counters.  With a workgroup-uniform
// base and a 32-bit offset it uses the scalar-base form of the global access
// instead of a 64-bit address per element.  Every field is below 4 GiB
// (sides up to 2048).
typedef float pwf_fv2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) pwf_fv2 pwf_gfv2;
typedef __attribute__((address_space(1))) float pwf_gf;
__device__ __forceinline__ float2 gld(const float2* p, uint32_t i) {
  const pwf_fv2 v = *(const pwf_gfv2*)((const char*)p + (i << 3));
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void gst(float2* p, uint32_t i, float2 a) {
  pwf_fv2 v;
  v.x = a.x;
  v.y = a.y;
  *(pwf_gfv2*)((char*)p + (i << 3)) = v;
}
__device__ __forceinline__ float gldf(const float* p, uint32_t i) { return *(const pwf_gf*)((const char*)p + (i << 2)); }
__device__ __forceinline__ void gstf(float* p, uint32_t i, float a) { *(pwf_gf*)((char*)p + (i << 2)) = a; }

// Paired column order of x-spectra: kx = 0 -> 0, kx = n/2 -> 1,
// 0 < kx < n/2 -> 2 kx, n/2 < kx < n -> 2 (n - kx) + 1.
__device__ __forceinline__ int col_of_kx(int kx, int n) {
  const int h = n >> 1;
  if (kx == 0) return 0;
  if (kx == h) return 1;
  return kx < h ? 2 * kx : 2 * (n - kx) + 1;
}
__device__ __forceinline__ int kx_of_col(int s, int n) {
  if (s == 0) return 0;
  if (s == 1) return n >> 1;
  return (s & 1) ? n - (s >> 1) : (s >> 1);
}
__device__ __forceinline__ int mirror_col(int s) { return s <= 1 ? s : (s ^ 1); }

// Scale of Re g in the forward transform of the gradient (S10), undone when
// the direction sweeps split the spectrum into F{Re g} and F{Im g}.  Below a
// few cycles per field the attenuation part's spectrum exceeds the phase
// part's by up to 1e5 (the phase is nearly invisible at low frequencies),
// and a transform that carries both at full size leaves FP32 rounding of
// F{Re g}'s size in F{Im g}, which P^-1 ~ n^2 / (4 pi^2 |k|^2) then
// amplifies (2.5e-3 relative error of d at 2048^2 in an FP32 model of the
// split).  With Re g scaled by 2^-7 that error is ~1e-5; the attenuation
// part, which P^-1 does not amplify, loses at most 7 bits of its own
// accuracy.  Powers of two: the scaling itself is exact.
constexpr float kGradReScale = 0.0078125f;   // 2^-7
constexpr float kGradReUnscale = 128.0f;     // 2^7

// Signed frequency in cycles/pixel of DFT bin k of an n-point axis (exact).
__device__ __forceinline__ float freq_of(int k, int n) {
  return (float)(k < (n >> 1) ? k : k - n) / (float)n;
}

// Transfer function Q = exp(i theta) of FreePropagation over L, carrier dropped:
// theta / 2 pi = -(L lambda / 2 p^2) f^2 * 2 / (1 + sqrt(1 - s)), s = (lambda/p)^2 f^2.
// The argument is formed and reduced modulo one revolution in FP64; the
// reduced angle goes to an FP32 sincos.  conj selects the backward direction.
__device__ __forceinline__ float2 transfer(double chirp_rev, double s_coef, int series, float fx, float fy,
                                           bool conj) {
  const double r2 = (double)fx * (double)fx + (double)fy * (double)fy;
  const double s = s_coef * r2;
  double c;
  if (series) {
    // 2/(1+sqrt(1-s)) = sum_n Catalan(n) (s/4)^n; exact to FP64 for s < 1e-4
    c = 1.0 + s * (0.25 + s * (0.125 + s * (0.078125 + s * 0.0546875)));
  } else {
    if (s >= 1.0) return make_float2(0.f, 0.f);
    c = 2.0 / (1.0 + sqrt(1.0 - s));
  }
  double rev = -chirp_rev * r2 * c;
  rev -= rint(rev);
  const float th = (float)(rev * 6.283185307179586476925);
  float sn, cs;
  sincosf(th, &sn, &cs);
  return make_float2(cs, conj ? -sn : sn);
}

// IOTF and regularisation window Gamma^2 = 1 - STF at DFT bin (kx, ky), from the
// per-call 1-D tables (see build_tables_kernel).
__device__ __forceinline__ float iotf_at(const Inst& I, int kx, int ky) { return I.ix[kx] * I.iy[ky]; }
__device__ __forceinline__ float gamma2_at(const Inst& I, int kx, int ky) {
  const float gx = I.gx[kx];
  return gx + (1.f - gx) * I.gy[ky];   // 1 - STFx STFy without cancellation
}
__device__ __forceinline__ float pinv_of(const Inst& I, float fx, float fy) {
  const float r2 = fx * fx + fy * fy;
  if (I.pinv_scale < 0.f) return 1.f;
  // 1/r2 from the hardware reciprocal refined by one Newton step (within an
  // ulp), instead of the full division sequence per element
  float r = __builtin_amdgcn_rcpf(r2);
  r = fmaf(fmaf(-r2, r, 1.f), r, r);
  return r2 > 0.f ? I.pinv_scale * r : 0.f;
}

// ------------------------------------------------------------------ FFT configurations

// Row sweeps: T lanes per row, RW rows per workgroup.  RowCfgAlt is a second
// plan per side with fewer elements per lane, for the sweeps whose real-space
// step is heavy (exp(psi) and FP64 correlation sums in the update sweep);
// row_uses_alt names the sweeps that take it.
template <int N> struct RowCfg;
template <> struct RowCfg<128>  { using Plan = FftPlan<128, 16, 8>;      static constexpr int T = 8,   RW = 32; };
template <> struct RowCfg<256>  { using Plan = FftPlan<256, 16, 16>;     static constexpr int T = 16,  RW = 16; };
template <> struct RowCfg<512>  { using Plan = FftPlan<512, 16, 8, 4>;   static constexpr int T = 32,  RW = 8; };
template <> struct RowCfg<1024> { using Plan = FftPlan<1024, 32, 32>;    static constexpr int T = 32,  RW = 8; };
template <> struct RowCfg<2048> { using Plan = FftPlan<2048, 32, 8, 8>;  static constexpr int T = 64,  RW = 4; };
template <int N> struct RowCfgAlt : RowCfg<N> {};
template <> struct RowCfgAlt<1024> { using Plan = FftPlan<1024, 16, 16, 4>; static constexpr int T = 64,  RW = 4; };
template <> struct RowCfgAlt<2048> { using Plan = FftPlan<2048, 16, 16, 8>; static constexpr int T = 128, RW = 2; };
// A third plan on the large sides: the alternative plan's radices in the other
// order (small radix first), searched by the autotuner.
template <int N> struct RowCfgAlt2 : RowCfg<N> {};
template <> struct RowCfgAlt2<1024> { using Plan = FftPlan<1024, 4, 16, 16>; static constexpr int T = 64,  RW = 4; };
template <> struct RowCfgAlt2<2048> { using Plan = FftPlan<2048, 8, 16, 16>; static constexpr int T = 128, RW = 2; };
template <int N> constexpr int row_plan_count() { return (N == 1024 || N == 2048) ? 3 : 2; }

// Column sweeps: T lanes per column and W adjacent columns per workgroup
// (lane index = t * W + w, so the W columns of one row are one coalesced
// segment).  Two tile widths are compiled per side; the launcher picks one.
// The 1024-point transforms (the halves of 2048-point columns) come in 8 and
// 16 columns: 16 (147 KB of LDS, one 1024-lane workgroup per CU) covers whole
// 128-byte lines, which S11 turns into 6% more bandwidth (4.9 against
// 4.65 TB/s at 180 x 2048^2), while the chirp sweeps keep 8 (4.6 against 3.9:
// two workgroups per CU overlap one's loads with the other's transform).
// 4-column tiles (32-byte segments) were slower than 8 everywhere.
template <int N> struct ColCfg;
template <> struct ColCfg<128>  { using Plan = FftPlan<128, 16, 8>;      static constexpr int T = 8,   WA = 32, WB = 16; };
template <> struct ColCfg<256>  { using Plan = FftPlan<256, 16, 16>;     static constexpr int T = 16,  WA = 16, WB = 32; };
template <> struct ColCfg<512>  { using Plan = FftPlan<512, 16, 8, 4>;   static constexpr int T = 32,  WA = 16, WB = 8; };
template <> struct ColCfg<1024> { using Plan = FftPlan<1024, 16, 16, 4>; static constexpr int T = 64,  WA = 8,  WB = 16; };
template <> struct ColCfg<2048> { using Plan = FftPlan<2048, 16, 16, 8>; static constexpr int T = 128, WA = 4,  WB = 8; };

// Radix-2 split of the column transforms of the sweeps on sides of 512 and
// more.  A 2048-point column needs 16 KB of LDS, so a tile of 8 columns
// (64-byte row segments) would run alone on its CU, and 4-column tiles read
// 32-byte segments; at 1024 and 512 points the halves admit twice the tile
// width at the same LDS and registers (16 columns, 128-byte row segments, in
// place of 8 at 1024; 16 or 32 in place of 16 or 8 at 512: the column sweeps
// gain 4-9%).  The sweeps therefore take the first radix-2
// stage of the y transform out of the column sweeps (decimation in
// frequency):
//   forward: a[n] = x[n] + x[n + H],  b[n] = (x[n] - x[n + H]) w^n,  H = ny/2,
//            then X[2j] = FFT_H(a)[j] and X[2j + 1] = FFT_H(b)[j];
//   inverse: x[n] = A[n] + w^-n B[n],  x[n + H] = A[n] - w^-n B[n], with A, B
//            the inverse H-point transforms of the even and odd ky,
// w = exp(-2 pi i / ny).  Row sweeps handle rows n and n + H together and
// apply these butterflies as they read and write W; a column sweep's
// workgroup runs one H-point half (ky = 2 j + p for position j of half p).
// The spectra kept between iterations (Psi^, Z^, Y^) store half p's position
// j at row p H + j.
template <int NY> constexpr bool col_split() { return NY >= 512; }
constexpr bool col_split_n(int ny) { return ny >= 512; }

// Stored row of W, x and v for position j of half p of a split transform (row
// p ny/2 + j): the halves are interleaved in blocks of kSplitBlock rows, so
// that the two rows of a row sweep's pair lie kSplitBlock rows apart (the
// workgroups in flight read and write one region, not two ny/2 rows apart)
// while a column sweep still reads runs of kSplitBlock consecutive rows.
constexpr int kSplitBlock = 8;
__host__ __device__ constexpr int split_row(int j, int p) {
  return ((j & ~(kSplitBlock - 1)) << 1) + p * kSplitBlock + (j & (kSplitBlock - 1));
}
template <int NY> constexpr int col_fft_len() { return col_split<NY>() ? NY / 2 : NY; }
// Column configuration of the sweeps on side NY (transform length and tile widths).
template <int NY> using ColSweepCfg = ColCfg<col_fft_len<NY>()>;

// Arguments common to every sweep launch.
struct Sweep {
  const Inst* inst;       // device array of descriptors
  int32_t blocks_per_inst;
  int32_t iter;           // iteration index within this call
  const double* beta;     // momentum table (Algorithm S1), indexed by k0 + iter
  const float2* tw_row;   // twiddles of the row plan (forward, then reversed plan)
  const float2* tw_alt;   // twiddles of the alternative row plan (forward, then reversed plan)
  const float2* tw_alt2;  // twiddles of the third row plan (forward, then reversed plan)
  const float2* twn_row;  // w_nx^m, m = 0..nx-1
  const float2* twn_col;  // w_L^m, m = 0..L-1, L = the column sweeps' transform length
  const float2* tw_col;   // twiddles of the column plan (forward, then reversed plan)
  const float2* twn_pair; // w_ny^m, m = 0..ny-1: twiddles of the split's butterflies (row sweeps)
  int32_t pair_half;      // H = ny/2 when the column transform is split (col_split), else 0
  int32_t* status;        // bit 0: non-finite loss seen
  double corr_tol;        // stopping correlation threshold (used when corr_partial is set)
};

// One launch over several size classes: class c owns the logical blocks
// [first[c], first[c + 1]) and runs the sweep body of its side and plan (row
// sweeps) or side (column sweeps) with its own Sweep arguments.
constexpr int kMaxMerged = 4;
struct MultiSweep {
  Sweep s[kMaxMerged];
  int32_t first[kMaxMerged + 1];
  int32_t side[kMaxMerged];
  int32_t plan[kMaxMerged];
  int32_t nc;
};

// True when the instance has met the correlation stop: its sweeps are skipped.
__device__ __forceinline__ bool instance_stopped(const Inst& I) {
  return I.stop_iter != nullptr && *(volatile const int32_t*)I.stop_iter != 0;
}

}  // namespace pwf
