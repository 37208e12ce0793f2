// Host-side entry points of the PWF kernels (C++ linkage, internal to libpwf).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "pwf_device.h"

namespace pwf {

enum RowOp {
  ROW_PSI_UPDATE = 0,  // S0: psi = IFFT_x(W); store psi; x = exp(psi); FFT_x
  ROW_START,           // start of a forward pass from real-space psi_src
  ROW_MUL_T,           // S2
  ROW_MUL_CONJ_T,      // S8
  ROW_INTENSITY,       // S4
  ROW_BACKBLUR,        // S6 (+ final loss sum)
  ROW_GRAD,            // S10
  ROW_FORWARD_OUT,     // f = Re IFFT_x(W)
  ROW_REAL_FFT,        // W = FFT_x(y)
  ROW_CPLX_FFT,        // W = FFT_x(psi_src) (psi_src null: zeros)
  ROW_IFFT_OUT,        // out = IFFT_x(W)
  ROW_PSI_UPDATE_CORR, // S0 with the stopping rule's sums (runs with the plan of ROW_PSI_UPDATE)
};

// Row sweeps of the iteration (S0, S2, S4, S6, S8, S10) are compiled with every
// plan of their side (two, three at 1024 and 2048) and the plan is chosen at
// run time (pwf_set_row_plan, pwf_autotune).  Default (what the autotuner picks on the 180 x 1024^2
// workload): the alternative plan (RowCfgAlt) for every tunable sweep at 1024,
// for the update, intensity and gradient sweeps at 2048, for the update sweep
// elsewhere.  Other row sweeps always use RowCfg.
constexpr bool row_plan_tunable(int op) {
  return op == ROW_PSI_UPDATE || op == ROW_MUL_T || op == ROW_INTENSITY || op == ROW_BACKBLUR ||
         op == ROW_MUL_CONJ_T || op == ROW_GRAD;
}
template <int N> constexpr bool row_alt_default(int op) {
  return op == ROW_PSI_UPDATE || (N == 1024 && row_plan_tunable(op)) ||
         (N == 2048 && (op == ROW_GRAD || op == ROW_INTENSITY));
}

enum ColOp {
  COL_CHIRP1 = 0,      // S1
  COL_CHIRP2,          // S3
  COL_CHIRP2_CONJ,     // S7
  COL_CHIRP1_CONJ,     // S9
  COL_BLUR_LOSS,       // S5
  COL_BLUR,            // forward-only source blur
  COL_NESTEROV,        // S11
  COL_DIRECTION,       // spectrum of the update direction d
  COL_SPEC_YHAT,       // y_hat = FFT_y(W)
  COL_SPEC_PSIHAT,     // psi_hat = FFT_y(W); z_hat = psi_hat
};

// Sweeps on the real intensity path work on x-spectra in half form: the
// spectra of real rows are Hermitian, so a row keeps kx = 1 .. nx/2 - 1 at
// position kx and packs the two real values at kx = 0 and kx = nx/2 into
// position 0.  S4 scales the kx = nx/2 value by the IOTF's x factor there, so
// that the blur sweeps apply only the y factors to the packed column (the x
// factor at kx = 0 is 1); the residual sweep applies the IOTF a second time,
// and the back-blur row sweep multiplies the kx = nx/2 value by that x factor
// once more.  A row keeps its place (pitch nx, the first nx/2 values used), so
// each row sweep still rewrites only the row it read.
constexpr bool col_op_half(int op) { return op == COL_BLUR_LOSS || op == COL_BLUR || op == COL_SPEC_YHAT; }

enum PlainWindow {
  PLAIN_W_Q1 = 0, PLAIN_W_Q2, PLAIN_W_Q2C, PLAIN_W_Q1C, PLAIN_W_IOTF, PLAIN_W_PINV, PLAIN_W_GAMMA2,
  PLAIN_W_WIENER  // IOTF / (IOTF^2 + wiener_eps)
};

enum PlainOp {
  PLAIN_EXP = 0, PLAIN_MUL_T, PLAIN_MUL_CONJ_T, PLAIN_ABS2, PLAIN_REAL, PLAIN_NEG_ERR, PLAIN_MUL,
  PLAIN_GRAD, PLAIN_IMAG, PLAIN_DIRECTION, PLAIN_NESTEROV,
  PLAIN_FROM_REAL,  // out = (y, 0) from the descriptor's real image
  PLAIN_SQRT_POS    // out = (sqrt(max(Re a, 0)), 0)
};

bool row_alt_default_n(int n, int op);
int row_plan_count_n(int n);
int row_rows_per_block(int n, int plan);
int col_default_width(int n);
int col_alt_width(int n);
bool col_width_supported(int n, int w);
hipError_t launch_row(int nx, int op, int plan, int nblocks, const Sweep& S, hipStream_t st);
hipError_t launch_col(int ny, int width, int op, int nblocks, const Sweep& S, hipStream_t st);
hipError_t launch_build_tables(const Inst* insts, int n, hipStream_t st);

// Merged launches over size classes (pwf_sweeps_multi.hip).  A class can join a
// merged row sweep when multi_row_supported(nx, ny, plan) and a merged column sweep
// when multi_col_width(ny) > 0 (the tile width the merged kernel uses); ops are
// the twelve sweeps of the iteration.
bool multi_row_supported(int nx, int ny, int plan);
int multi_col_width(int ny);
hipError_t launch_row_multi(int op, int nblocks, const MultiSweep& M, hipStream_t st);
hipError_t launch_col_multi(int op, int nblocks, const MultiSweep& M, hipStream_t st);

hipError_t launch_plain_rows(int nx, int dir, const float2* src, float2* dst, int ny, const float2* tw,
                             hipStream_t st);
// In-place column FFTs of `planes` [ny][nx] planes plane_stride elements apart.
hipError_t launch_plain_cols(int ny, int dir, float2* a, int nx, const float2* tw, hipStream_t st, int planes = 1,
                             size_t plane_stride = 0);
hipError_t launch_plain_window(float2* a, const Inst* inst, int which, size_t m, hipStream_t st);
int plain_elementwise_blocks();
hipError_t launch_plain_elementwise(int op, size_t m, const float2* a, const float2* b, float2* c, float2* out,
                                    const Inst* inst, const double* beta, int iter, double* partial,
                                    hipStream_t st);
hipError_t launch_plain_loss_final(const double* partial, int np, double* dst, int iter, int32_t* status,
                                   hipStream_t st);

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);
// loss_dst[0] = inv_m * sum of the instance's loss partials, per instance (one workgroup each)
hipError_t launch_loss_final(const Inst* insts, int n, int32_t* status, hipStream_t st);
// Filtered back-projection (pwf_tomo.hip)
hipError_t launch_fbp_pad(const float2* const* psi, int n_proj, int nx, int ny, int n_pad, float2* dst,
                          hipStream_t st);
hipError_t launch_fbp_ramp(float2* a, const float* h, int n_pad, size_t rows, hipStream_t st);
hipError_t launch_fbp_backproject(const float2* q, int n_proj, int nx, int ny, int n_pad, const float2* cs, int n_out,
                                  float scale, float2* vol, hipStream_t st);
// Fourier shell correlation (pwf_tomo.hip): out[s], out[nsh + s], out[2 nsh + s]
// = shell sums of Re(G1* G2), |G1|^2, |G2|^2, nsh = n/2 + 1.
int fsc_blocks();
// (partial: 2 fsc_blocks() doubles of scratch; scale: 2 floats of device memory)
hipError_t launch_fsc_pack(const float2* g1, const float2* g2, int part, float2* dst, size_t m, double* partial,
                           float* scale, hipStream_t st);
hipError_t launch_fsc_shells(const float2* spec, int n, int dims, double* partial, double* out, hipStream_t st);
// Quadratic background removal (pwf_tomo.hip): n a multiple of 16; slices are
// split into bands of bg_rows_per_band(n) rows (n a multiple of that).
// partial: n_slices * (n / rows) * 12 doubles; minv: the inverse 6 x 6 normal
// matrix (row-major); coef: n_slices * 12 doubles.
int bg_rows_per_band(int n);
hipError_t launch_bg_moments(const float2* vol, int n_slices, int n, double r_bg, double* partial, hipStream_t st);
hipError_t launch_bg_subtract(float2* vol, int n_slices, int n, const double* partial, const double* minv,
                              double* coef, hipStream_t st);
// Calibration: FP64 partial sums, per workgroup, of sum I, sum I(x,y) I(x+d,y)
// and sum I(x,y) I(x,y+d) for d = 0..max_shift (circular shifts), then their
// ordered total -> out[0] = sum I, out[1 + d] = x-shift sum, out[2 + kMaxShift + d]
// = y-shift sum (entries past max_shift are 0).  max_shift <= kMaxShift.
constexpr int kMaxShift = 32;
int speckle_sum_blocks();
hipError_t launch_speckle_sums(const float* img, int nx, int ny, int max_shift, double* partial, double* out,
                               hipStream_t st);
// Joint diffuser step (see joint_update_kernel): normalisation from the S2
// maxima (u1max is overwritten), then t <- t - eta_t sum_j G_j / sum_j max|u1_j|^2.
hipError_t launch_joint_update(float* u1max, int n, int count, size_t max_stride, const float2* g,
                               size_t field_stride, size_t m, float2* t, double eta_t, double* dsum,
                               hipStream_t st);
int maxabs2_blocks();
hipError_t launch_maxabs2(const float2* t, size_t m, float* partial, float* out, hipStream_t st);
// max |t|^2 of B.n <= kMaxabs2Batch diffusers in two launches; partial holds
// maxabs2_blocks() floats per diffuser (diffuser d at d * maxabs2_blocks()).
constexpr int kMaxabs2Batch = 32;
struct Maxabs2Batch {
  const float2* t[kMaxabs2Batch];
  size_t m[kMaxabs2Batch];
  float* out[kMaxabs2Batch];
  int32_t n;
};
hipError_t launch_maxabs2_batch(const Maxabs2Batch& B, float* partial, hipStream_t st);

// Number of float2 twiddles of the N-point row (which = 0), column (1),
// alternative row (2) or third row (3) plan, forward and reversed; fills
// `out` when it is not null.  Returns -1 for unsupported N.
int plan_twiddles(int n, int which, float2* out);

}  // namespace pwf
