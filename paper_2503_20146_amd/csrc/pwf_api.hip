// C ABI of libpwf: argument validation, workspace layout, launch sequences of
// the fused path (Algorithm S1 as twelve sweeps per iteration), the plain
// reference path, and hipGraph capture of the solve loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/pwf.h"
#include "pwf_device.h"
#include "pwf_kernels.h"

using pwf::Inst;
using pwf::Sweep;

namespace {

constexpr int kVersion = 10301;        // 1.3.1
constexpr int kBetaCap = 1 << 16;      // iterations covered by the momentum table
constexpr size_t kAlign = 256;
constexpr int kSizes[] = {128, 256, 512, 1024, 2048};
constexpr int kMaxDevices = 64;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool supported_side(int n) {
  for (int s : kSizes)
    if (s == n) return true;
  return false;
}
int size_index(int n) {
  for (int i = 0; i < 5; ++i)
    if (kSizes[i] == n) return i;
  return -1;
}

// ------------------------------------------------------------------ device context

struct GraphKey {
  void* ws;
  int n;
  int iters;
  std::vector<int> dims;
  bool operator<(const GraphKey& o) const {
    return std::tie(ws, n, iters, dims) < std::tie(o.ws, o.n, o.iters, o.dims);
  }
};

struct Context {
  bool ready = false;
  float2* tw[5] = {};          // row-plan twiddle tables per supported side
  float2* twc[5] = {};         // column-plan twiddle tables per supported side
  float2* twa[5] = {};         // alternative row-plan twiddle tables per supported side
  float2* twa2[5] = {};        // third row-plan twiddle tables per supported side
  float2* twn[5] = {};         // w_N^m, m = 0..N-1, per supported side
  double* beta = nullptr;      // momentum table
  hipStream_t side = nullptr;  // internal stream for graph launches
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // streams that run the size classes of an uneven batch side by side
  static constexpr int kForks = 3;
  hipStream_t fork[kForks] = {};
  hipEvent_t fork_ev[kForks + 1] = {};
  std::map<GraphKey, hipGraphExec_t> graphs;
  // pinned staging for descriptor uploads (ring of slots)
  static constexpr int kSlots = 4;
  void* stage[kSlots] = {};
  size_t stage_bytes[kSlots] = {};
  hipEvent_t stage_ev[kSlots] = {};
  int next_slot = 0;
};

// Column-tile width per supported side and column sweep op (0: compiled
// default); set by pwf_set_column_tile or pwf_autotune.
int g_col_width[5][16] = {};

int col_width(int n, int op) {
  const int i = size_index(n);
  if (i < 0 || op < 0 || op >= 16) return 0;
  return g_col_width[i][op] ? g_col_width[i][op] : pwf::col_default_width(n);
}

// Column op of iteration sweep S1, S3, ..., S11 (-1 for other indices).
int col_op_of_sweep(int sweep) {
  switch (sweep) {
    case 1: return pwf::COL_CHIRP1;
    case 3: return pwf::COL_CHIRP2;
    case 5: return pwf::COL_BLUR_LOSS;
    case 7: return pwf::COL_CHIRP2_CONJ;
    case 9: return pwf::COL_CHIRP1_CONJ;
    case 11: return pwf::COL_NESTEROV;
    default: return -1;
  }
}

// Row plan per side and row sweep: -1 = default, 0 = RowCfg, 1 = RowCfgAlt,
// 2 = RowCfgAlt2 (sides with three plans).  Set by pwf_set_row_plan or pwf_autotune.
int g_row_plan[5][16];
struct RowPlanInit {
  RowPlanInit() {
    for (auto& r : g_row_plan)
      for (int& v : r) v = -1;
  }
} g_row_plan_init;

int row_plan(int n, int op) {
  const int i = size_index(n);
  if (i < 0 || !pwf::row_plan_tunable(op) || g_row_plan[i][op] < 0) return pwf::row_alt_default_n(n, op) ? 1 : 0;
  return g_row_plan[i][op];
}

// Row op of iteration sweep S0, S2, ..., S10 (-1 for other indices).
int row_op_of_sweep(int sweep) {
  switch (sweep) {
    case 0: return pwf::ROW_PSI_UPDATE;
    case 2: return pwf::ROW_MUL_T;
    case 4: return pwf::ROW_INTENSITY;
    case 6: return pwf::ROW_BACKBLUR;
    case 8: return pwf::ROW_MUL_CONJ_T;
    case 10: return pwf::ROW_GRAD;
    default: return -1;
  }
}

// Bumped by every change of a tuning setting; part of the graph cache key, so
// that a cached graph never mixes launch shapes with descriptors computed
// under other settings.
int g_tune_gen = 0;

std::mutex g_mu;
Context g_ctx[kMaxDevices];
bool g_graph_mode = true;
// Uneven batches: one launch per sweep over all size classes (1) or one launch
// per class on parallel streams (0, default: the merged kernels carry the
// register pressure of all their bodies and measured slower).
int g_merge_mode = 0;

pwf_status hip_fail(hipError_t e) { return e == hipSuccess ? PWF_OK : PWF_ERR_HIP; }
#define PWF_HIP(call)                              \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return PWF_ERR_HIP;      \
  } while (0)

// Immutable tables of a device, built on the host in FP64 and rounded: the
// twiddles of every row, column and alternative-row plan and w_N^m of every
// supported side, and the momentum table.  `emit` receives each table and
// returns where it will live on the device.
struct HostTables {
  std::vector<float2> plan[5][4];  // which = 0 row, 1 column, 2 alternative row, 3 third row
  std::vector<float2> twn[5];
  std::vector<double> beta;
};

const HostTables& host_tables() {
  static const HostTables T = [] {
    HostTables h;
    for (int i = 0; i < 5; ++i) {
      for (int which = 0; which < 4; ++which) {
        const int cnt = pwf::plan_twiddles(kSizes[i], which, nullptr);
        h.plan[i][which].assign(std::max(cnt, 1), make_float2(0.f, 0.f));
        pwf::plan_twiddles(kSizes[i], which, h.plan[i][which].data());
      }
      const int n = kSizes[i];
      h.twn[i].resize(n);
      for (int m = 0; m < n; ++m) {
        const double ang = -2.0 * M_PI * (double)m / (double)n;
        h.twn[i][m] = make_float2((float)std::cos(ang), (float)std::sin(ang));
      }
    }
    // beta_k = (tau_k - 1) / tau_{k+1}, tau_0 = 1, tau_{k+1} = (1 + sqrt(1 + 4 tau_k^2)) / 2
    h.beta.resize(kBetaCap);
    double tau = 1.0;
    for (int k = 0; k < kBetaCap; ++k) {
      const double nt = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tau * tau));
      h.beta[k] = (tau - 1.0) / nt;
      tau = nt;
    }
    return h;
  }();
  return T;
}

#define PWF_TRY(x)                      \
  do {                                  \
    const pwf_status s_ = (x);          \
    if (s_ != PWF_OK) return s_;        \
  } while (0)

pwf_status context_for_current(Context** out) {
  int dev = 0;
  PWF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return PWF_ERR_HIP;
  Context& c = g_ctx[dev];
  if (!c.ready) {
    const HostTables& h = host_tables();
    auto put = [](const auto& host, auto** dst) -> pwf_status {
      const size_t bytes = sizeof(host[0]) * host.size();
      PWF_HIP(hipMalloc((void**)dst, bytes));
      PWF_HIP(hipMemcpy(*dst, host.data(), bytes, hipMemcpyHostToDevice));
      return PWF_OK;
    };
    for (int i = 0; i < 5; ++i) {
      PWF_TRY(put(h.plan[i][0], &c.tw[i]));
      PWF_TRY(put(h.plan[i][1], &c.twc[i]));
      PWF_TRY(put(h.plan[i][2], &c.twa[i]));
      PWF_TRY(put(h.plan[i][3], &c.twa2[i]));
      PWF_TRY(put(h.twn[i], &c.twn[i]));
    }
    PWF_TRY(put(h.beta, &c.beta));
    PWF_HIP(hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking));
    PWF_HIP(hipEventCreateWithFlags(&c.ev_in, hipEventDisableTiming));
    PWF_HIP(hipEventCreateWithFlags(&c.ev_out, hipEventDisableTiming));
    for (int i = 0; i < Context::kForks; ++i) PWF_HIP(hipStreamCreateWithFlags(&c.fork[i], hipStreamNonBlocking));
    for (int i = 0; i <= Context::kForks; ++i) PWF_HIP(hipEventCreateWithFlags(&c.fork_ev[i], hipEventDisableTiming));
    for (int i = 0; i < Context::kSlots; ++i) PWF_HIP(hipEventCreateWithFlags(&c.stage_ev[i], hipEventDisableTiming));
    c.ready = true;
  }
  *out = &c;
  return PWF_OK;
}

// Copy descriptors to the workspace through a pinned staging slot.
pwf_status upload(Context& c, const void* src, size_t bytes, void* dst, hipStream_t st) {
  const int slot = c.next_slot;
  c.next_slot = (c.next_slot + 1) % Context::kSlots;
  PWF_HIP(hipEventSynchronize(c.stage_ev[slot]));
  if (c.stage_bytes[slot] < bytes) {
    if (c.stage[slot]) PWF_HIP(hipHostFree(c.stage[slot]));
    c.stage[slot] = nullptr;
    c.stage_bytes[slot] = 0;
    PWF_HIP(hipHostMalloc(&c.stage[slot], bytes));
    c.stage_bytes[slot] = bytes;
  }
  std::memcpy(c.stage[slot], src, bytes);
  PWF_HIP(hipMemcpyAsync(dst, c.stage[slot], bytes, hipMemcpyHostToDevice, st));
  PWF_HIP(hipEventRecord(c.stage_ev[slot], st));
  return PWF_OK;
}

// ------------------------------------------------------------------ validation

bool finite(double x) { return std::isfinite(x); }

pwf_status validate_problem(const pwf_problem& p) {
  const pwf_geometry& g = p.geom;
  if (!supported_side(g.nx) || !supported_side(g.ny)) return PWF_ERR_SIZE;
  if (!finite(g.pixel_m) || g.pixel_m <= 0 || !finite(g.wavelength_m) || g.wavelength_m <= 0) return PWF_ERR_ARG;
  if (!finite(g.z1_m) || !finite(g.z2_m) || g.z1_m < 0 || g.z2_m < 0) return PWF_ERR_ARG;
  // largest lambda^2 rho^2 on the grid is (lambda/p)^2 / 2 (corner bin)
  const double lp = g.wavelength_m / g.pixel_m;
  if (0.5 * lp * lp >= 1.0) return PWF_ERR_EVANESCENT;
  const pwf_source& s = p.source;
  switch (s.kind) {
    case PWF_SRC_GAUSS:
      if (!finite(s.sigma_x_px) || !finite(s.sigma_y_px) || s.sigma_x_px < 0 || s.sigma_y_px < 0) return PWF_ERR_ARG;
      break;
    case PWF_SRC_COHERENCE:
      if (!finite(s.x_coh_m) || !finite(s.y_coh_m) || s.x_coh_m < 0 || s.y_coh_m < 0) return PWF_ERR_ARG;
      break;
    case PWF_SRC_IOTF:
      if (!s.iotf_x || !s.iotf_y) return PWF_ERR_ARG;
      break;
    default:
      return PWF_ERR_ARG;
  }
  const pwf_params& q = p.params;
  if (!finite(q.eta) || !finite(q.alpha_re) || !finite(q.alpha_im) || !finite(q.gamma) || q.gamma < 0)
    return PWF_ERR_ARG;
  if (q.precondition && (!finite(q.precond_scale) || q.precond_scale <= 0)) return PWF_ERR_ARG;
  if (!p.diffuser) return PWF_ERR_ARG;
  return PWF_OK;
}

pwf_status validate_batch(const pwf_problem* probs, int32_t n) {
  if (!probs || n <= 0) return PWF_ERR_ARG;
  for (int i = 0; i < n; ++i) {
    const pwf_status st = validate_problem(probs[i]);
    if (st != PWF_OK) return st;
  }
  return PWF_OK;
}

// ------------------------------------------------------------------ workspace layout

size_t field_bytes(const pwf_problem& p) { return align_up((size_t)p.geom.nx * p.geom.ny * sizeof(float2)); }
// Workgroups of a column sweep per instance: one per tile of `width` columns
// (nx/2 columns in half form), times the two halves of a split transform.
int col_blocks(int nx, int ny, int op, int width) {
  return (pwf::col_op_half(op) ? nx / 2 : nx) / width * (pwf::col_split_n(ny) ? 2 : 1);
}
// loss partials: one per workgroup of the residual sweep
int n_partials(const pwf_problem& p) {
  return col_blocks(p.geom.nx, p.geom.ny, pwf::COL_BLUR_LOSS, col_width(p.geom.ny, pwf::COL_BLUR_LOSS));
}
// room for per-workgroup partials of a column sweep at the narrowest compiled tile
int max_partials(const pwf_problem& p) {
  const int narrow = std::min(pwf::col_default_width(p.geom.ny), pwf::col_alt_width(p.geom.ny));
  return col_blocks(p.geom.nx, p.geom.ny, pwf::COL_CHIRP1, narrow);
}
size_t table_bytes(const pwf_problem& p) {
  return align_up((size_t)(p.geom.nx + p.geom.ny) * (2 * sizeof(float2) + 2 * sizeof(float)));
}

struct Layout {
  size_t status = 0, maxt2 = 0, maxt2_part = 0, desc = 0, partials = 0;
  std::vector<size_t> W, psi_hat, z_hat, v, psi, y_hat, extra0, extra1, part, tables, corr;
  std::vector<size_t> u1;            // joint diffuser mode only
  size_t u1max = 0, dsum = 0;        // joint diffuser mode only
  size_t stop = 0;
  size_t total = 0;
};

// Region order keeps W, psi_hat and z_hat of all instances contiguous so that
// one fill kernel clears them.
Layout make_layout(const pwf_problem* probs, int n, bool joint = false) {
  Layout L;
  size_t off = 0;
  L.status = off;
  off += kAlign;
  L.maxt2 = off;
  off += align_up(sizeof(float) * n);
  L.maxt2_part = off;
  off += align_up(sizeof(float) * (size_t)pwf::maxabs2_blocks() * n);
  L.desc = off;
  off += align_up(sizeof(Inst) * n);
  L.part.resize(n);
  L.partials = off;
  for (int i = 0; i < n; ++i) {
    L.part[i] = off;
    // room for the loss partials at any compiled column tile and the plain path's partials
    off += align_up(sizeof(double) * std::max(max_partials(probs[i]), pwf::plain_elementwise_blocks()));
  }
  L.tables.resize(n);
  for (int i = 0; i < n; ++i) {
    L.tables[i] = off;
    off += table_bytes(probs[i]);
  }
  L.corr.resize(n);
  for (int i = 0; i < n; ++i) {
    L.corr[i] = off;
    off += align_up(sizeof(double) * 4 * (size_t)probs[i].geom.ny);
  }
  L.stop = off;
  off += align_up(sizeof(int32_t) * n);
  auto region = [&](std::vector<size_t>& r) {
    r.resize(n);
    for (int i = 0; i < n; ++i) {
      r[i] = off;
      off += field_bytes(probs[i]);
    }
  };
  region(L.W);
  region(L.psi_hat);
  region(L.z_hat);
  region(L.v);
  region(L.psi);
  region(L.y_hat);
  // two more fields for the first instance (the plain path's buffers)
  L.extra0.assign(1, off);
  off += field_bytes(probs[0]);
  L.extra1.assign(1, off);
  off += field_bytes(probs[0]);
  if (joint) {
    // u1 then conj(u1) a2 per instance (contiguous, one field apart), the S2
    // workgroup maxima (ny floats per instance) and the normalisation
    region(L.u1);
    L.u1max = off;
    off += align_up(sizeof(float) * (size_t)probs[0].geom.ny * n);
    L.dsum = off;
    off += kAlign;
  }
  L.total = off;
  return L;
}

// Layout of only the regions pwf_loss_grad uses (status, descriptors, loss
// partials, window tables and four fields per instance: W, v, x, y_hat), for
// the allocation-free variant whose buffer has a fixed size.
Layout make_loss_grad_layout(const pwf_problem* probs, int n) {
  Layout L;
  size_t off = 0;
  L.status = off;
  off += kAlign;
  L.maxt2 = off;
  off += align_up(sizeof(float) * n);
  L.desc = off;
  off += align_up(sizeof(Inst) * n);
  L.part.resize(n);
  L.partials = off;
  for (int i = 0; i < n; ++i) {
    L.part[i] = off;
    off += align_up(sizeof(double) * max_partials(probs[i]));
  }
  L.tables.resize(n);
  for (int i = 0; i < n; ++i) {
    L.tables[i] = off;
    off += table_bytes(probs[i]);
  }
  for (std::vector<size_t>* r : {&L.W, &L.v, &L.psi, &L.y_hat}) {
    r->resize(n);
    for (int i = 0; i < n; ++i) {
      (*r)[i] = off;
      off += field_bytes(probs[i]);
    }
  }
  L.total = off;
  return L;
}

// ------------------------------------------------------------------ descriptors

Inst base_inst(const pwf_problem& p) {
  Inst I;
  std::memset(&I, 0, sizeof(I));
  const pwf_geometry& g = p.geom;
  I.nx = g.nx;
  I.ny = g.ny;
  I.n_partials = n_partials(p);
  I.t = (const float2*)p.diffuser;
  const double p2 = g.pixel_m * g.pixel_m;
  I.chirp1_rev = g.z1_m * g.wavelength_m / (2.0 * p2);
  I.chirp2_rev = g.z2_m * g.wavelength_m / (2.0 * p2);
  I.s_coef = (g.wavelength_m / g.pixel_m) * (g.wavelength_m / g.pixel_m);
  I.series = (0.5 * I.s_coef < 1e-4) ? 1 : 0;
  {
    // cross term of the separable chirp at the corner bin (rho^2 = 1/2), its
    // largest value: applied only where it reaches a quarter ulp of 1 (2^-26)
    const double s_max = 0.5 * I.s_coef;
    const double a_max = 2.0 * M_PI * std::max(I.chirp1_rev, I.chirp2_rev);
    const double th_max = a_max * 0.5 * s_max * (0.25 + 0.125 * s_max);
    I.cross = th_max >= std::ldexp(1.0, -26) ? 1 : 0;
  }
  I.two_pi_a1 = (float)(2.0 * M_PI * I.chirp1_rev);
  I.two_pi_a2 = (float)(2.0 * M_PI * I.chirp2_rev);
  I.s_coef_f = (float)I.s_coef;
  // Coherence lengths in pixels: Eq. 4's Gaussian of std sigma has x_coh = 2 sqrt(pi) sigma p.
  // IOTF (Eq. 5) exp(-(pi/2) u^2 x_coh^2) and STF (Eq. 14) exp(-pi gamma u^2 x_coh^2), with
  // u = f / p for f in cycles per pixel.
  const pwf_source& src = p.source;
  double cx = 0.0, cy = 0.0;
  if (src.kind == PWF_SRC_GAUSS) {
    cx = 2.0 * std::sqrt(M_PI) * src.sigma_x_px;
    cy = 2.0 * std::sqrt(M_PI) * src.sigma_y_px;
  } else if (src.kind == PWF_SRC_COHERENCE) {
    cx = src.x_coh_m / g.pixel_m;
    cy = src.y_coh_m / g.pixel_m;
  } else {
    I.src_ix = src.iotf_x;
    I.src_iy = src.iotf_y;
  }
  I.iotf_cx = (float)(0.5 * M_PI * cx * cx);
  I.iotf_cy = (float)(0.5 * M_PI * cy * cy);
  I.stf_cx = (float)(M_PI * p.params.gamma * cx * cx);
  I.stf_cy = (float)(M_PI * p.params.gamma * cy * cy);
  I.two_gamma = (float)(2.0 * p.params.gamma);
  I.pinv_scale = p.params.precondition ? (float)p.params.precond_scale : -1.0f;
  I.alpha_c1 = (float)(0.5 * (p.params.alpha_re + p.params.alpha_im));
  I.alpha_c2 = (float)(0.5 * (p.params.alpha_re - p.params.alpha_im));
  I.eta = (float)p.params.eta;
  I.inv_m_d = 1.0 / ((double)g.nx * g.ny);
  I.inv_m = (float)I.inv_m_d;
  return I;
}

void attach_tables(Inst& I, char* ws, const Layout& L, int i) {
  char* b = ws + L.tables[i];
  const size_t nx = (size_t)I.nx, ny = (size_t)I.ny;
  I.qx1 = (float2*)b;
  I.qx2 = I.qx1 + nx;
  I.qy1 = I.qx2 + nx;
  I.qy2 = I.qy1 + ny;
  I.ix = (float*)(I.qy2 + ny);
  I.gx = I.ix + nx;
  I.iy = I.gx + nx;
  I.gy = I.iy + ny;
}

// Instances grouped by grid shape; each class is a contiguous run of the
// (reordered) descriptor table.
struct Class {
  int nx, ny, first, count;
};

struct Batch {
  std::vector<int> order;  // descriptor slot -> caller index
  std::vector<Class> classes;
};

Batch group(const pwf_problem* probs, int n) {
  Batch b;
  b.order.resize(n);
  for (int i = 0; i < n; ++i) b.order[i] = i;
  std::stable_sort(b.order.begin(), b.order.end(), [&](int a, int c) {
    return std::make_pair(probs[a].geom.ny, probs[a].geom.nx) < std::make_pair(probs[c].geom.ny, probs[c].geom.nx);
  });
  for (int s = 0; s < n;) {
    const pwf_problem& p = probs[b.order[s]];
    int e = s;
    while (e < n && probs[b.order[e]].geom.nx == p.geom.nx && probs[b.order[e]].geom.ny == p.geom.ny) ++e;
    b.classes.push_back({p.geom.nx, p.geom.ny, s, e - s});
    s = e;
  }
  return b;
}

// A batch of several grid shapes is launched one sweep at a time over all its
// classes (merged kernels) when merge mode is on, every side is one the merged
// kernels hold and there are at most kMaxMerged classes.  Each class keeps its
// own row plans and tile widths, so the results are those of per-class
// launches; a class whose plan or width the merged kernels do not hold gets a
// launch of its own in that sweep (the autotuner, tuning such a batch,
// chooses among the plans and widths the merged kernels hold).
bool batch_merged(const Batch& B) {
  if (!g_merge_mode || B.classes.size() <= 1 || (int)B.classes.size() > pwf::kMaxMerged) return false;
  for (const Class& c : B.classes)
    if (pwf::multi_col_width(c.nx) == 0 || pwf::multi_col_width(c.ny) == 0) return false;
  return true;
}

struct Launcher {
  Context& ctx;
  char* ws;
  const Layout& L;
  const Batch& B;
  hipStream_t st;
  double corr_tol = 0.0;
  bool merged = false;   // batch_merged(B): one launch per sweep over the classes
  int width_of(int ny, int op) const { return col_width(ny, op); }
  int plan_of(int nx, int op) const {
    return row_plan(nx, op == pwf::ROW_PSI_UPDATE_CORR ? (int)pwf::ROW_PSI_UPDATE : op);
  }
  Inst* dev_desc() const { return (Inst*)(ws + L.desc); }
  int32_t* status() const { return (int32_t*)(ws + L.status); }

  Sweep sweep(const Class& c, int iter) const {
    Sweep S;
    S.inst = dev_desc() + c.first;
    S.iter = iter;
    S.beta = ctx.beta;
    S.tw_row = ctx.tw[size_index(c.nx)];
    S.tw_alt = ctx.twa[size_index(c.nx)];
    S.tw_alt2 = ctx.twa2[size_index(c.nx)];
    S.twn_row = ctx.twn[size_index(c.nx)];
    // a split column transform runs ny/2-point transforms (pwf_device.h, col_split)
    const bool split = pwf::col_split_n(c.ny);
    const int nf = split ? c.ny / 2 : c.ny;
    S.twn_col = ctx.twn[size_index(nf)];
    S.tw_col = ctx.twc[size_index(nf)];
    S.twn_pair = ctx.twn[size_index(c.ny)];
    S.pair_half = split ? c.ny / 2 : 0;
    S.status = status();
    S.blocks_per_inst = 0;
    S.corr_tol = corr_tol;
    return S;
  }
  pwf_status row(int op, int iter = 0) const {
    for (const Class& c : B.classes) {
      Sweep S = sweep(c, iter);
      const int plan = plan_of(c.nx, op);
      S.blocks_per_inst = c.ny / pwf::row_rows_per_block(c.nx, plan);
      PWF_HIP(pwf::launch_row(c.nx, op, plan, S.blocks_per_inst * c.count, S, st));
    }
    return PWF_OK;
  }
  pwf_status col(int op, int iter = 0) const {
    for (const Class& c : B.classes) {
      Sweep S = sweep(c, iter);
      const int width = width_of(c.ny, op);
      S.blocks_per_inst = col_blocks(c.nx, c.ny, op, width);
      PWF_HIP(pwf::launch_col(c.ny, width, op, S.blocks_per_inst * c.count, S, st));
    }
    return PWF_OK;
  }
  // One launch over the classes whose row plan (tile width) the merged
  // kernels hold, and one launch per class for the others.
  pwf_status row_merged(int op, int iter) const {
    pwf::MultiSweep M;
    std::memset(&M, 0, sizeof(M));
    int total = 0, m = 0;
    for (const Class& c : B.classes) {
      const int plan = plan_of(c.nx, op);
      Sweep S = sweep(c, iter);
      S.blocks_per_inst = c.ny / pwf::row_rows_per_block(c.nx, plan);
      if (!pwf::multi_row_supported(c.nx, c.ny, plan) || m == pwf::kMaxMerged) {
        PWF_HIP(pwf::launch_row(c.nx, op, plan, S.blocks_per_inst * c.count, S, st));
        continue;
      }
      M.s[m] = S;
      M.first[m] = total;
      M.side[m] = c.nx;
      M.plan[m] = plan;
      total += S.blocks_per_inst * c.count;
      ++m;
    }
    if (m == 0) return PWF_OK;
    M.first[m] = total;
    M.nc = m;
    PWF_HIP(pwf::launch_row_multi(op, total, M, st));
    return PWF_OK;
  }
  pwf_status col_merged(int op, int iter) const {
    pwf::MultiSweep M;
    std::memset(&M, 0, sizeof(M));
    int total = 0, m = 0;
    for (const Class& c : B.classes) {
      const int width = width_of(c.ny, op);
      Sweep S = sweep(c, iter);
      S.blocks_per_inst = col_blocks(c.nx, c.ny, op, width);
      if (width != pwf::multi_col_width(c.ny) || m == pwf::kMaxMerged) {
        PWF_HIP(pwf::launch_col(c.ny, width, op, S.blocks_per_inst * c.count, S, st));
        continue;
      }
      M.s[m] = S;
      M.first[m] = total;
      M.side[m] = c.ny;
      total += S.blocks_per_inst * c.count;
      ++m;
    }
    if (m == 0) return PWF_OK;
    M.first[m] = total;
    M.nc = m;
    PWF_HIP(pwf::launch_col_multi(op, total, M, st));
    return PWF_OK;
  }
};

pwf_status check_ws(const pwf_problem* probs, int n, void* ws, size_t ws_bytes, Layout* out, bool joint = false) {
  if (!ws || ((uintptr_t)ws % kAlign) != 0) return PWF_ERR_WORKSPACE;
  *out = make_layout(probs, n, joint);
  if (ws_bytes < out->total) return PWF_ERR_WORKSPACE;
  return PWF_OK;
}

// max|t|^2 for every distinct diffuser; sets inst.maxt2.
// (the distinct diffusers in launches of up to kMaxabs2Batch: a batch of
// distinct ROIs would otherwise queue two small launches per instance)
pwf_status launch_maxt2(const pwf_problem* probs, int n, const Batch& B, std::vector<Inst>& desc, char* ws,
                        const Layout& L, hipStream_t st) {
  std::vector<const void*> seen;
  pwf::Maxabs2Batch mb;
  std::memset(&mb, 0, sizeof(mb));
  int first = 0;  // slot of mb's first entry
  auto flush = [&]() -> pwf_status {
    if (mb.n == 0) return PWF_OK;
    float* part = (float*)(ws + L.maxt2_part) + (size_t)first * pwf::maxabs2_blocks();
    PWF_HIP(pwf::launch_maxabs2_batch(mb, part, st));
    first += mb.n;
    mb.n = 0;
    return PWF_OK;
  };
  for (int s = 0; s < n; ++s) {
    const pwf_problem& p = probs[B.order[s]];
    int slot = -1;
    for (size_t j = 0; j < seen.size(); ++j)
      if (seen[j] == p.diffuser) slot = (int)j;
    if (slot < 0) {
      slot = (int)seen.size();
      seen.push_back(p.diffuser);
      if (mb.n == pwf::kMaxabs2Batch) PWF_TRY(flush());
      mb.t[mb.n] = (const float2*)p.diffuser;
      mb.m[mb.n] = (size_t)p.geom.nx * p.geom.ny;
      mb.out[mb.n] = (float*)(ws + L.maxt2) + slot;
      ++mb.n;
    }
    desc[s].maxt2 = (const float*)(ws + L.maxt2) + slot;
  }
  return flush();
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

const char* pwf_status_string(int32_t s) {
  switch (s) {
    case PWF_OK: return "ok";
    case PWF_ERR_ARG: return "invalid argument";
    case PWF_ERR_SIZE: return "unsupported grid size (nx, ny must be 128, 256, 512, 1024 or 2048)";
    case PWF_ERR_EVANESCENT: return "geometry has evanescent frequency bins (lambda/p >= sqrt(2))";
    case PWF_ERR_WORKSPACE: return "workspace missing, misaligned (256 B) or too small";
    case PWF_ERR_HIP: return "HIP runtime error";
    case PWF_ERR_NONFINITE: return "non-finite loss (NaN or Inf) on the GPU";
    case PWF_ERR_SCRATCH: return "batch does not fit the static scratch buffer of pwf_loss_grad_noalloc (64 MiB, 64 instances)";
    default: return "unknown status";
  }
}

int32_t pwf_version(void) { return kVersion; }

size_t pwf_workspace_size(const pwf_problem* problems, int32_t n) {
  if (validate_batch(problems, n) != PWF_OK) return 0;
  return make_layout(problems, n).total;
}

void pwf_set_graph_mode(int32_t on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_graph_mode = on != 0;
}

void pwf_set_merged_launch(int32_t on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_merge_mode = on != 0 ? 1 : 0;
  ++g_tune_gen;   // cached graphs hold the other launch structure
}

}  // extern "C"

namespace {
// PhysicalModel (Eq. 1) for every instance; with y and ref_mean the output is
// the RMSE image 100 |y - f| / ref_mean instead of f.
pwf_status forward_impl(const pwf_problem* problems, int32_t n, const void* const* psi, float* const* f_out,
                        const float* const* y, const double* ref_mean, void* workspace, size_t workspace_bytes,
                        void* stream) {
  PWF_TRY(validate_batch(problems, n));
  if (!psi || !f_out) return PWF_ERR_ARG;
  for (int i = 0; i < n; ++i) {
    if (!psi[i] || !f_out[i]) return PWF_ERR_ARG;
    if (y && (!y[i] || !(ref_mean[i] > 0.0) || !std::isfinite(ref_mean[i]))) return PWF_ERR_ARG;
  }
  Layout L;
  PWF_TRY(check_ws(problems, n, workspace, workspace_bytes, &L));
  std::lock_guard<std::mutex> lk(g_mu);
  Context* ctx;
  PWF_TRY(context_for_current(&ctx));
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const Batch B = group(problems, n);
  std::vector<Inst> desc(n);
  for (int s = 0; s < n; ++s) {
    const int i = B.order[s];
    Inst& I = desc[s];
    I = base_inst(problems[i]);
    attach_tables(I, ws, L, i);
    I.W = (float2*)(ws + L.W[i]);
    I.psi_src = (const float2*)psi[i];
    I.f_out = f_out[i];
    I.loss_partial = (double*)(ws + L.part[i]);
    if (y) {
      I.y = y[i];
      I.rmse_scale = (float)(100.0 / ref_mean[i]);
    }
  }
  PWF_TRY(upload(*ctx, desc.data(), sizeof(Inst) * n, ws + L.desc, st));
  PWF_HIP(pwf::launch_build_tables((const Inst*)(ws + L.desc), n, st));
  const Launcher K{*ctx, ws, L, B, st};
  PWF_TRY(K.row(pwf::ROW_START));
  PWF_TRY(K.col(pwf::COL_CHIRP1));
  PWF_TRY(K.row(pwf::ROW_MUL_T));
  PWF_TRY(K.col(pwf::COL_CHIRP2));
  PWF_TRY(K.row(pwf::ROW_INTENSITY));
  PWF_TRY(K.col(pwf::COL_BLUR));
  PWF_TRY(K.row(pwf::ROW_FORWARD_OUT));
  return PWF_OK;
}

// pwf_loss_grad (and its allocation-free variant): argument checks, the
// descriptors at the regions of a layout, and the launch sequence.
pwf_status validate_loss_grad(const pwf_problem* problems, int32_t n, const void* const* psi, const float* const* y,
                              void* const* grad_out) {
  PWF_TRY(validate_batch(problems, n));
  if (!psi || !y || !grad_out) return PWF_ERR_ARG;
  for (int i = 0; i < n; ++i)
    if (!psi[i] || !y[i] || !grad_out[i]) return PWF_ERR_ARG;
  return PWF_OK;
}

void loss_grad_descriptors(const pwf_problem* problems, int32_t n, const Batch& B, const void* const* psi,
                           const float* const* y, void* const* grad_out, double* loss_out, char* ws,
                           const Layout& L, Inst* desc) {
  for (int s = 0; s < n; ++s) {
    const int i = B.order[s];
    Inst& I = desc[s];
    I = base_inst(problems[i]);
    attach_tables(I, ws, L, i);
    I.W = (float2*)(ws + L.W[i]);
    I.v = (float2*)(ws + L.v[i]);
    I.x = (float2*)(ws + L.psi[i]);
    I.psi_src = (const float2*)psi[i];
    I.y_hat = (float2*)(ws + L.y_hat[i]);
    I.y = y[i];
    I.g_out = (float2*)grad_out[i];
    I.grad_mul = 4.0f;  // dL/dRe psi + i dL/dIm psi = 4 x* P1+(t* P2+(v Filter(-e)))
    I.maxt2 = (const float*)(ws + L.maxt2);
    I.loss_partial = (double*)(ws + L.part[i]);
    I.loss_dst = loss_out ? loss_out + i : nullptr;
  }
}

// After the descriptors are in place: window tables, spectrum of y, forward
// model, loss and the back-propagated gradient.
pwf_status loss_grad_sequence(const Launcher& K, int32_t n) {
  PWF_HIP(pwf::launch_build_tables((const Inst*)(K.ws + K.L.desc), n, K.st));
  PWF_TRY(K.row(pwf::ROW_REAL_FFT));
  PWF_TRY(K.col(pwf::COL_SPEC_YHAT));
  PWF_TRY(K.row(pwf::ROW_START));
  PWF_TRY(K.col(pwf::COL_CHIRP1));
  PWF_TRY(K.row(pwf::ROW_MUL_T));
  PWF_TRY(K.col(pwf::COL_CHIRP2));
  PWF_TRY(K.row(pwf::ROW_INTENSITY));
  PWF_TRY(K.col(pwf::COL_BLUR_LOSS));
  PWF_TRY(K.row(pwf::ROW_BACKBLUR));
  PWF_TRY(K.col(pwf::COL_CHIRP2_CONJ));
  PWF_TRY(K.row(pwf::ROW_MUL_CONJ_T));
  PWF_TRY(K.col(pwf::COL_CHIRP1_CONJ));
  PWF_TRY(K.row(pwf::ROW_GRAD));
  return PWF_OK;
}
}  // namespace

extern "C" {

pwf_status pwf_forward(const pwf_problem* problems, int32_t n, const void* const* psi, float* const* f_out,
                       void* workspace, size_t workspace_bytes, void* stream) {
  return forward_impl(problems, n, psi, f_out, nullptr, nullptr, workspace, workspace_bytes, stream);
}

pwf_status pwf_rmse_image(const pwf_problem* problems, int32_t n, const void* const* psi, const float* const* y,
                          const double* ref_mean, float* const* out, void* workspace, size_t workspace_bytes,
                          void* stream) {
  if (!y || !ref_mean) return PWF_ERR_ARG;
  return forward_impl(problems, n, psi, out, y, ref_mean, workspace, workspace_bytes, stream);
}

pwf_status pwf_gradient(const pwf_problem* problems, int32_t n, const void* const* psi, const float* const* y,
                        void* const* g_out, void* const* d_out, double* loss_out, void* workspace,
                        size_t workspace_bytes, void* stream) {
  PWF_TRY(validate_batch(problems, n));
  if (!psi || !y) return PWF_ERR_ARG;
  bool want_d = false, want_g = false;
  for (int i = 0; i < n; ++i) {
    if (!psi[i] || !y[i]) return PWF_ERR_ARG;
    if (d_out && d_out[i]) want_d = true;
    if (g_out && g_out[i]) want_g = true;
  }
  Layout L;
  PWF_TRY(check_ws(problems, n, workspace, workspace_bytes, &L));
  std::lock_guard<std::mutex> lk(g_mu);
  Context* ctx;
  PWF_TRY(context_for_current(&ctx));
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const Batch B = group(problems, n);
  std::vector<Inst> desc(n);
  for (int s = 0; s < n; ++s) {
    const int i = B.order[s];
    Inst& I = desc[s];
    I = base_inst(problems[i]);
    attach_tables(I, ws, L, i);
    I.W = (float2*)(ws + L.W[i]);
    I.v = (float2*)(ws + L.v[i]);
    I.x = (float2*)(ws + L.psi[i]);
    I.psi_src = (const float2*)psi[i];
    I.psi_hat = (float2*)(ws + L.psi_hat[i]);
    I.y_hat = (float2*)(ws + L.y_hat[i]);
    I.y = y[i];
    I.g_out = g_out ? (float2*)g_out[i] : nullptr;
    I.out = d_out ? (float2*)d_out[i] : nullptr;
    I.loss_partial = (double*)(ws + L.part[i]);
    I.loss_dst = loss_out ? loss_out + i : nullptr;
  }
  PWF_HIP(pwf::launch_fill_zero(ws + L.status, 16, st));
  PWF_TRY(launch_maxt2(problems, n, B, desc, ws, L, st));
  PWF_TRY(upload(*ctx, desc.data(), sizeof(Inst) * n, ws + L.desc, st));
  PWF_HIP(pwf::launch_build_tables((const Inst*)(ws + L.desc), n, st));
  const Launcher K{*ctx, ws, L, B, st};
  if (want_d) {
    // spectrum of psi for the regulariser (I.psi is null: nothing is copied)
    PWF_TRY(K.row(pwf::ROW_CPLX_FFT));
    PWF_TRY(K.col(pwf::COL_SPEC_PSIHAT));
  }
  PWF_TRY(K.row(pwf::ROW_REAL_FFT));
  PWF_TRY(K.col(pwf::COL_SPEC_YHAT));
  PWF_TRY(K.row(pwf::ROW_START));
  PWF_TRY(K.col(pwf::COL_CHIRP1));
  PWF_TRY(K.row(pwf::ROW_MUL_T));
  PWF_TRY(K.col(pwf::COL_CHIRP2));
  PWF_TRY(K.row(pwf::ROW_INTENSITY));
  PWF_TRY(K.col(pwf::COL_BLUR_LOSS));
  if (!want_g && !want_d) {
    // loss only: the forward half (Eq. 1) and the misfit (Eq. 2)
    PWF_HIP(pwf::launch_loss_final((const Inst*)(ws + L.desc), n, (int32_t*)(ws + L.status), st));
    return PWF_OK;
  }
  PWF_TRY(K.row(pwf::ROW_BACKBLUR));
  PWF_TRY(K.col(pwf::COL_CHIRP2_CONJ));
  PWF_TRY(K.row(pwf::ROW_MUL_CONJ_T));
  PWF_TRY(K.col(pwf::COL_CHIRP1_CONJ));
  PWF_TRY(K.row(pwf::ROW_GRAD));
  if (want_d) {
    PWF_TRY(K.col(pwf::COL_DIRECTION));
    PWF_TRY(K.row(pwf::ROW_IFFT_OUT));
  }
  return PWF_OK;
}

pwf_status pwf_loss_grad(const pwf_problem* problems, int32_t n, const void* const* psi, const float* const* y,
                         void* const* grad_out, double* loss_out, void* workspace, size_t workspace_bytes,
                         void* stream) {
  PWF_TRY(validate_loss_grad(problems, n, psi, y, grad_out));
  Layout L;
  PWF_TRY(check_ws(problems, n, workspace, workspace_bytes, &L));
  std::lock_guard<std::mutex> lk(g_mu);
  Context* ctx;
  PWF_TRY(context_for_current(&ctx));
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const Batch B = group(problems, n);
  std::vector<Inst> desc(n);
  loss_grad_descriptors(problems, n, B, psi, y, grad_out, loss_out, ws, L, desc.data());
  PWF_HIP(pwf::launch_fill_zero(ws + L.status, 16, st));
  PWF_TRY(upload(*ctx, desc.data(), sizeof(Inst) * n, ws + L.desc, st));
  return loss_grad_sequence(Launcher{*ctx, ws, L, B, st}, n);
}

pwf_status pwf_state_init(const pwf_problem* problems, int32_t n, pwf_state* states, const void* const* psi0,
                          const float* const* y, void* workspace, size_t workspace_bytes, void* stream) {
  PWF_TRY(validate_batch(problems, n));
  if (!states || !y) return PWF_ERR_ARG;
  for (int i = 0; i < n; ++i)
    if (!y[i] || !states[i].psi || !states[i].psi_hat || !states[i].z_hat || !states[i].y_hat) return PWF_ERR_ARG;
  Layout L;
  PWF_TRY(check_ws(problems, n, workspace, workspace_bytes, &L));
  std::lock_guard<std::mutex> lk(g_mu);
  Context* ctx;
  PWF_TRY(context_for_current(&ctx));
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const Batch B = group(problems, n);
  std::vector<Inst> desc(n);
  for (int s = 0; s < n; ++s) {
    const int i = B.order[s];
    Inst& I = desc[s];
    I = base_inst(problems[i]);
    attach_tables(I, ws, L, i);
    I.W = (float2*)(ws + L.W[i]);
    I.y = y[i];
    I.y_hat = (float2*)states[i].y_hat;
    I.psi_src = psi0 ? (const float2*)psi0[i] : nullptr;
    I.psi = (float2*)states[i].psi;
    I.psi_hat = (float2*)states[i].psi_hat;
    I.z_hat = (float2*)states[i].z_hat;
    I.loss_partial = (double*)(ws + L.part[i]);
  }
  PWF_TRY(upload(*ctx, desc.data(), sizeof(Inst) * n, ws + L.desc, st));
  PWF_HIP(pwf::launch_build_tables((const Inst*)(ws + L.desc), n, st));
  const Launcher K{*ctx, ws, L, B, st};
  PWF_TRY(K.row(pwf::ROW_REAL_FFT));
  PWF_TRY(K.col(pwf::COL_SPEC_YHAT));
  PWF_TRY(K.row(pwf::ROW_CPLX_FFT));
  PWF_TRY(K.col(pwf::COL_SPEC_PSIHAT));
  for (int i = 0; i < n; ++i) states[i].k = 0;
  return PWF_OK;
}

pwf_status pwf_step(const pwf_problem* problems, int32_t n, pwf_state* states, double* loss_out, void* workspace,
                    size_t workspace_bytes, void* stream) {
  PWF_TRY(validate_batch(problems, n));
  if (!states) return PWF_ERR_ARG;
  for (int i = 0; i < n; ++i) {
    if (!states[i].psi || !states[i].psi_hat || !states[i].z_hat || !states[i].y_hat) return PWF_ERR_ARG;
    if (states[i].k < 0 || states[i].k >= kBetaCap) return PWF_ERR_ARG;
  }
  Layout L;
  PWF_TRY(check_ws(problems, n, workspace, workspace_bytes, &L));
  std::lock_guard<std::mutex> lk(g_mu);
  Context* ctx;
  PWF_TRY(context_for_current(&ctx));
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const Batch B = group(problems, n);
  std::vector<Inst> desc(n);
  for (int s = 0; s < n; ++s) {
    const int i = B.order[s];
    Inst& I = desc[s];
    I = base_inst(problems[i]);
    attach_tables(I, ws, L, i);
    I.k0 = states[i].k;
    I.W = (float2*)(ws + L.W[i]);
    I.v = (float2*)(ws + L.v[i]);
    I.x = (float2*)(ws + L.psi[i]);
    I.psi_src = (const float2*)states[i].psi;
    I.psi_hat = (float2*)states[i].psi_hat;
    I.z_hat = (float2*)states[i].z_hat;
    I.y_hat = (float2*)states[i].y_hat;
    I.out = (float2*)states[i].psi;
    I.loss_partial = (double*)(ws + L.part[i]);
    I.loss_dst = loss_out ? loss_out + i : nullptr;
  }
  PWF_HIP(pwf::launch_fill_zero(ws + L.status, 16, st));
  PWF_TRY(launch_maxt2(problems, n, B, desc, ws, L, st));
  PWF_TRY(upload(*ctx, desc.data(), sizeof(Inst) * n, ws + L.desc, st));
  PWF_HIP(pwf::launch_build_tables((const Inst*)(ws + L.desc), n, st));
  const Launcher K{*ctx, ws, L, B, st};
  PWF_TRY(K.row(pwf::ROW_START));
  PWF_TRY(K.col(pwf::COL_CHIRP1));
  PWF_TRY(K.row(pwf::ROW_MUL_T));
  PWF_TRY(K.col(pwf::COL_CHIRP2));
  PWF_TRY(K.row(pwf::ROW_INTENSITY));
  PWF_TRY(K.col(pwf::COL_BLUR_LOSS));
  PWF_TRY(K.row(pwf::ROW_BACKBLUR));
  PWF_TRY(K.col(pwf::COL_CHIRP2_CONJ));
  PWF_TRY(K.row(pwf::ROW_MUL_CONJ_T));
  PWF_TRY(K.col(pwf::COL_CHIRP1_CONJ));
  PWF_TRY(K.row(pwf::ROW_GRAD));
  PWF_TRY(K.col(pwf::COL_NESTEROV));
  PWF_TRY(K.row(pwf::ROW_IFFT_OUT));
  for (int i = 0; i < n; ++i) states[i].k += 1;
  return PWF_OK;
}

}  // extern "C"

namespace {

// The solve sequence after the descriptor upload: setup, iters x 12 sweeps,
// final inverse pass into psi_out.
// Joint diffuser refinement (Results, "Diffuser transmission function"):
// after every iteration, t <- t - eta_t sum_j conj(u1_j) a2_j / sum_j max|u1_j|^2
// over all instances (which share t), then max|t|^2 for the next gradient.
struct JointCfg {
  bool on = false;
  double eta_t = 0.0;
};

pwf_status joint_step(const Launcher& K, const pwf_problem* probs, int n, const JointCfg& jc) {
  const pwf_problem& p = probs[0];
  const size_t m = (size_t)p.geom.nx * p.geom.ny;
  const int count = p.geom.ny / pwf::row_rows_per_block(p.geom.nx, row_plan(p.geom.nx, pwf::ROW_MUL_T));
  float2* t = (float2*)p.diffuser;
  PWF_HIP(pwf::launch_joint_update((float*)(K.ws + K.L.u1max), n, count, (size_t)p.geom.ny,
                                   (const float2*)(K.ws + K.L.u1[0]), field_bytes(p) / sizeof(float2), m, t,
                                   jc.eta_t, (double*)(K.ws + K.L.dsum), K.st));
  PWF_HIP(pwf::launch_maxabs2(t, m, (float*)(K.ws + K.L.maxt2_part), (float*)(K.ws + K.L.maxt2), K.st));
  return PWF_OK;
}

pwf_status solve_sequence(const Launcher& K, const pwf_problem* probs, int n, std::vector<Inst>& desc, int iters,
                          const JointCfg& jc) {
  (void)desc;
  // spectrum of y (uses W as scratch), then clear the status word and W,
  // psi_hat, z_hat of every instance (contiguous regions): psi = z = 0
  PWF_TRY(K.row(pwf::ROW_REAL_FFT));
  PWF_TRY(K.col(pwf::COL_SPEC_YHAT));
  PWF_HIP(pwf::launch_fill_zero(K.ws + K.L.status, 16, K.st));
  PWF_HIP(pwf::launch_fill_zero(K.ws + K.L.W[0], K.L.v[0] - K.L.W[0], K.st));
  const int s0 = K.corr_tol > 0.0 ? pwf::ROW_PSI_UPDATE_CORR : pwf::ROW_PSI_UPDATE;
  auto iterate = [&](const Launcher& Q) -> pwf_status {
    for (int k = 0; k < iters; ++k) {
      PWF_TRY(Q.row(s0, k));
      PWF_TRY(Q.col(pwf::COL_CHIRP1, k));
      PWF_TRY(Q.row(pwf::ROW_MUL_T, k));
      PWF_TRY(Q.col(pwf::COL_CHIRP2, k));
      PWF_TRY(Q.row(pwf::ROW_INTENSITY, k));
      PWF_TRY(Q.col(pwf::COL_BLUR_LOSS, k));
      PWF_TRY(Q.row(pwf::ROW_BACKBLUR, k));
      PWF_TRY(Q.col(pwf::COL_CHIRP2_CONJ, k));
      PWF_TRY(Q.row(pwf::ROW_MUL_CONJ_T, k));
      PWF_TRY(Q.col(pwf::COL_CHIRP1_CONJ, k));
      PWF_TRY(Q.row(pwf::ROW_GRAD, k));
      PWF_TRY(Q.col(pwf::COL_NESTEROV, k));
      if (jc.on) PWF_TRY(joint_step(Q, probs, n, jc));
    }
    PWF_TRY(Q.row(pwf::ROW_IFFT_OUT, iters));
    return PWF_OK;
  };
  const int nc = (int)K.B.classes.size();
  if (nc <= 1 || jc.on) return iterate(K);
  if (K.merged) {
    // One launch per sweep over every size class (a sweep whose row plan or
    // tile width the merged kernels do not hold is launched per class).
    for (int k = 0; k < iters; ++k) {
      PWF_TRY(K.row_merged(s0, k));
      PWF_TRY(K.col_merged(pwf::COL_CHIRP1, k));
      PWF_TRY(K.row_merged(pwf::ROW_MUL_T, k));
      PWF_TRY(K.col_merged(pwf::COL_CHIRP2, k));
      PWF_TRY(K.row_merged(pwf::ROW_INTENSITY, k));
      PWF_TRY(K.col_merged(pwf::COL_BLUR_LOSS, k));
      PWF_TRY(K.row_merged(pwf::ROW_BACKBLUR, k));
      PWF_TRY(K.col_merged(pwf::COL_CHIRP2_CONJ, k));
      PWF_TRY(K.row_merged(pwf::ROW_MUL_CONJ_T, k));
      PWF_TRY(K.col_merged(pwf::COL_CHIRP1_CONJ, k));
      PWF_TRY(K.row_merged(pwf::ROW_GRAD, k));
      PWF_TRY(K.col_merged(pwf::COL_NESTEROV, k));
    }
    PWF_TRY(K.row(pwf::ROW_IFFT_OUT, iters));
    return PWF_OK;
  }
  // The size classes of an uneven batch are independent problems: their
  // iterations run on parallel streams (classes dealt round-robin), forked
  // from and joined back into K.st with events, so that a small class's short
  // launches overlap the large ones instead of alternating with them.
  const int ns = std::min(nc, Context::kForks + 1);
  std::vector<Batch> subs(ns);
  for (int c = 0; c < nc; ++c) {
    subs[c % ns].order = K.B.order;
    subs[c % ns].classes.push_back(K.B.classes[c]);
  }
  PWF_HIP(hipEventRecord(K.ctx.fork_ev[0], K.st));
  for (int j = 1; j < ns; ++j) PWF_HIP(hipStreamWaitEvent(K.ctx.fork[j - 1], K.ctx.fork_ev[0], 0));
  for (int j = 0; j < ns; ++j) {
    Launcher Kj{K.ctx, K.ws, K.L, subs[j], j == 0 ? K.st : K.ctx.fork[j - 1]};
    Kj.corr_tol = K.corr_tol;
    PWF_TRY(iterate(Kj));
  }
  for (int j = 1; j < ns; ++j) {
    PWF_HIP(hipEventRecord(K.ctx.fork_ev[j], K.ctx.fork[j - 1]));
    PWF_HIP(hipStreamWaitEvent(K.st, K.ctx.fork_ev[j], 0));
  }
  return PWF_OK;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

pwf_status solve_impl(const pwf_problem* problems, int32_t n, const float* const* y, void* const* psi_out,
                      int32_t iters, double corr_tol, double* loss_hist, int32_t* iters_done, void* workspace,
                      size_t workspace_bytes, void* stream, const JointCfg& jc) {
  PWF_TRY(validate_batch(problems, n));
  if (!y || !psi_out || iters < 0 || iters > kBetaCap || std::isnan(corr_tol) || corr_tol >= 1.0) return PWF_ERR_ARG;
  const bool corr_mode = corr_tol > 0.0;
  for (int i = 0; i < n; ++i)
    if (!y[i] || !psi_out[i]) return PWF_ERR_ARG;
  Layout L;
  PWF_TRY(check_ws(problems, n, workspace, workspace_bytes, &L, jc.on));
  std::lock_guard<std::mutex> lk(g_mu);
  Context* ctx;
  PWF_TRY(context_for_current(&ctx));
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const Batch B = group(problems, n);
  const bool merged = !jc.on && batch_merged(B);
  std::vector<Inst> desc(n);
  for (int s = 0; s < n; ++s) {
    const int i = B.order[s];
    Inst& I = desc[s];
    I = base_inst(problems[i]);
    attach_tables(I, ws, L, i);
    I.W = (float2*)(ws + L.W[i]);
    I.v = (float2*)(ws + L.v[i]);
    I.x = (float2*)(ws + L.psi[i]);
    I.psi_hat = (float2*)(ws + L.psi_hat[i]);
    I.z_hat = (float2*)(ws + L.z_hat[i]);
    I.y_hat = (float2*)(ws + L.y_hat[i]);
    I.y = y[i];
    I.out = (float2*)psi_out[i];
    I.loss_partial = (double*)(ws + L.part[i]);
    I.loss_dst = loss_hist ? loss_hist + (size_t)i * iters : nullptr;
    if (jc.on) {
      I.u1 = (float2*)(ws + L.u1[i]);
      I.u1max = (float*)(ws + L.u1max) + (size_t)i * problems[i].geom.ny;
    }
    if (corr_mode) {
      I.corr_partial = (double*)(ws + L.corr[i]);
      I.n_corr_partials = problems[i].geom.ny /
                          pwf::row_rows_per_block(problems[i].geom.nx, row_plan(problems[i].geom.nx, pwf::ROW_PSI_UPDATE));
      I.stop_iter = (int32_t*)(ws + L.stop) + i;
    }
  }
  // maxt2 slots depend only on the diffuser pointers; fill desc before upload
  {
    std::vector<const void*> seen;
    for (int s = 0; s < n; ++s) {
      const pwf_problem& p = problems[B.order[s]];
      int slot = -1;
      for (size_t j = 0; j < seen.size(); ++j)
        if (seen[j] == p.diffuser) slot = (int)j;
      if (slot < 0) {
        slot = (int)seen.size();
        seen.push_back(p.diffuser);
      }
      desc[s].maxt2 = (const float*)(ws + L.maxt2) + slot;
    }
  }
  PWF_TRY(upload(*ctx, desc.data(), sizeof(Inst) * n, ws + L.desc, st));
  PWF_HIP(pwf::launch_build_tables((const Inst*)(ws + L.desc), n, st));
  if (iters_done)
    for (int i = 0; i < n; ++i) iters_done[i] = iters;

  auto enqueue = [&](hipStream_t s) -> pwf_status {
    Launcher K{*ctx, ws, L, B, s};
    K.corr_tol = corr_tol;
    K.merged = merged;
    if (corr_mode) PWF_HIP(pwf::launch_fill_zero(ws + L.stop, align_up(sizeof(int32_t) * n), s));
    std::vector<Inst> tmp = desc;
    PWF_TRY(launch_maxt2(problems, n, B, tmp, ws, L, s));
    return solve_sequence(K, problems, n, desc, iters, jc);
  };

  auto report = [&]() -> pwf_status {
    if (!corr_mode || !iters_done) return PWF_OK;
    std::vector<int32_t> stop(n);
    PWF_HIP(hipMemcpyAsync(stop.data(), ws + L.stop, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
    PWF_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) iters_done[i] = stop[i] > 0 ? stop[i] : iters;
    return PWF_OK;
  };

  if (!g_graph_mode) {
    PWF_TRY(enqueue(st));
    return report();
  }

  GraphKey key{workspace, n, iters, {}};
  key.dims.push_back(corr_mode ? 1 : 0);
  key.dims.push_back(g_tune_gen);
  key.dims.push_back(jc.on ? 1 : 0);
  key.dims.push_back(merged ? 1 : 0);
  for (double d : {corr_tol, jc.eta_t}) {
    int64_t bits;
    std::memcpy(&bits, &d, sizeof(bits));
    key.dims.push_back((int)(bits & 0x7fffffff));
    key.dims.push_back((int)((bits >> 31) & 0x7fffffff));
    key.dims.push_back((int)(bits >> 62));
  }
  for (int s = 0; s < n; ++s) {
    const pwf_problem& p = problems[B.order[s]];
    key.dims.push_back(p.geom.nx);
    key.dims.push_back(p.geom.ny);
    key.dims.push_back((int)(((uintptr_t)p.diffuser) & 0x7fffffff));
    key.dims.push_back((int)(((uintptr_t)p.diffuser) >> 31));
  }
  hipGraphExec_t exec = nullptr;
  auto it = ctx->graphs.find(key);
  if (it != ctx->graphs.end()) {
    exec = it->second;
  } else {
    hipGraph_t graph = nullptr;
    PWF_HIP(hipStreamBeginCapture(ctx->side, hipStreamCaptureModeThreadLocal));
    const pwf_status cs = enqueue(ctx->side);
    const hipError_t ee = hipStreamEndCapture(ctx->side, &graph);
    if (cs != PWF_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return cs;
    }
    PWF_HIP(ee);
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    PWF_HIP(ie);
    if (ctx->graphs.size() >= 8) {
      (void)hipGraphExecDestroy(ctx->graphs.begin()->second);
      ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs[key] = exec;
  }
  PWF_HIP(hipEventRecord(ctx->ev_in, st));
  PWF_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_in, 0));
  PWF_HIP(hipGraphLaunch(exec, ctx->side));
  PWF_HIP(hipEventRecord(ctx->ev_out, ctx->side));
  PWF_HIP(hipStreamWaitEvent(st, ctx->ev_out, 0));
  return report();
}

}  // namespace

extern "C" {

pwf_status pwf_solve(const pwf_problem* problems, int32_t n, const float* const* y, void* const* psi_out,
                     int32_t iters, double corr_tol, double* loss_hist, int32_t* iters_done, void* workspace,
                     size_t workspace_bytes, void* stream) {
  return solve_impl(problems, n, y, psi_out, iters, corr_tol, loss_hist, iters_done, workspace, workspace_bytes,
                    stream, JointCfg{});
}

size_t pwf_joint_workspace_size(const pwf_problem* problems, int32_t n) {
  if (validate_batch(problems, n) != PWF_OK) return 0;
  return make_layout(problems, n, true).total;
}

pwf_status pwf_solve_joint(const pwf_problem* problems, int32_t n, const float* const* y, void* const* psi_out,
                           int32_t iters, double eta_t, double* loss_hist, void* workspace, size_t workspace_bytes,
                           void* stream) {
  PWF_TRY(validate_batch(problems, n));
  if (!std::isfinite(eta_t) || eta_t < 0.0) return PWF_ERR_ARG;
  for (int i = 1; i < n; ++i)
    if (problems[i].diffuser != problems[0].diffuser || problems[i].geom.nx != problems[0].geom.nx ||
        problems[i].geom.ny != problems[0].geom.ny)
      return PWF_ERR_ARG;
  return solve_impl(problems, n, y, psi_out, iters, 0.0, loss_hist, nullptr, workspace, workspace_bytes, stream,
                    JointCfg{true, eta_t});
}

pwf_status pwf_bench_sweep(const pwf_problem* problems, int32_t n, int32_t sweep, int32_t reps, void* workspace,
                           size_t workspace_bytes, void* stream) {
  PWF_TRY(validate_batch(problems, n));
  if (sweep < 0 || sweep > 11 || reps < 1) return PWF_ERR_ARG;
  Layout L;
  PWF_TRY(check_ws(problems, n, workspace, workspace_bytes, &L));
  std::lock_guard<std::mutex> lk(g_mu);
  Context* ctx;
  PWF_TRY(context_for_current(&ctx));
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const Batch B = group(problems, n);
  std::vector<Inst> desc(n);
  std::vector<const void*> seen;
  for (int s = 0; s < n; ++s) {
    const int i = B.order[s];
    Inst& I = desc[s];
    I = base_inst(problems[i]);
    attach_tables(I, ws, L, i);
    I.W = (float2*)(ws + L.W[i]);
    I.v = (float2*)(ws + L.v[i]);
    I.x = (float2*)(ws + L.psi[i]);
    I.psi_hat = (float2*)(ws + L.psi_hat[i]);
    I.z_hat = (float2*)(ws + L.z_hat[i]);
    I.y_hat = (float2*)(ws + L.y_hat[i]);
    I.loss_partial = (double*)(ws + L.part[i]);
    int slot = -1;
    for (size_t j = 0; j < seen.size(); ++j)
      if (seen[j] == problems[i].diffuser) slot = (int)j;
    if (slot < 0) {
      slot = (int)seen.size();
      seen.push_back(problems[i].diffuser);
    }
    I.maxt2 = (const float*)(ws + L.maxt2) + slot;
  }
  PWF_TRY(upload(*ctx, desc.data(), sizeof(Inst) * n, ws + L.desc, st));
  PWF_HIP(pwf::launch_build_tables((const Inst*)(ws + L.desc), n, st));
  const Launcher K{*ctx, ws, L, B, st};
  static const int kOps[12][2] = {
      {0, pwf::ROW_PSI_UPDATE}, {1, pwf::COL_CHIRP1},      {0, pwf::ROW_MUL_T},      {1, pwf::COL_CHIRP2},
      {0, pwf::ROW_INTENSITY},  {1, pwf::COL_BLUR_LOSS},   {0, pwf::ROW_BACKBLUR},   {1, pwf::COL_CHIRP2_CONJ},
      {0, pwf::ROW_MUL_CONJ_T}, {1, pwf::COL_CHIRP1_CONJ}, {0, pwf::ROW_GRAD},       {1, pwf::COL_NESTEROV}};
  for (int r = 0; r < reps; ++r) {
    if (kOps[sweep][0] == 0) {
      PWF_TRY(K.row(kOps[sweep][1], 0));
    } else {
      PWF_TRY(K.col(kOps[sweep][1], 0));
    }
  }
  return PWF_OK;
}

pwf_status pwf_set_column_tile(int32_t n, int32_t sweep, int32_t width) {
  const int i = size_index(n);
  if (i < 0) return PWF_ERR_SIZE;
  if (width != 0 && !pwf::col_width_supported(n, width)) return PWF_ERR_ARG;
  const int op = sweep < 0 ? -1 : col_op_of_sweep(sweep);
  if (sweep >= 0 && op < 0) return PWF_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  if (op < 0) {
    for (int& w : g_col_width[i]) w = width;
  } else {
    g_col_width[i][op] = width;
  }
  ++g_tune_gen;
  return PWF_OK;
}

int32_t pwf_column_tile(int32_t n, int32_t sweep) {
  const int op = col_op_of_sweep(sweep);
  if (op < 0) return 0;
  std::lock_guard<std::mutex> lk(g_mu);
  return col_width(n, op);
}

pwf_status pwf_set_row_plan(int32_t n, int32_t sweep, int32_t plan) {
  const int i = size_index(n);
  if (i < 0) return PWF_ERR_SIZE;
  const int op = row_op_of_sweep(sweep);
  if (op < 0 || plan < -1 || plan >= pwf::row_plan_count_n(n)) return PWF_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  g_row_plan[i][op] = plan;
  ++g_tune_gen;
  return PWF_OK;
}

int32_t pwf_row_plan(int32_t n, int32_t sweep) {
  const int op = row_op_of_sweep(sweep);
  if (size_index(n) < 0 || op < 0) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  return row_plan(n, op);
}

pwf_status pwf_autotune(const pwf_problem* problems, int32_t n, int32_t reps, void* workspace,
                        size_t workspace_bytes, void* stream) {
  PWF_TRY(validate_batch(problems, n));
  if (reps < 1) return PWF_ERR_ARG;
  Layout L;
  PWF_TRY(check_ws(problems, n, workspace, workspace_bytes, &L));
  std::lock_guard<std::mutex> lk(g_mu);
  Context* ctx;
  PWF_TRY(context_for_current(&ctx));
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const Batch B = group(problems, n);
  std::vector<Inst> desc(n);
  for (int s = 0; s < n; ++s) {
    const int i = B.order[s];
    Inst& I = desc[s];
    I = base_inst(problems[i]);
    attach_tables(I, ws, L, i);
    I.W = (float2*)(ws + L.W[i]);
    I.v = (float2*)(ws + L.v[i]);
    I.x = (float2*)(ws + L.psi[i]);
    I.psi_hat = (float2*)(ws + L.psi_hat[i]);
    I.z_hat = (float2*)(ws + L.z_hat[i]);
    I.y_hat = (float2*)(ws + L.y_hat[i]);
    I.loss_partial = (double*)(ws + L.part[i]);
    I.maxt2 = (const float*)(ws + L.maxt2);
  }
  PWF_TRY(upload(*ctx, desc.data(), sizeof(Inst) * n, ws + L.desc, st));
  PWF_HIP(pwf::launch_build_tables((const Inst*)(ws + L.desc), n, st));
  // every field region (timing does not depend on the values)
  PWF_HIP(pwf::launch_fill_zero(ws + L.W[0], L.extra0[0] - L.W[0], st));
  hipEvent_t e0, e1;
  PWF_HIP(hipEventCreate(&e0));
  PWF_HIP(hipEventCreate(&e1));
  pwf_status result = PWF_OK;
  const bool merged = batch_merged(B);
  for (const Class& c : B.classes) {
    Batch one;
    one.order = B.order;
    one.classes = {c};
    const Launcher K{*ctx, ws, L, one, st};
    const int cidx = size_index(c.ny), ridx = size_index(c.nx);
    // time `reps` launches of one sweep (after a warm-up launch)
    auto timed = [&](auto launch, float* ms) -> pwf_status {
      PWF_TRY(launch());
      PWF_HIP(hipEventRecord(e0, st));
      for (int r = 0; r < reps; ++r) PWF_TRY(launch());
      PWF_HIP(hipEventRecord(e1, st));
      PWF_HIP(hipEventSynchronize(e1));
      PWF_HIP(hipEventElapsedTime(ms, e0, e1));
      return PWF_OK;
    };
    // every sweep of the iteration, one at a time: tile width of the column
    // sweeps, radix plan of the row sweeps
    for (int sweep = 0; sweep < 12 && result == PWF_OK; ++sweep) {
      float best = 0.f, ms = 0.f;
      if (sweep & 1) {
        const int op = col_op_of_sweep(sweep);
        const int cands[2] = {pwf::col_default_width(c.ny), pwf::col_alt_width(c.ny)};
        int best_w = merged ? pwf::multi_col_width(c.ny) : col_width(c.ny, op);
        for (int w : cands) {
          if (c.nx % w) continue;
          if (merged && w != pwf::multi_col_width(c.ny)) continue;
          g_col_width[cidx][op] = w;
          result = timed([&]() { return K.col(op); }, &ms);
          if (result != PWF_OK) break;
          if (best == 0.f || ms < best) {
            best = ms;
            best_w = w;
          }
        }
        g_col_width[cidx][op] = best_w;
      } else {
        const int op = row_op_of_sweep(sweep);
        int best_plan = row_plan(c.nx, op);
        if (merged && !pwf::multi_row_supported(c.nx, c.ny, best_plan)) best_plan = c.nx == 512 ? 0 : 1;
        for (int plan = 0; plan < pwf::row_plan_count_n(c.nx); ++plan) {
          if (merged && !pwf::multi_row_supported(c.nx, c.ny, plan)) continue;
          g_row_plan[ridx][op] = plan;
          result = timed([&]() { return K.row(op); }, &ms);
          if (result != PWF_OK) break;
          if (best == 0.f || ms < best) {
            best = ms;
            best_plan = plan;
          }
        }
        g_row_plan[ridx][op] = best_plan;
      }
    }
    if (result != PWF_OK) break;
  }
  ++g_tune_gen;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return result;
}

}  // extern "C"

// ------------------------------------------------------------ persistent tuning cache
//
// One line per (architecture, class mix, grid side):
//   <arch> <mix> <side> c <w S1> <w S3> <w S5> <w S7> <w S9> <w S11> r <p S0> <p S2> ... <p S10>
// mix lists the batch's grid shapes and instance counts, e.g. 512x512*24+1024x1024*32.
namespace {

// Architecture of the current device and the library version: a cached
// schedule was timed on these kernels, so another version re-times it.
std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a(prop.gcnArchName);
  const size_t colon = a.find(':');
  return (colon == std::string::npos ? a : a.substr(0, colon)) + "/v" + std::to_string(kVersion);
}

// Tuning-cache key of a batch: its class mix, marked "/merged" when the batch
// launches merged (the tuner then chooses only among the plans and widths the
// merged kernels hold, so those choices are kept apart from per-class ones).
std::string class_mix(const Batch& B) {
  std::string m;
  for (const Class& c : B.classes) {
    if (!m.empty()) m += '+';
    m += std::to_string(c.nx) + 'x' + std::to_string(c.ny) + '*' + std::to_string(c.count);
  }
  return batch_merged(B) ? m + "/merged" : m;
}

std::vector<int> batch_sides(const Batch& B) {
  std::vector<int> sides;
  for (const Class& c : B.classes)
    for (int sd : {c.nx, c.ny})
      if (std::find(sides.begin(), sides.end(), sd) == sides.end()) sides.push_back(sd);
  std::sort(sides.begin(), sides.end());
  return sides;
}

std::string tuning_line(const std::string& arch, const std::string& mix, int side) {
  std::string l = arch + ' ' + mix + ' ' + std::to_string(side) + " c";
  for (int sw = 1; sw < 12; sw += 2) l += ' ' + std::to_string(col_width(side, col_op_of_sweep(sw)));
  l += " r";
  for (int sw = 0; sw < 12; sw += 2) l += ' ' + std::to_string(row_plan(side, row_op_of_sweep(sw)));
  return l;
}

// Apply the line's settings when it matches arch and mix; returns its side, or 0.
int apply_tuning_line(const std::string& line, const std::string& arch, const std::string& mix) {
  std::istringstream in(line);
  std::string a, m, c, r;
  int side = 0;
  int w[6], pl[6];
  if (!(in >> a >> m >> side >> c) || a != arch || m != mix || c != "c") return 0;
  for (int& v : w)
    if (!(in >> v)) return 0;
  if (!(in >> r) || r != "r") return 0;
  for (int& v : pl)
    if (!(in >> v)) return 0;
  const int i = size_index(side);
  if (i < 0) return 0;
  for (int k = 0; k < 6; ++k) {
    if (!pwf::col_width_supported(side, w[k]) || pl[k] < 0 || pl[k] >= pwf::row_plan_count_n(side)) return 0;
  }
  for (int k = 0; k < 6; ++k) {
    g_col_width[i][col_op_of_sweep(2 * k + 1)] = w[k];
    g_row_plan[i][row_op_of_sweep(2 * k)] = pl[k];
  }
  return side;
}

}  // namespace

extern "C" {

pwf_status pwf_autotune_cached(const pwf_problem* problems, int32_t n, int32_t reps, const char* cache_path,
                               int32_t force, int32_t* tuned, void* workspace, size_t workspace_bytes,
                               void* stream) {
  PWF_TRY(validate_batch(problems, n));
  if (!cache_path || reps < 1) return PWF_ERR_ARG;
  const Batch B = group(problems, n);
  const std::vector<int> sides = batch_sides(B);
  std::string mix;
  {
    std::lock_guard<std::mutex> lk(g_mu);  // (the merge mode is read under the lock)
    mix = class_mix(B);
  }
  std::vector<std::string> lines;
  {
    std::ifstream in(cache_path);
    for (std::string l; std::getline(in, l);)
      if (!l.empty()) lines.push_back(l);
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    const std::string arch = device_arch();
    std::vector<int> found;
    for (const std::string& l : lines) {
      std::istringstream in(l);
      std::string a, m;
      int side = 0;
      if (in >> a >> m >> side && a == arch && m == mix && size_index(side) >= 0 &&
          std::find(sides.begin(), sides.end(), side) != sides.end())
        found.push_back(side);
    }
    bool all = !force;
    for (int sd : sides) all = all && std::find(found.begin(), found.end(), sd) != found.end();
    if (all) {
      for (const std::string& l : lines) apply_tuning_line(l, arch, mix);
      ++g_tune_gen;
      if (tuned) *tuned = 0;
      return PWF_OK;
    }
  }
  PWF_TRY(pwf_autotune(problems, n, reps, workspace, workspace_bytes, stream));
  std::lock_guard<std::mutex> lk(g_mu);
  const std::string arch = device_arch();
  std::vector<std::string> keep;
  for (const std::string& l : lines) {
    std::istringstream in(l);
    std::string a, m;
    if (in >> a >> m && a == arch && m == mix) continue;   // replaced below
    keep.push_back(l);
  }
  for (int sd : sides) keep.push_back(tuning_line(arch, mix, sd));
  const std::string tmp = std::string(cache_path) + ".tmp";
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) return PWF_ERR_ARG;
    for (const std::string& l : keep) out << l << '\n';
    if (!out) return PWF_ERR_ARG;
  }
  if (std::rename(tmp.c_str(), cache_path) != 0) return PWF_ERR_ARG;
  if (tuned) *tuned = 1;
  return PWF_OK;
}

pwf_status pwf_solve_plain(const pwf_problem* problem, const float* y, void* psi_out, int32_t iters,
                           double* loss_hist, void* workspace, size_t workspace_bytes, void* stream) {
  PWF_TRY(validate_batch(problem, 1));
  if (!y || !psi_out || iters < 0 || iters > kBetaCap) return PWF_ERR_ARG;
  Layout L;
  PWF_TRY(check_ws(problem, 1, workspace, workspace_bytes, &L));
  std::lock_guard<std::mutex> lk(g_mu);
  Context* ctx;
  PWF_TRY(context_for_current(&ctx));
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const pwf_problem& p = *problem;
  const int nx = p.geom.nx, ny = p.geom.ny;
  const size_t m = (size_t)nx * ny;
  Inst I = base_inst(p);
  attach_tables(I, ws, L, 0);
  I.y = y;
  I.maxt2 = (const float*)(ws + L.maxt2);
  Inst* dI = (Inst*)(ws + L.desc);
  PWF_TRY(upload(*ctx, &I, sizeof(Inst), dI, st));
  PWF_HIP(pwf::launch_build_tables(dI, 1, st));
  float2* psi = (float2*)psi_out;
  float2* Z = (float2*)(ws + L.W[0]);
  float2* X = (float2*)(ws + L.psi_hat[0]);
  float2* V = (float2*)(ws + L.z_hat[0]);
  float2* A = (float2*)(ws + L.v[0]);
  float2* Bf = (float2*)(ws + L.psi[0]);
  float2* Cc = (float2*)(ws + L.y_hat[0]);
  float2* G = (float2*)(ws + L.extra0[0]);
  double* part = (double*)(ws + L.part[0]);
  int32_t* status = (int32_t*)(ws + L.status);
  const float2* twx = ctx->tw[size_index(nx)];
  const float2* twy = ctx->twc[size_index(ny)];

  PWF_HIP(pwf::launch_fill_zero(status, 16, st));
  PWF_HIP(pwf::launch_maxabs2((const float2*)p.diffuser, m, (float*)(ws + L.maxt2_part), (float*)(ws + L.maxt2), st));
  PWF_HIP(pwf::launch_fill_zero(psi, m * sizeof(float2), st));
  PWF_HIP(pwf::launch_fill_zero(Z, m * sizeof(float2), st));

  // Filter (Algorithm S2): F^-1{ F{src} W_k } -> dst, one kernel per step
  auto filter = [&](const float2* src, float2* dst, int window) -> pwf_status {
    PWF_HIP(pwf::launch_plain_rows(nx, -1, src, dst, ny, twx, st));
    PWF_HIP(pwf::launch_plain_cols(ny, -1, dst, nx, twy, st));
    PWF_HIP(pwf::launch_plain_window(dst, dI, window, m, st));
    PWF_HIP(pwf::launch_plain_cols(ny, 1, dst, nx, twy, st));
    PWF_HIP(pwf::launch_plain_rows(nx, 1, dst, dst, ny, twx, st));
    return PWF_OK;
  };
  auto ew = [&](int op, const float2* a, const float2* b, float2* c, float2* out, int iter) -> pwf_status {
    PWF_HIP(pwf::launch_plain_elementwise(op, m, a, b, c, out, dI, ctx->beta, iter, part, st));
    return PWF_OK;
  };
  for (int k = 0; k < iters; ++k) {
    PWF_TRY(ew(pwf::PLAIN_EXP, psi, nullptr, nullptr, X, k));         // x = exp(psi)
    PWF_TRY(filter(X, V, pwf::PLAIN_W_Q1));                           // sample -> diffuser
    PWF_TRY(ew(pwf::PLAIN_MUL_T, V, nullptr, nullptr, V, k));         // t v
    PWF_TRY(filter(V, V, pwf::PLAIN_W_Q2));                           // diffuser -> detector
    PWF_TRY(ew(pwf::PLAIN_ABS2, V, nullptr, nullptr, A, k));          // |v|^2
    PWF_TRY(filter(A, A, pwf::PLAIN_W_IOTF));                         // f
    PWF_TRY(ew(pwf::PLAIN_NEG_ERR, A, nullptr, nullptr, A, k));       // -e and the loss
    PWF_HIP(pwf::launch_plain_loss_final(part, pwf::plain_elementwise_blocks(),
                                         loss_hist, k, status, st));
    PWF_TRY(filter(A, A, pwf::PLAIN_W_IOTF));                         // Filter(-e, IOTF)
    PWF_TRY(ew(pwf::PLAIN_MUL, V, A, nullptr, A, k));                 // v h
    PWF_TRY(filter(A, A, pwf::PLAIN_W_Q2C));                          // propagate -L2
    PWF_TRY(ew(pwf::PLAIN_MUL_CONJ_T, A, nullptr, nullptr, A, k));    // t* (.)
    PWF_TRY(filter(A, A, pwf::PLAIN_W_Q1C));                          // propagate -L1
    PWF_TRY(ew(pwf::PLAIN_GRAD, A, X, nullptr, G, k));                // g = x* (.) / max|t|^2
    PWF_TRY(ew(pwf::PLAIN_IMAG, G, nullptr, nullptr, Bf, k));         // Im g
    PWF_TRY(filter(Bf, Bf, pwf::PLAIN_W_PINV));                       // preconditioner
    PWF_TRY(filter(psi, Cc, pwf::PLAIN_W_GAMMA2));                    // Filter(psi, Gamma^2)
    PWF_TRY(ew(pwf::PLAIN_DIRECTION, G, Bf, Cc, A, k));               // d
    PWF_TRY(ew(pwf::PLAIN_NESTEROV, psi, A, Z, psi, k));              // z, tau, psi
  }
  return PWF_OK;
}

// ------------------------------------------------------------ calibration front end

size_t pwf_speckle_workspace_size(void) {
  const int nv = 1 + 2 * (pwf::kMaxShift + 1);
  return align_up(sizeof(double) * ((size_t)pwf::speckle_sum_blocks() + 1) * nv);
}

pwf_status pwf_speckle_g2(const float* ref, int32_t nx, int32_t ny, int32_t max_shift, double* g2x, double* g2y,
                          void* workspace, size_t workspace_bytes, void* stream) {
  if (!ref || !g2x || !g2y || nx < 1 || ny < 1 || max_shift < 0 || max_shift > pwf::kMaxShift ||
      max_shift >= nx || max_shift >= ny)
    return PWF_ERR_ARG;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || workspace_bytes < pwf_speckle_workspace_size())
    return PWF_ERR_WORKSPACE;
  const int K = pwf::kMaxShift + 1, nv = 1 + 2 * K;
  double* partial = (double*)workspace;
  double* out = partial + (size_t)pwf::speckle_sum_blocks() * nv;
  hipStream_t st = (hipStream_t)stream;
  PWF_HIP(pwf::launch_speckle_sums(ref, nx, ny, max_shift, partial, out, st));
  std::vector<double> h(nv);
  PWF_HIP(hipMemcpyAsync(h.data(), out, sizeof(double) * nv, hipMemcpyDeviceToHost, st));
  PWF_HIP(hipStreamSynchronize(st));
  // g2(d) = <I(r) I(r + d)> / <I>^2 (Methods, Eq. 3)
  const double m = (double)nx * ny;
  const double mean = h[0] / m;
  if (!(mean > 0.0)) return PWF_ERR_ARG;
  for (int d = 0; d <= max_shift; ++d) {
    g2x[d] = h[1 + d] / m / (mean * mean);
    g2y[d] = h[1 + K + d] / m / (mean * mean);
  }
  return PWF_OK;
}

pwf_status pwf_fit_coherence(const double* g2, int32_t count, double pixel_m, double* coh_m, double* contrast) {
  if (!g2 || !coh_m || count < 3 || !(pixel_m > 0.0)) return PWF_ERR_ARG;
  // ln(g2 - 1) = ln c - pi (d p)^2 / coh^2 over d = 1..K; K: the last shift
  // before g2 - 1 first drops below 2% of g2(1) - 1
  const double floor = 0.02 * (g2[1] - 1.0);
  if (!(g2[1] - 1.0 > 0.0)) return PWF_ERR_ARG;
  int k = 1;
  while (k + 1 < count && g2[k + 1] - 1.0 >= floor) ++k;
  if (k < 2) return PWF_ERR_ARG;
  double sx = 0, sy = 0, sxx = 0, sxy = 0;
  for (int d = 1; d <= k; ++d) {
    const double xv = (d * pixel_m) * (d * pixel_m), yv = std::log(g2[d] - 1.0);
    sx += xv;
    sy += yv;
    sxx += xv * xv;
    sxy += xv * yv;
  }
  const double nk = k, den = nk * sxx - sx * sx;
  const double slope = (nk * sxy - sx * sy) / den, icpt = (sy - slope * sx) / nk;
  if (!(slope < 0.0)) return PWF_ERR_ARG;
  *coh_m = std::sqrt(-M_PI / slope);
  if (contrast) *contrast = std::exp(icpt);
  return PWF_OK;
}

pwf_status pwf_diffuser_from_reference(const pwf_problem* problem, const float* ref, double eps, void* t_out,
                                       void* workspace, size_t workspace_bytes, void* stream) {
  PWF_TRY(validate_batch(problem, 1));
  if (!ref || !t_out || !std::isfinite(eps) || eps < 0.0) return PWF_ERR_ARG;
  Layout L;
  PWF_TRY(check_ws(problem, 1, workspace, workspace_bytes, &L));
  std::lock_guard<std::mutex> lk(g_mu);
  Context* ctx;
  PWF_TRY(context_for_current(&ctx));
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const pwf_problem& p = *problem;
  const int nx = p.geom.nx, ny = p.geom.ny;
  const size_t m = (size_t)nx * ny;
  Inst I = base_inst(p);
  attach_tables(I, ws, L, 0);
  I.y = ref;
  I.wiener_eps = (float)eps;
  Inst* dI = (Inst*)(ws + L.desc);
  PWF_TRY(upload(*ctx, &I, sizeof(Inst), dI, st));
  PWF_HIP(pwf::launch_build_tables(dI, 1, st));
  float2* X = (float2*)(ws + L.W[0]);
  float2* t = (float2*)t_out;
  double* part = (double*)(ws + L.part[0]);
  const float2* twx = ctx->tw[size_index(nx)];
  const float2* twy = ctx->twc[size_index(ny)];
  auto filter = [&](const float2* src, float2* dst, int window) -> pwf_status {
    PWF_HIP(pwf::launch_plain_rows(nx, -1, src, dst, ny, twx, st));
    PWF_HIP(pwf::launch_plain_cols(ny, -1, dst, nx, twy, st));
    PWF_HIP(pwf::launch_plain_window(dst, dI, window, m, st));
    PWF_HIP(pwf::launch_plain_cols(ny, 1, dst, nx, twy, st));
    PWF_HIP(pwf::launch_plain_rows(nx, 1, dst, dst, ny, twx, st));
    return PWF_OK;
  };
  auto ew = [&](int op, const float2* a, float2* out) -> pwf_status {
    PWF_HIP(pwf::launch_plain_elementwise(op, m, a, nullptr, nullptr, out, dI, ctx->beta, 0, part, st));
    return PWF_OK;
  };
  // Results, "Diffuser transmission function": Wiener deconvolution by the
  // IOTF, zero-phase square root, back-propagation over L2
  PWF_TRY(ew(pwf::PLAIN_FROM_REAL, nullptr, X));
  PWF_TRY(filter(X, X, pwf::PLAIN_W_WIENER));
  PWF_TRY(ew(pwf::PLAIN_SQRT_POS, X, X));
  PWF_TRY(filter(X, t, pwf::PLAIN_W_Q2C));
  return PWF_OK;
}

// ------------------------------------------------------------ tomography

namespace {
constexpr int kMaxFbpAngles = 4096;

int fbp_pad_length(int nx) {
  int p = 64;
  while (p < 2 * nx) p <<= 1;
  return p;
}

struct FbpLayout {
  size_t q = 0, ramp = 0, cs = 0, ptrs = 0, total = 0;
};

bool fbp_layout(int n_proj, int nx, int ny, FbpLayout* L) {
  if (n_proj < 1 || n_proj > kMaxFbpAngles || nx < 64 || ny < 32 || ny % 32) return false;
  const int n_pad = fbp_pad_length(nx);
  if (size_index(n_pad) < 0) return false;
  size_t off = 0;
  L->q = off;
  off += align_up(sizeof(float2) * (size_t)n_proj * ny * n_pad);
  L->ramp = off;
  off += align_up(sizeof(float) * n_pad);
  L->cs = off;
  off += align_up(sizeof(float2) * n_proj);
  L->ptrs = off;
  off += align_up(sizeof(void*) * n_proj);
  L->total = off;
  return true;
}
}  // namespace

size_t pwf_fbp_workspace_size(int32_t n_proj, int32_t nx, int32_t ny) {
  FbpLayout L;
  return fbp_layout(n_proj, nx, ny, &L) ? L.total : 0;
}

pwf_status pwf_fbp(const void* const* psi, int32_t n_proj, int32_t nx, int32_t ny, const double* angles_rad,
                   int32_t n_out, double scale, void* vol_out, void* workspace, size_t workspace_bytes,
                   void* stream) {
  FbpLayout L;
  if (!fbp_layout(n_proj, nx, ny, &L)) return PWF_ERR_SIZE;
  if (!psi || !angles_rad || !vol_out || n_out < 16 || n_out % 16 || !std::isfinite(scale)) return PWF_ERR_ARG;
  for (int j = 0; j < n_proj; ++j)
    if (!psi[j] || !std::isfinite(angles_rad[j])) return PWF_ERR_ARG;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || workspace_bytes < L.total) return PWF_ERR_WORKSPACE;
  std::lock_guard<std::mutex> lk(g_mu);
  Context* ctx;
  PWF_TRY(context_for_current(&ctx));
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const int n_pad = fbp_pad_length(nx);
  // ramp response: DFT of the band-limited ramp h(0) = 1/4, h(odd n) =
  // -1/(pi^2 n^2) on the circular grid of n_pad samples, over n_pad for the
  // unnormalised inverse transform
  // (an O(n_pad^2) host loop: kept per n_pad for repeated calls)
  static std::mutex ramp_mu;
  static std::vector<float> ramp_cached;
  std::vector<float> H;
  {
    std::lock_guard<std::mutex> lk(ramp_mu);
    if ((int)ramp_cached.size() != n_pad) {
      ramp_cached.assign(n_pad, 0.f);
      for (int k = 0; k < n_pad; ++k) {
        double acc = 0.25;
        for (int n = 1; n <= n_pad / 2; n += 2) {
          const double hn = -1.0 / (M_PI * M_PI * (double)n * n);
          const double w = (n == n_pad / 2 ? 1.0 : 2.0) * std::cos(2.0 * M_PI * (double)k * n / n_pad);
          acc += hn * w;
        }
        ramp_cached[k] = (float)(acc / n_pad);
      }
    }
    H = ramp_cached;
  }
  std::vector<float2> cs(n_proj);
  for (int j = 0; j < n_proj; ++j) cs[j] = make_float2((float)std::cos(angles_rad[j]), (float)std::sin(angles_rad[j]));
  PWF_TRY(upload(*ctx, H.data(), sizeof(float) * n_pad, ws + L.ramp, st));
  PWF_TRY(upload(*ctx, cs.data(), sizeof(float2) * n_proj, ws + L.cs, st));
  PWF_TRY(upload(*ctx, psi, sizeof(void*) * n_proj, ws + L.ptrs, st));
  float2* q = (float2*)(ws + L.q);
  const size_t rows = (size_t)n_proj * ny;
  const float2* tw = ctx->tw[size_index(n_pad)];
  PWF_HIP(pwf::launch_fbp_pad((const float2* const*)(ws + L.ptrs), n_proj, nx, ny, n_pad, q, st));
  PWF_HIP(pwf::launch_plain_rows(n_pad, -1, q, q, (int)rows, tw, st));
  PWF_HIP(pwf::launch_fbp_ramp(q, (const float*)(ws + L.ramp), n_pad, rows, st));
  PWF_HIP(pwf::launch_plain_rows(n_pad, 1, q, q, (int)rows, tw, st));
  PWF_HIP(pwf::launch_fbp_backproject(q, n_proj, nx, ny, n_pad, (const float2*)(ws + L.cs), n_out,
                                      (float)(scale * M_PI / n_proj), (float2*)vol_out, st));
  return PWF_OK;
}

// ------------------------------------------------------------ background removal

namespace {
constexpr int kBgMaxN = 8192;

bool bg_layout(int n_slices, int n, size_t* part_off, size_t* coef_off, size_t* total) {
  if (n_slices < 1 || n < 16 || n % 16 || n > kBgMaxN) return false;
  const size_t bands = (size_t)(n / pwf::bg_rows_per_band(n));
  *part_off = align_up(sizeof(double) * 36);
  *coef_off = *part_off + align_up(sizeof(double) * 12 * bands * n_slices);
  *total = *coef_off + align_up(sizeof(double) * 12 * (size_t)n_slices);
  return true;
}

// Inverse of the 6 x 6 normal matrix of the quadratic monomials over the
// background voxels (radius >= r_bg), FP64 Gauss-Jordan with partial pivoting.
// False when fewer than 6 voxels or a pivot below 1e-12 of the largest
// diagonal entry leave the fit undetermined.
bool bg_normal_inverse(int n, double r_bg, double (&inv)[36]) {
  double M[36] = {0.0};
  const double h = 0.5 * n, inv_h = 1.0 / h, r2 = r_bg * r_bg;
  size_t count = 0;
  for (int iz = 0; iz < n; ++iz) {
    const double Z = iz + 0.5 - h;
    for (int ix = 0; ix < n; ++ix) {
      const double X = ix + 0.5 - h;
      if (X * X + Z * Z < r2) continue;
      const double x = X * inv_h, z = Z * inv_h;
      const double m[6] = {1.0, x, z, x * x, x * z, z * z};
      for (int a = 0; a < 6; ++a)
        for (int b = a; b < 6; ++b) M[a * 6 + b] += m[a] * m[b];
      ++count;
    }
  }
  if (count < 6) return false;
  double scale = 0.0;
  for (int a = 0; a < 6; ++a) {
    for (int b = 0; b < a; ++b) M[a * 6 + b] = M[b * 6 + a];
    scale = std::max(scale, M[a * 6 + a]);
  }
  for (int i = 0; i < 36; ++i) inv[i] = (i % 7 == 0) ? 1.0 : 0.0;
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    for (int r = c + 1; r < 6; ++r)
      if (std::fabs(M[r * 6 + c]) > std::fabs(M[piv * 6 + c])) piv = r;
    if (!(std::fabs(M[piv * 6 + c]) > 1e-12 * scale)) return false;
    for (int k = 0; k < 6; ++k) {
      std::swap(M[c * 6 + k], M[piv * 6 + k]);
      std::swap(inv[c * 6 + k], inv[piv * 6 + k]);
    }
    const double d = 1.0 / M[c * 6 + c];
    for (int k = 0; k < 6; ++k) {
      M[c * 6 + k] *= d;
      inv[c * 6 + k] *= d;
    }
    for (int r = 0; r < 6; ++r) {
      if (r == c) continue;
      const double f = M[r * 6 + c];
      for (int k = 0; k < 6; ++k) {
        M[r * 6 + k] -= f * M[c * 6 + k];
        inv[r * 6 + k] -= f * inv[c * 6 + k];
      }
    }
  }
  return true;
}
}  // namespace

size_t pwf_background_workspace_size(int32_t n_slices, int32_t n) {
  size_t part_off, coef_off, total;
  return bg_layout(n_slices, n, &part_off, &coef_off, &total) ? total : 0;
}

pwf_status pwf_background_quadratic(void* vol, int32_t n_slices, int32_t n, double r_bg, double* coef_out,
                                    void* workspace, size_t workspace_bytes, void* stream) {
  size_t part_off, coef_off, total;
  if (!bg_layout(n_slices, n, &part_off, &coef_off, &total)) return PWF_ERR_SIZE;
  if (!vol || !std::isfinite(r_bg) || r_bg < 0.0) return PWF_ERR_ARG;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || workspace_bytes < total) return PWF_ERR_WORKSPACE;
  // the normal matrix depends only on (n, r_bg): keep the last inversion (an
  // O(n^2) host loop) for repeated calls on tomograms of one shape
  static std::mutex inv_mu;
  static int inv_n = 0;
  static double inv_r = -1.0, inv_cached[36];
  static bool inv_ok = false;
  double inv[36];
  {
    std::lock_guard<std::mutex> lk(inv_mu);
    if (inv_n != n || inv_r != r_bg) {
      inv_ok = bg_normal_inverse(n, r_bg, inv_cached);
      inv_n = n;
      inv_r = r_bg;
    }
    if (!inv_ok) return PWF_ERR_ARG;
    std::memcpy(inv, inv_cached, sizeof(inv));
  }
  std::lock_guard<std::mutex> lk(g_mu);
  Context* ctx;
  PWF_TRY(context_for_current(&ctx));
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  PWF_TRY(upload(*ctx, inv, sizeof(inv), ws, st));
  double* partial = (double*)(ws + part_off);
  double* coef = (double*)(ws + coef_off);
  PWF_HIP(pwf::launch_bg_moments((const float2*)vol, n_slices, n, r_bg, partial, st));
  PWF_HIP(pwf::launch_bg_subtract((float2*)vol, n_slices, n, partial, (const double*)ws, coef, st));
  if (coef_out) {
    PWF_HIP(hipMemcpyAsync(coef_out, coef, sizeof(double) * 12 * (size_t)n_slices, hipMemcpyDeviceToHost, st));
    PWF_HIP(hipStreamSynchronize(st));
  }
  return PWF_OK;
}

// ------------------------------------------------------------ shell correlation

namespace {
// workspace: the packed field and its DFT (one complex n^dims array), the
// workgroups' shell partials, the shell sums
bool fsc_layout(int n, int dims, size_t* part_off, size_t* out_off, size_t* total) {
  if ((dims != 2 && dims != 3) || size_index(n) < 0) return false;
  const size_t m = dims == 3 ? (size_t)n * n * n : (size_t)n * n;
  const size_t nsh = (size_t)n / 2 + 1;
  size_t off = align_up(sizeof(float2) * m);
  *part_off = off;
  off += align_up(sizeof(double) * 3 * nsh * pwf::fsc_blocks());
  *out_off = off;
  off += align_up(sizeof(double) * 3 * nsh);
  *total = off;
  return true;
}
}  // namespace

size_t pwf_shell_correlation_workspace_size(int32_t n, int32_t dims) {
  size_t b, c, total;
  return fsc_layout(n, dims, &b, &c, &total) ? total : 0;
}

pwf_status pwf_shell_correlation(const void* g1, const void* g2, int32_t n, int32_t dims, int32_t part,
                                 double* fsc_out, void* workspace, size_t workspace_bytes, void* stream) {
  size_t part_off, out_off, total;
  if (!fsc_layout(n, dims, &part_off, &out_off, &total)) return PWF_ERR_SIZE;
  if (!g1 || !g2 || !fsc_out || (part != 0 && part != 1)) return PWF_ERR_ARG;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || workspace_bytes < total) return PWF_ERR_WORKSPACE;
  std::lock_guard<std::mutex> lk(g_mu);
  Context* ctx;
  PWF_TRY(context_for_current(&ctx));
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const size_t m = dims == 3 ? (size_t)n * n * n : (size_t)n * n;
  float2* X = (float2*)ws;
  const float2* twr = ctx->tw[size_index(n)];
  const float2* twc = ctx->twc[size_index(n)];
  // both parts in one complex field, then its n^dims DFT as 1-D transforms
  // along x, y (per z plane) and z; the shell sums separate the two spectra
  // (the unit-RMS scales live in the shell-sum area until the sums overwrite it)
  PWF_HIP(pwf::launch_fsc_pack((const float2*)g1, (const float2*)g2, part, X, m, (double*)(ws + part_off),
                               (float*)(ws + out_off), st));
  PWF_HIP(pwf::launch_plain_rows(n, -1, X, X, (int)(m / n), twr, st));
  const int planes = dims == 3 ? n : 1;
  PWF_HIP(pwf::launch_plain_cols(n, -1, X, n, twc, st, planes, (size_t)n * n));
  if (dims == 3) PWF_HIP(pwf::launch_plain_cols(n, -1, X, n * n, twc, st));
  double* out = (double*)(ws + out_off);
  PWF_HIP(pwf::launch_fsc_shells(X, n, dims, (double*)(ws + part_off), out, st));
  const int nsh = n / 2 + 1;
  std::vector<double> h(3 * (size_t)nsh);
  PWF_HIP(hipMemcpyAsync(h.data(), out, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
  PWF_HIP(hipStreamSynchronize(st));
  // Eq. 16: shell cross-correlation over the geometric mean of the shell powers
  for (int s = 0; s < nsh; ++s) fsc_out[s] = h[s] / std::sqrt(h[nsh + s] * h[2 * nsh + s]);
  return PWF_OK;
}

}  // extern "C"

// ------------------------------------------------------------ allocation-free variant
//
// pwf_loss_grad_noalloc runs pwf_loss_grad's kernels with its workspace in a
// file-scope device array instead of caller memory.  Each device holds its own
// copy of the array, at its own address, from the library's load until the
// process ends.  The array's name is only a host-side stand-in for that
// memory: host code uses the address that hipGetSymbolAddress returns for the
// current device (kept per device at the first call there) and nothing else.
// The first kScratchTableBytes hold the immutable twiddle tables, copied in
// once per device at that first call; the rest is the per-call workspace.

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr size_t kScratchTableBytes = size_t(1) << 20;
constexpr int kScratchMaxInst = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchDevice {
  bool ready = false;
  char* base = nullptr;          // device address of `scratch` on this device
  Context tables;                // table pointers into base (no streams, events or graphs)
  hipEvent_t copied = nullptr;   // recorded after the last descriptor copy from host_desc
  Inst host_desc[kScratchMaxInst];
};
ScratchDevice g_scratch[kMaxDevices];

// Set-up of the current device, once: the array's address, the tables, the event.
pwf_status scratch_for_current(ScratchDevice** out) {
  int dev = 0;
  PWF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return PWF_ERR_HIP;
  ScratchDevice& d = g_scratch[dev];
  if (!d.ready) {
    void* p = nullptr;
    PWF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return PWF_ERR_HIP;
    char* base = (char*)p;
    const HostTables& h = host_tables();
    size_t off = 0;
    auto put = [&](const std::vector<float2>& host, float2** dst) -> pwf_status {
      const size_t bytes = sizeof(float2) * host.size();
      if (off + bytes > kScratchTableBytes) return PWF_ERR_HIP;
      PWF_HIP(hipMemcpy(base + off, host.data(), bytes, hipMemcpyHostToDevice));
      *dst = (float2*)(base + off);
      off = align_up(off + bytes);
      return PWF_OK;
    };
    for (int i = 0; i < 5; ++i) {
      PWF_TRY(put(h.plan[i][0], &d.tables.tw[i]));
      PWF_TRY(put(h.plan[i][1], &d.tables.twc[i]));
      PWF_TRY(put(h.plan[i][2], &d.tables.twa[i]));
      PWF_TRY(put(h.plan[i][3], &d.tables.twa2[i]));
      PWF_TRY(put(h.twn[i], &d.tables.twn[i]));
    }
    PWF_HIP(hipEventCreateWithFlags(&d.copied, hipEventDisableTiming));
    d.base = base;
    d.tables.ready = true;
    d.ready = true;
  }
  *out = &d;
  return PWF_OK;
}

}  // namespace

extern "C" {

size_t pwf_loss_grad_noalloc_limit(void) { return kScratchBytes - kScratchTableBytes; }

pwf_status pwf_loss_grad_noalloc(const pwf_problem* problems, int32_t n, const void* const* psi,
                                 const float* const* y, void* const* grad_out, double* loss_out, void* stream) {
  PWF_TRY(validate_loss_grad(problems, n, psi, y, grad_out));
  if (n > kScratchMaxInst) return PWF_ERR_SCRATCH;
  const Layout L = make_loss_grad_layout(problems, n);
  if (L.total > kScratchBytes - kScratchTableBytes) return PWF_ERR_SCRATCH;
  std::lock_guard<std::mutex> lk(g_mu);
  ScratchDevice* d;
  PWF_TRY(scratch_for_current(&d));
  hipStream_t st = (hipStream_t)stream;
  char* ws = d->base + kScratchTableBytes;
  const Batch B = group(problems, n);
  // the previous call's copy must have read host_desc before it is rewritten
  PWF_HIP(hipEventSynchronize(d->copied));
  loss_grad_descriptors(problems, n, B, psi, y, grad_out, loss_out, ws, L, d->host_desc);
  PWF_HIP(pwf::launch_fill_zero(ws + L.status, 16, st));
  PWF_HIP(hipMemcpyAsync(ws + L.desc, d->host_desc, sizeof(Inst) * n, hipMemcpyHostToDevice, st));
  PWF_HIP(hipEventRecord(d->copied, st));
  return loss_grad_sequence(Launcher{d->tables, ws, L, B, st}, n);
}

pwf_status pwf_sync_status(void* workspace, void* stream) {
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return PWF_ERR_WORKSPACE;
  PWF_HIP(hipStreamSynchronize((hipStream_t)stream));
  int32_t flag = 0;
  PWF_HIP(hipMemcpy(&flag, workspace, sizeof(flag), hipMemcpyDeviceToHost));
  return (flag & 1) ? PWF_ERR_NONFINITE : PWF_OK;
}

void pwf_finalize(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (Context& c : g_ctx) {
    if (!c.ready) continue;
    for (auto& kv : c.graphs) (void)hipGraphExecDestroy(kv.second);
    c.graphs.clear();
    for (float2*& t : c.tw) {
      if (t) (void)hipFree(t);
      t = nullptr;
    }
    for (float2*& t : c.twc) {
      if (t) (void)hipFree(t);
      t = nullptr;
    }
    for (float2*& t : c.twn) {
      if (t) (void)hipFree(t);
      t = nullptr;
    }
    for (float2*& t : c.twa) {
      if (t) (void)hipFree(t);
      t = nullptr;
    }
    for (float2*& t : c.twa2) {
      if (t) (void)hipFree(t);
      t = nullptr;
    }
    if (c.beta) (void)hipFree(c.beta);
    c.beta = nullptr;
    for (int i = 0; i < Context::kSlots; ++i) {
      if (c.stage_ev[i]) (void)hipEventSynchronize(c.stage_ev[i]);
      if (c.stage[i]) (void)hipHostFree(c.stage[i]);
      c.stage[i] = nullptr;
      c.stage_bytes[i] = 0;
      if (c.stage_ev[i]) (void)hipEventDestroy(c.stage_ev[i]);
      c.stage_ev[i] = nullptr;
    }
    for (hipStream_t& f : c.fork)
      if (f) (void)hipStreamDestroy(f);
    for (hipEvent_t& e : c.fork_ev)
      if (e) (void)hipEventDestroy(e);
    if (c.ev_in) (void)hipEventDestroy(c.ev_in);
    if (c.ev_out) (void)hipEventDestroy(c.ev_out);
    if (c.side) (void)hipStreamDestroy(c.side);
    c = Context();
  }
}

}  // extern "C"
