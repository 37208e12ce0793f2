// Sweeps of the iteration launched once over several size classes of an
// uneven batch.  Every class keeps its own descriptors and launch arguments;
// each workgroup finds its class from the block offsets and runs that side's
// sweep body.  Row bodies: 256 threads on every side (512: 32 x 8 rows; 1024
// and 2048: the 64- and 128-lane plans, 4 and 2 rows), rows paired for the
// split column transforms of these sides; column bodies: 512 threads (one
// half of the split transform: 256, 512 and 1024 points, 32, 16 and 8
// columns).  The LDS pools below are the largest each body needs, so every
// class runs at the occupancy of its own kernel or close to it.
#include "pwf_sweeps.h"

namespace pwf {

namespace {

template <int OP>
constexpr int multi_row_exchange() {
  return cmax(cmax(RowLds<512, OP, 0>::kExchange, RowLds<1024, OP, 1>::kExchange),
              cmax(cmax(RowLds<1024, OP, 2>::kExchange, RowLds<2048, OP, 1>::kExchange),
                   RowLds<2048, OP, 2>::kExchange));
}
template <int OP>
constexpr int multi_row_twiddles() {
  return cmax(cmax(RowLds<512, OP, 0>::kTwiddles, RowLds<1024, OP, 1>::kTwiddles),
              cmax(cmax(RowLds<1024, OP, 2>::kTwiddles, RowLds<2048, OP, 1>::kTwiddles),
                   RowLds<2048, OP, 2>::kTwiddles));
}
// Register bounds: every body alone fits them (the row bodies in 168
// registers, the column bodies in 128), and the bound keeps the merged
// kernel from exceeding them: at 134 registers a 512-thread column
// workgroup would run alone on its CU.
template <int OP>
constexpr int multi_row_waves() { return OP == ROW_INTENSITY ? 4 : 3; }

template <int OP>
__global__ void __launch_bounds__(256, (multi_row_waves<OP>())) row_sweep_multi(MultiSweep M) {
  __shared__ float2 lds[multi_row_exchange<OP>()];
  __shared__ float2 twl[multi_row_twiddles<OP>()];
  const int b = xcd_contiguous<false>(blockIdx.x, gridDim.x);
  int c = 0;
  while (c + 1 < M.nc && b >= M.first[c + 1]) ++c;
  const int lb = b - M.first[c];
  // (the merged sides all come with split column transforms: paired rows)
  const int key = M.side[c] * 4 + M.plan[c];
  if (key == 512 * 4 + 0) row_body<512, OP, 0, true>(M.s[c], lb, lds, twl);
  else if (key == 1024 * 4 + 1) row_body<1024, OP, 1, true>(M.s[c], lb, lds, twl);
  else if (key == 1024 * 4 + 2) row_body<1024, OP, 2, true>(M.s[c], lb, lds, twl);
  else if (key == 2048 * 4 + 1) row_body<2048, OP, 1, true>(M.s[c], lb, lds, twl);
  else if (key == 2048 * 4 + 2) row_body<2048, OP, 2, true>(M.s[c], lb, lds, twl);
}

// column tile of the merged kernel's body on side N: 512 threads
template <int N> constexpr int multi_w() { return 512 / ColSweepCfg<N>::T; }
constexpr int kMultiColExchange = cmax(cmax(ColLds<512, multi_w<512>()>::kExchange, ColLds<1024, multi_w<1024>()>::kExchange),
                                       ColLds<2048, multi_w<2048>()>::kExchange);
constexpr int kMultiColTwiddles = cmax(cmax(ColLds<512, multi_w<512>()>::kTwiddles, ColLds<1024, multi_w<1024>()>::kTwiddles),
                                       ColLds<2048, multi_w<2048>()>::kTwiddles);
constexpr int kMultiYTable = cmax(cmax(ColLds<512, multi_w<512>()>::kYTable, ColLds<1024, multi_w<1024>()>::kYTable),
                                  ColLds<2048, multi_w<2048>()>::kYTable);

template <int OP>
__global__ void __launch_bounds__(512, 4) col_sweep_multi(MultiSweep M) {
  __shared__ float2 lds[kMultiColExchange];
  __shared__ float2 twl[kMultiColTwiddles];
  __shared__ float2 qyl[col_op_ystage(OP) ? kMultiYTable : 1];
  const int b = xcd_contiguous<true>(blockIdx.x, gridDim.x);
  int c = 0;
  while (c + 1 < M.nc && b >= M.first[c + 1]) ++c;
  const int lb = b - M.first[c];
  switch (M.side[c]) {
    case 512: col_body<512, multi_w<512>(), OP>(M.s[c], lb, lds, twl, qyl); break;
    case 1024: col_body<1024, multi_w<1024>(), OP>(M.s[c], lb, lds, twl, qyl); break;
    case 2048: col_body<2048, multi_w<2048>(), OP>(M.s[c], lb, lds, twl, qyl); break;
    default: break;
  }
}

}  // namespace

bool multi_row_supported(int nx, int ny, int plan) {
  // the merged row bodies pair their rows: classes whose column transform is split
  if (!col_split_n(ny)) return false;
  return (nx == 512 && plan == 0) || ((nx == 1024 || nx == 2048) && (plan == 1 || plan == 2));
}

int multi_col_width(int ny) {
  return ny == 512 ? multi_w<512>() : ny == 1024 ? multi_w<1024>() : ny == 2048 ? multi_w<2048>() : 0;
}

hipError_t launch_row_multi(int op, int nblocks, const MultiSweep& M, hipStream_t st) {
  const dim3 grid(nblocks), block(256);
  switch (op) {
#define PWF_CASE(o) case o: hipLaunchKernelGGL(row_sweep_multi<o>, grid, block, 0, st, M); break;
    PWF_CASE(ROW_PSI_UPDATE) PWF_CASE(ROW_PSI_UPDATE_CORR) PWF_CASE(ROW_MUL_T) PWF_CASE(ROW_INTENSITY)
    PWF_CASE(ROW_BACKBLUR) PWF_CASE(ROW_MUL_CONJ_T) PWF_CASE(ROW_GRAD)
#undef PWF_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_col_multi(int op, int nblocks, const MultiSweep& M, hipStream_t st) {
  const dim3 grid(nblocks), block(512);
  switch (op) {
#define PWF_CASE(o) case o: hipLaunchKernelGGL(col_sweep_multi<o>, grid, block, 0, st, M); break;
    PWF_CASE(COL_CHIRP1) PWF_CASE(COL_CHIRP2) PWF_CASE(COL_BLUR_LOSS) PWF_CASE(COL_CHIRP2_CONJ)
    PWF_CASE(COL_CHIRP1_CONJ) PWF_CASE(COL_NESTEROV)
#undef PWF_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pwf
