// Sweep kernels for grid side 256.
#include "pwf_sweeps.h"

namespace pwf {
template hipError_t launch_row_n<256>(int, int, int, const Sweep&, hipStream_t);
template hipError_t launch_col_n<256>(int, int, int, const Sweep&, hipStream_t);
template hipError_t plain_rows_n<256>(int, const float2*, float2*, int, const float2*, hipStream_t);
template hipError_t plain_cols_n<256>(int, float2*, int, const float2*, int, size_t, hipStream_t);
template int plan_twiddles_n<256>(int, float2*);
}  // namespace pwf
