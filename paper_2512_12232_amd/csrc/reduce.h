// Wavefront and block sums in a fixed order (DPP lane moves), shared by the solver
// kernels.
#pragma once

#include "mfp_internal.h"

namespace mfp {

// A double moved across lanes by one DPP pattern (lanes of rows outside ROWS get 0).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over the wavefront; every lane receives the same total.  All 64 lanes must be
// active.  DPP steps within each row of 16 lanes (quad swaps, half-row and row
// mirrors: every lane then holds its row's sum), then the row sums are combined
// towards lane 63 with the row broadcasts, (r0 + r1) + (r2 + r3), and lane 63's value
// is read out.  A fixed order, so results are reproducible; each step is a register
// move instead of the round trip through the LDS crossbar that a shuffle takes.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1, 0xf>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_move<0x4E, 0xf>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_move<0x141, 0xf>(v);  // row_half_mirror
  v += dpp_move<0x140, 0xf>(v);  // row_mirror
  v += dpp_move<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Sum of N per-wavefront values held in LDS at s[0], s[4], s[8], ... (four values per
// wavefront), as a balanced tree in a fixed order: (w0 + w1) + (w2 + w3), and so on.
template <int N>
__device__ __forceinline__ double wave_tree(const double* s) {
  if constexpr (N == 1)
    return s[0];
  else
    return wave_tree<N / 2>(s) + wave_tree<N / 2>(s + 4 * (N / 2));
}

// Sum over a 256-thread block; every thread receives the total.  Fixed reduction
// order, so results are reproducible run to run.
__device__ __forceinline__ double block_sum(double v, double* s_red) {
  v = wave_sum(v);
  const int tid = threadIdx.x;
  __syncthreads();
  if ((tid & 63) == 0) s_red[tid >> 6] = v;
  __syncthreads();
  const double t = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
  return t;
}

}  // namespace mfp
