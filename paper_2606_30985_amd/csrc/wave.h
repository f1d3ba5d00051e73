// Wave-level reductions shared by the kernels (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace hpt {

// one DPP move of a double (both 32-bit halves); lanes without a source in
// the pattern, or outside row_mask, read 0
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_move(double v) {
  int lo, hi;
  __builtin_memcpy(&lo, &v, 4);
  __builtin_memcpy(&hi, (const char*)&v + 4, 4);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, false);
  double r;
  __builtin_memcpy(&r, &lo, 4);
  __builtin_memcpy((char*)&r + 4, &hi, 4);
  return r;
}

// sum over the 64 lanes of a wave, the same value returned to every lane;
// all lanes must be active.  DPP row shifts build each 16-lane row's sum in
// its lane 15, two row broadcasts carry the rows into lane 63, which is read
// out: a fixed order (deterministic), shorter latency than a permute-based
// butterfly (used in the float64 factorisations and the measurement
// reductions, each worth 1% on the 10x10 chi=100 layer).
__device__ inline double wave_sum(double v) {
  v += dpp_move<0x111, 0xf>(v);   // row_shr:1
  v += dpp_move<0x112, 0xf>(v);   // row_shr:2
  v += dpp_move<0x114, 0xf>(v);   // row_shr:4
  v += dpp_move<0x118, 0xf>(v);   // row_shr:8
  v += dpp_move<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  int lo, hi;
  __builtin_memcpy(&lo, &v, 4);
  __builtin_memcpy(&hi, (const char*)&v + 4, 4);
  lo = __builtin_amdgcn_readlane(lo, 63);
  hi = __builtin_amdgcn_readlane(hi, 63);
  double r;
  __builtin_memcpy(&r, &lo, 4);
  __builtin_memcpy((char*)&r + 4, &hi, 4);
  return r;
}

}  // namespace hpt
