// Wavefront-wide reductions for 64-lane waves: DPP moves within rows of 16
// lanes, then two lane shuffles across the rows.
#pragma once
#include <hip/hip_runtime.h>

namespace mkpw {

// lane i takes lane i^1 (DPP quad permutation 1,0,3,2), i^2 (2,3,0,1), and the
// mirrors within 8 and 16 lanes
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// sum over the 64 lanes of a wavefront, returned on every lane: four DPP steps
// give each 16-lane row its sum, two lane shuffles combine the rows
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp<0xB1>(v);   // quad_perm 1,0,3,2
  v += dpp<0x4E>(v);   // quad_perm 2,3,0,1
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

}  // namespace mkpw
