// Wave-wide reductions on DPP moves (gfx950, 64-lane waves), shared by the
// LU panel kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace hexla {
namespace k {

// One step of a wave-wide argmax (largest a, lowest i on ties): lanes whose
// DPP source lies outside the row, or whose row is masked off, keep their
// own pair.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void argmax_step(double& a, int& i) {
  const int lo = __double2loint(a), hi = __double2hiint(a);
  const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, 0xF, false);
  const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, 0xF, false);
  const int i2 = __builtin_amdgcn_update_dpp(i, i, CTRL, ROW_MASK, 0xF, false);
  const double a2 = __hiloint2double(hi2, lo2);
  const bool take = (a2 > a) | ((a2 == a) & (i2 < i));  // selects, no branch
  a = take ? a2 : a;
  i = take ? i2 : i;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void argmax_step(float& a, int& i) {
  const int b = __float_as_int(a);
  const float a2 = __int_as_float(__builtin_amdgcn_update_dpp(b, b, CTRL, ROW_MASK, 0xF, false));
  const int i2 = __builtin_amdgcn_update_dpp(i, i, CTRL, ROW_MASK, 0xF, false);
  const bool take = (a2 > a) | ((a2 == a) & (i2 < i));
  a = take ? a2 : a;
  i = take ? i2 : i;
}

__device__ __forceinline__ double lane63(double a) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(a), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(a), 63);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane63(float a) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a), 63));
}

// Argmax over the 64 lanes of a wave (every lane active), returned to every
// lane in scalar registers: row shifts 1, 2, 4, 8 leave each row's result in
// its lane 15, the row broadcasts 15 and 31 combine the rows into lane 63,
// which is read back.
template <typename T>
__device__ __forceinline__ void wave_argmax(T& a, int& i) {
  argmax_step<0x111, 0xF>(a, i);  // row_shr:1
  argmax_step<0x112, 0xF>(a, i);  // row_shr:2
  argmax_step<0x114, 0xF>(a, i);  // row_shr:4
  argmax_step<0x118, 0xF>(a, i);  // row_shr:8
  argmax_step<0x142, 0xA>(a, i);  // row_bcast:15 into rows 1 and 3
  argmax_step<0x143, 0xC>(a, i);  // row_bcast:31 into rows 2 and 3
  i = __builtin_amdgcn_readlane(i, 63);
  a = lane63(a);
}

// |x| as an unsigned key pair that orders like |x|: the high word of the bit
// pattern plus one, then the low word (FP64 only). NaN gets (0, 0), which
// also stands for "no candidate", so it ranks below every number.
__device__ __forceinline__ void abs_key(float x, unsigned& h, unsigned& l) {
  const unsigned b = __float_as_uint(x) & 0x7fffffffu;
  h = b > 0x7f800000u ? 0u : b + 1u;
  l = 0u;
}
__device__ __forceinline__ void abs_key(double x, unsigned& h, unsigned& l) {
  const unsigned hb = unsigned(__double2hiint(x)) & 0x7fffffffu, lb = unsigned(__double2loint(x));
  const bool nan = hb > 0x7ff00000u || (hb == 0x7ff00000u && lb != 0u);
  h = nan ? 0u : hb + 1u;
  l = nan ? 0u : lb;
}

// Wave-wide max of unsigned values and min of ints, returned to every lane.
// The DPP source is the operation's identity where a lane has no source
// (bound_ctrl zero for max, old = INT_MAX for min), so the compiler folds
// each move into one v_max_u32_dpp / v_min_i32_dpp.
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ unsigned max_step(unsigned a) {
  return max(a, unsigned(__builtin_amdgcn_update_dpp(0u, a, CTRL, ROW_MASK, 0xF, BOUND)));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int min_step(int a) {
  return min(a, __builtin_amdgcn_update_dpp(0x7fffffff, a, CTRL, ROW_MASK, 0xF, false));
}
__device__ __forceinline__ unsigned wave_max_u32(unsigned a) {
  a = max_step<0x111, 0xF, true>(a);
  a = max_step<0x112, 0xF, true>(a);
  a = max_step<0x114, 0xF, true>(a);
  a = max_step<0x118, 0xF, true>(a);
  a = max_step<0x142, 0xA, false>(a);
  a = max_step<0x143, 0xC, false>(a);
  return __builtin_amdgcn_readlane(a, 63);
}
__device__ __forceinline__ int wave_min_i32(int a) {
  a = min_step<0x111, 0xF>(a);
  a = min_step<0x112, 0xF>(a);
  a = min_step<0x114, 0xF>(a);
  a = min_step<0x118, 0xF>(a);
  a = min_step<0x142, 0xA>(a);
  a = min_step<0x143, 0xC>(a);
  return __builtin_amdgcn_readlane(a, 63);
}

}  // namespace k
}  // namespace hexla
