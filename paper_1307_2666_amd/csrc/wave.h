// Wave-wide reductions shared by the QR kernels.  Internal, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

namespace hif {

constexpr int kRs = 32;  // values reduced at once by wave_rs32

// Sum of p[c] over the 64 lanes for all kRs = 32 indices at once
// (reduce-scatter: at each step a lane keeps one half of its values, sends the
// other half to its partner and adds what it receives).  Returns the total of
// index lane >> 1; p is destroyed.
template <int H>
__device__ __forceinline__ void rs_step(double (&p)[kRs], int lane) {
  const bool up = (lane & (2 * H)) != 0;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double send = up ? p[i] : p[i + H];
    const double keep = up ? p[i + H] : p[i];
    p[i] = keep + __shfl_xor(send, 2 * H, 64);
  }
}
// Pair sums across lane halves with the gfx950 lane-swap instructions:
// (a, b) = this lane's values of indices i and i + h; the result is the sum
// of index i over lanes l and l ^ 2h for the lower lane of each pair and of
// index i + h for the upper one (h = 16: halves of the wave, h = 8: rows of
// 16 lanes).  The sum does not depend on which output holds which half.
template <int H>
__device__ __forceinline__ double swap_pair_sum(double a, double b) {
  const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
  const unsigned alo = unsigned(ua), ahi = unsigned(ua >> 32), blo = unsigned(ub), bhi = unsigned(ub >> 32);
  unsigned r0l, r1l, r0h, r1h;
  if constexpr (H == 16) {
    const auto rl = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    r0l = rl[0]; r1l = rl[1]; r0h = rh[0]; r1h = rh[1];
  } else {
    const auto rl = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    r0l = rl[0]; r1l = rl[1]; r0h = rh[0]; r1h = rh[1];
  }
  const double r0 = __longlong_as_double((static_cast<long long>(r0h) << 32) | r0l);
  const double r1 = __longlong_as_double((static_cast<long long>(r1h) << 32) | r1l);
  return r0 + r1;
}

__device__ __forceinline__ double wave_rs32(double (&p)[kRs]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 16; ++i) p[i] = swap_pair_sum<16>(p[i], p[i + 16]);
#pragma unroll
  for (int i = 0; i < 8; ++i) p[i] = swap_pair_sum<8>(p[i], p[i + 8]);
  rs_step<4>(p, lane);
  rs_step<2>(p, lane);
  rs_step<1>(p, lane);
  return p[0] + __shfl_xor(p[0], 1, 64);
}

// Sum of p[c] over the 64 lanes for all 8 indices at once, the same
// reduce-scatter on 8 values: the total of index lane >> 3 (held by all 8
// lanes of the group); p is destroyed.
__device__ __forceinline__ double wave_rs8(double (&p)[8]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 4; ++i) p[i] = swap_pair_sum<16>(p[i], p[i + 4]);  // index + 4 on the upper half
#pragma unroll
  for (int i = 0; i < 2; ++i) p[i] = swap_pair_sum<8>(p[i], p[i + 2]);  // index + 2 on odd rows of 16
  const bool up = (lane & 8) != 0;
  double t = (up ? p[1] : p[0]) + __shfl_xor(up ? p[0] : p[1], 8, 64);  // index + 1 on lanes with bit 3
  t += __shfl_xor(t, 4, 64);
  t += __shfl_xor(t, 2, 64);
  t += __shfl_xor(t, 1, 64);
  return t;
}

}  // namespace hif
