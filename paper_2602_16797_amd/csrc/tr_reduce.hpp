// Wave reductions by butterfly stages on gfx950 lane swaps and DPP, shared
// by the A-stream pass and the column-wave TSQR.
#pragma once

#include "common.hpp"

namespace rl {

// Butterfly stages of the reductions below.  Across rows of 16 lanes (o = 32,
// 16) the exchange uses the gfx950 lane swaps: permlane32_swap(x, y) leaves
// x = [x(0:31), y(0:31)] and y = [x(32:63), y(32:63)], and permlane16_swap does
// the same with 16-lane groups inside each half, so with x the lower-half
// values and y the upper-half values of a stage, x + y is in every lane the
// sum that lane keeps, with no selects and no LDS traffic.  Inside a row
// (o = 8, 4, 2, 1) the partner is read with a DPP lane permutation (row
// mirror, half-row mirror, quad permutations); its partner differs in the
// stage's bit and agrees in every higher bit, which is all the reductions rely
// on.
template <int O>
__device__ inline void lane_swap(double& x, double& y) {
  static_assert(O == 32 || O == 16, "lane swaps exist for 32 and 16");
  if constexpr (O == 32) {
    auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(y), false, false);
    auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(y), false, false);
    x = __hiloint2double((int)hi[0], (int)lo[0]);
    y = __hiloint2double((int)hi[1], (int)lo[1]);
  } else {
    auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(y), false, false);
    auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(y), false, false);
    x = __hiloint2double((int)hi[0], (int)lo[0]);
    y = __hiloint2double((int)hi[1], (int)lo[1]);
  }
}

template <int O>
__device__ inline double dpp_partner(double v) {
  if constexpr (O == 8) return dpp_d<DPP_ROW_MIRROR>(v);
  else if constexpr (O == 4) return dpp_d<DPP_ROW_HALF_MIRROR>(v);
  else if constexpr (O == 2) return dpp_d<DPP_QUAD_2301>(v);
  else return dpp_d<DPP_QUAD_1032>(v);
}

// one transposed stage: values k < H pair with k + H; lanes with bit log2(O)
// clear keep the lower half
template <int O, int H, int V2>
__device__ inline void tr_stage_dot2(double (&s)[V2], double (&e)[V2], int lane) {
#pragma unroll
  for (int k = 0; k < H; ++k) {
    double t;
    if constexpr (O >= 16) {
      double xs = s[k], ys = s[k + H], xe = e[k], ye = e[k + H];
      lane_swap<O>(xs, ys);
      lane_swap<O>(xe, ye);
      two_sum(xs, ys, s[k], t);
      e[k] = (xe + ye) + t;
    } else {
      const bool hi = (lane & O) != 0;
      const double ks = hi ? s[k + H] : s[k];
      const double ke = hi ? e[k + H] : e[k];
      const double rs = dpp_partner<O>(hi ? s[k] : s[k + H]);
      const double re = dpp_partner<O>(hi ? e[k] : e[k + H]);
      two_sum(ks, rs, s[k], t);
      e[k] = (ke + re) + t;
    }
  }
}

// all-reduce stage of one (sum, error) pair
template <int O>
__device__ inline void ar_stage_dot2(double& s, double& e) {
  double rs, re;
  if constexpr (O >= 16) {
    double xs = s, ys = s, xe = e, ye = e;
    lane_swap<O>(xs, ys);
    lane_swap<O>(xe, ye);
    double t;
    two_sum(xs, ys, s, t);
    e = (xe + ye) + t;
  } else {
    rs = dpp_partner<O>(s);
    re = dpp_partner<O>(e);
    double t;
    two_sum(s, rs, s, t);
    e = (e + re) + t;
  }
}

template <int O>
__device__ inline double ar_stage_plain(double v) {
  if constexpr (O >= 16) {
    double x = v, y = v;
    lane_swap<O>(x, y);
    return x + y;
  } else {
    return v + dpp_partner<O>(v);
  }
}

template <int O, int H, int V2>
__device__ inline void tr_stage_plain(double (&s)[V2], int lane) {
#pragma unroll
  for (int k = 0; k < H; ++k) {
    if constexpr (O >= 16) {
      double x = s[k], y = s[k + H];
      lane_swap<O>(x, y);
      s[k] = x + y;
    } else {
      const bool hi = (lane & O) != 0;
      const double ks = hi ? s[k + H] : s[k];
      s[k] = ks + dpp_partner<O>(hi ? s[k] : s[k + H]);
    }
  }
}

// Compensated transpose-reduction of V2 = 2^LOG2V (sum, error) pairs over the
// wave: stage st halves the values each lane carries (bit 5 - st of the lane
// picks the half); the remaining stages all-reduce one pair.  On return lane l
// holds in (s[0], e[0]) the wave sum of value tr_src_lane^-1(l).
template <int V2, int LOG2V>
__device__ inline void tr_reduce_dot2(double (&s)[V2], double (&e)[V2], int lane) {
  if constexpr (LOG2V >= 1) tr_stage_dot2<32, V2 / 2, V2>(s, e, lane);
  if constexpr (LOG2V >= 2) tr_stage_dot2<16, V2 / 4, V2>(s, e, lane);
  if constexpr (LOG2V >= 3) tr_stage_dot2<8, V2 / 8, V2>(s, e, lane);
  if constexpr (LOG2V >= 4) tr_stage_dot2<4, V2 / 16, V2>(s, e, lane);
  if constexpr (LOG2V >= 5) tr_stage_dot2<2, V2 / 32, V2>(s, e, lane);
  if constexpr (LOG2V >= 6) tr_stage_dot2<1, V2 / 64, V2>(s, e, lane);
  if constexpr (LOG2V < 1) ar_stage_dot2<32>(s[0], e[0]);
  if constexpr (LOG2V < 2) ar_stage_dot2<16>(s[0], e[0]);
  if constexpr (LOG2V < 3) ar_stage_dot2<8>(s[0], e[0]);
  if constexpr (LOG2V < 4) ar_stage_dot2<4>(s[0], e[0]);
  if constexpr (LOG2V < 5) ar_stage_dot2<2>(s[0], e[0]);
  if constexpr (LOG2V < 6) ar_stage_dot2<1>(s[0], e[0]);
}

template <int V2, int LOG2V>
__device__ inline void tr_reduce_plain(double (&s)[V2], int lane) {
  if constexpr (LOG2V >= 1) tr_stage_plain<32, V2 / 2, V2>(s, lane);
  if constexpr (LOG2V >= 2) tr_stage_plain<16, V2 / 4, V2>(s, lane);
  if constexpr (LOG2V >= 3) tr_stage_plain<8, V2 / 8, V2>(s, lane);
  if constexpr (LOG2V >= 4) tr_stage_plain<4, V2 / 16, V2>(s, lane);
  if constexpr (LOG2V >= 5) tr_stage_plain<2, V2 / 32, V2>(s, lane);
  if constexpr (LOG2V >= 6) tr_stage_plain<1, V2 / 64, V2>(s, lane);
  if constexpr (LOG2V < 1) s[0] = ar_stage_plain<32>(s[0]);
  if constexpr (LOG2V < 2) s[0] = ar_stage_plain<16>(s[0]);
  if constexpr (LOG2V < 3) s[0] = ar_stage_plain<8>(s[0]);
  if constexpr (LOG2V < 4) s[0] = ar_stage_plain<4>(s[0]);
  if constexpr (LOG2V < 5) s[0] = ar_stage_plain<2>(s[0]);
  if constexpr (LOG2V < 6) s[0] = ar_stage_plain<1>(s[0]);
}

// lane holding value index k after the transpose-reduction
template <int LOG2V>
__device__ constexpr int tr_src_lane(int k) {
  int l = 0;
  for (int st = 0; st < LOG2V; ++st) l |= ((k >> (LOG2V - 1 - st)) & 1) << (5 - st);
  return l;
}

}  // namespace rl
