// Row transforms shared by the pair-density and full-grid FFT kernels: a line
// of N points is spread over L lanes with M = N / L points each (sample l + L*s
// in lane l); a register FFT of M points is followed by an L-point DFT across
// the lanes (DPP / swizzle exchanges).
#pragma once
#include "bse_internal.h"

namespace bse {

template <int N>
struct Split;  // N = L * M: L lanes per row, M points per lane (register FFT)
template <> struct Split<8>  { static constexpr int L = 2, M = 4; };
template <> struct Split<12> { static constexpr int L = 2, M = 6; };
template <> struct Split<16> { static constexpr int L = 2, M = 8; };
template <> struct Split<24> { static constexpr int L = 2, M = 12; };
template <> struct Split<32> { static constexpr int L = 2, M = 16; };
template <> struct Split<48> { static constexpr int L = 4, M = 12; };
template <> struct Split<64> { static constexpr int L = 4, M = 16; };
template <> struct Split<96> { static constexpr int L = 8, M = 12; };

// Split of a pass-2 line: the kept window of pass 1 leaves few lines, so more
// lanes go to each line.
template <int N>
struct SplitB {
  static constexpr int L = (N == 16 || N == 24 || N == 32 || N == 48 || N == 64) ? 4 : Split<N>::L;
  static constexpr int M = N / L;
};

template <int L>
__device__ __forceinline__ int bitrev(int l) {
  if constexpr (L == 2) return l;
  if constexpr (L == 4) return ((l & 1) << 1) | (l >> 1);
  if constexpr (L == 8) return ((l & 1) << 2) | (l & 2) | (l >> 2);
  return 0;
}

// value of lane (lane ^ H) for H in {1, 2, 4}; all lanes active
template <int H>
__device__ __forceinline__ double xor_lane(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  int rlo, rhi;
  if constexpr (H == 1) {  // quad_perm [1,0,3,2]
    rlo = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false);
    rhi = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false);
  } else if constexpr (H == 2) {  // quad_perm [2,3,0,1]
    rlo = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false);
    rhi = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false);
  } else {  // swizzle, bit-mask mode: and 0x1F, xor H
    static_assert(H == 4 || H == 8 || H == 16, "xor distance");
    rlo = __builtin_amdgcn_ds_swizzle(lo, (H << 10) | 0x1F);
    rhi = __builtin_amdgcn_ds_swizzle(hi, (H << 10) | 0x1F);
  }
  return __hiloint2double(rhi, rlo);
}

template <int H>
__device__ __forceinline__ double2 xor_lane2(double2 v) {
  return make_double2(xor_lane<H>(v.x), xor_lane<H>(v.y));
}

// One radix-2 decimation-in-frequency stage of an L-point DFT across lanes,
// branch free: lower lane x + o, upper lane (o - x) * w.
template <int M, int H>
__device__ __forceinline__ void xlane_stage(double2 (&x)[M], int l, const double2* tw, int N) {
  const int p = l & (2 * H - 1);
  const double s = p >= H ? -1.0 : 1.0;
  if constexpr (H == 1) {
#pragma unroll
    for (int f = 0; f < M; ++f) {
      const double2 o = xor_lane2<1>(x[f]);
      x[f] = make_double2(fma(s, x[f].x, o.x), fma(s, x[f].y, o.y));
    }
  } else {
    const bool upper = p >= H;
    const double2 wt = tw[(p & (H - 1)) * (N / (2 * H))];
    const double2 w = csel(upper, wt, make_double2(1.0, 0.0));
#pragma unroll
    for (int f = 0; f < M; ++f) {
      const double2 o = xor_lane2<H>(x[f]);
      const double2 t = make_double2(fma(s, x[f].x, o.x), fma(s, x[f].y, o.y));
      x[f] = cmul(t, w);
    }
  }
}

// L-point DFT across the L lanes of a row group for each of the M values a
// lane holds; afterwards lane l holds output index bitrev(l).
template <int L, int M>
__device__ __forceinline__ void cross_lane_dft(double2 (&x)[M], int l, const double2* tw, int N) {
  if constexpr (L >= 8) xlane_stage<M, 4>(x, l, tw, N);
  if constexpr (L >= 4) xlane_stage<M, 2>(x, l, tw, N);
  if constexpr (L >= 2) xlane_stage<M, 1>(x, l, tw, N);
}

// Row transform: x holds samples l + L*s (s < M) of a length-N row; afterwards
// slot fft_pos<M>(f') holds output f' + M * bitrev(l).  tw[t] = exp(-2 pi i t / N).
template <int N, int L, int M>
__device__ __forceinline__ void row_fft(double2 (&x)[M], int l, const double2* tw) {
  static_assert(L * M == N, "row split");
  reg_fft<M, 1, 0>(x);
  if constexpr (L == 2) {
    // twiddle exp(-2 pi i l f'/N), l in {0, 1}: a compile-time constant per f'
    static_for<1, M>([&](auto fc) {
      constexpr int f = decltype(fc)::value, p = fft_pos<M>(f);
      const double2 y = cmul_root<N, f>(x[p]);
      x[p] = csel(l != 0, y, x[p]);
    });
  } else if constexpr (L > 2) {
    static_for<1, M>([&](auto fc) {
      constexpr int f = decltype(fc)::value, p = fft_pos<M>(f);
      x[p] = cmul(x[p], tw[(l * f) % N]);
    });
  }
  cross_lane_dft<L, M>(x, l, tw, N);
}

}  // namespace bse
