// Tile engines of the MFMA contractions: a (64 MR) x 64 complex output tile
// per 256-thread workgroup (4 waves, (32 MR) x 32 each; MR = 1 or 2),
// operands staged through LDS.
//   tile_gemm     FP64: four real v_mfma_f64_16x16x4 products per step
//   tile_gemm_mx  split operands (FP32 or BF16 hi + lo), FP32 accumulation
#pragma once
#include <hip/hip_bf16.h>

#include "../../include/bse.h"
#include "bse_internal.h"

namespace bse {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int TM = 64, TN = 64, KC = 16;

// (64 MR) x 64 complex tile of C = op(A) * B with op(A) = conj(A) if CONJ_A.
// A[m][k] = Am[(a_off + m) * lda + k]   (A_T: Am[k * lda + a_off + m]), valid a_off + m < a_lim;
// B[k][n] = Bm[k * ldb + b_off + n]     (B_T: Bm[(b_off + n) * ldb + k]), valid b_off + n < b_lim;
// valid k < K.  The result lands in cre/cim (f64 MFMA accumulator layout).
// ZERO = false adds to the accumulators instead of starting from zero.
// B_MAP (B not transposed): B[k][n] = Bm[bmap[k] * ldb + bmap[n]], conjugated
// when bconj (a matrix read through a permutation of its rows and columns);
// bmap holds at least max(K, b_lim) entries, or is null (B read directly, so
// that one instantiation, with one set of LDS arrays, serves both).
// Each thread stages 4 elements of A and 4 of B per K chunk; the next chunk's
// elements are loaded into registers while the MFMAs consume the current one
// (out-of-range elements are read from the array start and replaced by zero,
// so the loads need no branches).
// G3: three real products per complex step instead of four (Gauss's form:
// P1 = sum a_r b_r, P2 = sum a_i b_i, P3 = sum (a_r + a_i)(b_r + b_i), then
// Re = P1 - P2, Im = P3 - P1 - P2), accumulated separately over K and
// combined at the end; three quarters of the MFMA work, one extra addition per
// operand fragment.  Im then carries rounding of the order of the unit
// roundoff times sum |a||b| rather than times |Im| (starting from zero only).
template <bool CONJ_A, bool B_T, bool A_T = false, bool ZERO = true, bool B_MAP = false, int MR = 1, bool G3 = false>
__device__ __forceinline__ void tile_gemm(const double2* __restrict__ A, int lda, int a_off, int a_lim,
                                          const double2* __restrict__ B, int ldb, int b_off, int b_lim, int K,
                                          d4 (&cre)[2 * MR][2], d4 (&cim)[2 * MR][2],
                                          const int* __restrict__ bmap = nullptr, bool bconj = false) {
  static_assert(!(B_MAP && B_T), "the mapped B operand is read untransposed");
  static_assert(MR == 1 || MR == 2, "64 or 128 rows per tile");
  static_assert(ZERO || !G3, "the three-product form starts from zero");
  d4 p2[G3 ? 2 * MR : 1][2];  // G3: sum a_i b_i (cre holds P1, cim P3 until the end)
  if constexpr (G3) {
#pragma unroll
    for (int i = 0; i < 2 * MR; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) p2[i][j] = d4{0, 0, 0, 0};
  }
  __shared__ double As_re[TM * MR][KC + 1], As_im[TM * MR][KC + 1];
  __shared__ double Bs_re[KC][TN + 1], Bs_im[KC][TN + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  if constexpr (ZERO) {
#pragma unroll
    for (int i = 0; i < 2 * MR; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        cre[i][j] = d4{0, 0, 0, 0};
        cim[i][j] = d4{0, 0, 0, 0};
      }
  }
  // this thread's staging positions: A (rows ar + 64 m, k ac + i) or,
  // transposed, (k ak, rows am + 64 m + i); B (k bk, cols bc + i) or,
  // transposed, (col bn, k bkc + i)
  const int ar = t >> 2, ac = (t & 3) * 4;
  const int ak = t >> 4, am = (t & 15) * 4;
  const int bk = t >> 4, bc = (t & 15) * 4;
  const int bn = t >> 2, bkc = (t & 3) * 4;
  double2 ra[4 * MR], rb[4];
  int mn[B_MAP ? 4 : 1];  // mapped columns of this thread's B elements (fixed over k)
  if constexpr (B_MAP) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int n = b_off + bc + i;
      mn[i] = n < b_lim ? (bmap ? bmap[n] : n) : 0;
    }
  }
  // mapped B: the row map entry of this thread's k for the chunk being
  // loaded, read one chunk ahead so that the W load does not wait on it
  int mk = 0;
  if constexpr (B_MAP) mk = bk < K ? (bmap ? bmap[bk] : bk) : 0;
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 4 * MR; ++e) {
      const int i = e & 3, m64 = (e >> 2) * 64;
      bool ok;
      size_t idx;
      if constexpr (!A_T) {
        const int gr = a_off + ar + m64, k = k0 + ac + i;
        ok = gr < a_lim && k < K;
        idx = (size_t)gr * lda + k;
      } else {
        const int m = a_off + am + m64 + i, k = k0 + ak;
        ok = m < a_lim && k < K;
        idx = (size_t)k * lda + m;
      }
      const double2 v = gld(A, ok ? idx : 0);
      ra[e] = make_double2(ok ? v.x : 0.0, ok ? v.y : 0.0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bool ok;
      size_t idx;
      if constexpr (B_T) {
        const int gn = b_off + bn, k = k0 + bkc + i;
        ok = gn < b_lim && k < K;
        idx = (size_t)gn * ldb + k;
      } else if constexpr (B_MAP) {
        const int n = b_off + bc + i, k = k0 + bk;
        ok = k < K && n < b_lim;
        idx = (size_t)(k < K ? mk : 0) * ldb + mn[i];
      } else {
        const int n = b_off + bc + i, k = k0 + bk;
        ok = k < K && n < b_lim;
        idx = (size_t)k * ldb + n;
      }
      const double2 v = gld(B, ok ? idx : 0);
      rb[i] = make_double2(ok ? v.x : 0.0, ok ? (B_MAP && bconj ? -v.y : v.y) : 0.0);
    }
    if constexpr (B_MAP) {
      const int kn = k0 + KC + bk;  // the next chunk's row
      mk = kn < K ? (bmap ? bmap[kn] : kn) : 0;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < 4 * MR; ++e) {
      const int i = e & 3, m64 = (e >> 2) * 64;
      if constexpr (!A_T) {
        As_re[ar + m64][ac + i] = ra[e].x;
        As_im[ar + m64][ac + i] = CONJ_A ? -ra[e].y : ra[e].y;
      } else {
        As_re[am + m64 + i][ak] = ra[e].x;
        As_im[am + m64 + i][ak] = CONJ_A ? -ra[e].y : ra[e].y;
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if constexpr (B_T) {
        Bs_re[bkc + i][bn] = rb[i].x;
        Bs_im[bkc + i][bn] = rb[i].y;
      } else {
        Bs_re[bk][bc + i] = rb[i].x;
        Bs_im[bk][bc + i] = rb[i].y;
      }
    }
  };
  if (K > 0) load(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
    store();
    __syncthreads();
    if (k0 + KC < K) load(k0 + KC);  // in flight during the MFMAs below
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      double are[2 * MR], aim[2 * MR], bre[2], bim[2];
#pragma unroll
      for (int i = 0; i < 2 * MR; ++i) {
        are[i] = As_re[wr * 32 * MR + i * 16 + (lane & 15)][kk + (lane >> 4)];
        aim[i] = As_im[wr * 32 * MR + i * 16 + (lane & 15)][kk + (lane >> 4)];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        bre[i] = Bs_re[kk + (lane >> 4)][wc * 32 + i * 16 + (lane & 15)];
        bim[i] = Bs_im[kk + (lane >> 4)][wc * 32 + i * 16 + (lane & 15)];
      }
      if constexpr (G3) {
        double asum[2 * MR], bsum[2];
#pragma unroll
        for (int i = 0; i < 2 * MR; ++i) asum[i] = are[i] + aim[i];
#pragma unroll
        for (int j = 0; j < 2; ++j) bsum[j] = bre[j] + bim[j];
#pragma unroll
        for (int i = 0; i < 2 * MR; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            cre[i][j] = mfma64(are[i], bre[j], cre[i][j]);
            p2[i][j] = mfma64(aim[i], bim[j], p2[i][j]);
            cim[i][j] = mfma64(asum[i], bsum[j], cim[i][j]);
          }
      } else {
#pragma unroll
        for (int i = 0; i < 2 * MR; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            cre[i][j] = mfma64(are[i], bre[j], cre[i][j]);
            cre[i][j] = mfma64(-aim[i], bim[j], cre[i][j]);
            cim[i][j] = mfma64(are[i], bim[j], cim[i][j]);
            cim[i][j] = mfma64(aim[i], bre[j], cim[i][j]);
          }
      }
    }
    __syncthreads();
  }
  if constexpr (G3) {
#pragma unroll
    for (int i = 0; i < 2 * MR; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const d4 a = cre[i][j], b = p2[i][j];
        cre[i][j] = a - b;
        cim[i][j] = cim[i][j] - a - b;
      }
  }
}


// ------------------------------------------------------------------ split operands

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));

constexpr int MTM = 64, MTN = 64, MKC = 32;

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  __hip_bfloat16 b = __float2bfloat16(f);
  return *reinterpret_cast<unsigned short*>(&b);
}
__device__ __forceinline__ float bf16_value(unsigned short u) {
  return __uint_as_float(((unsigned int)u) << 16);
}

template <int P>
struct Split;
// FP32 parts
template <>
struct Split<BSE_SPLIT_FP32> {
  typedef float T;
  __device__ static void split(double x, float& h, float& l) {
    h = (float)x;
    l = (float)(x - (double)h);
  }
};
// BF16 parts, stored as raw 16-bit patterns
template <>
struct Split<BSE_BF16X3> {
  typedef unsigned short T;
  __device__ static void split(double x, unsigned short& h, unsigned short& l) {
    h = bf16_bits((float)x);
    l = bf16_bits((float)(x - (double)bf16_value(h)));
  }
};

// LDS image of an R x 32 complex operand tile: 4 planes (re hi, re lo, im hi,
// im lo), each [R rows][32 k] with k contiguous, row stride padded.
template <int P, int R = 64>
struct TileLds {
  typedef typename Split<P>::T T;
  static constexpr int STRIDE = P == BSE_BF16X3 ? 40 : 33;
  T v[4][R * STRIDE];
};
// Dynamic LDS bytes of tile_gemm_mx with MR.
template <int P, int MR>
constexpr size_t tile_mx_lds() {
  return sizeof(TileLds<P, 64 * MR>) + sizeof(TileLds<P>);
}

// Stores 8 consecutive k values (row r, k0..k0+7) of one operand after the split.
template <int P, int R>
__device__ __forceinline__ void put8(TileLds<P, R>& L, int r, int k0, const double2* x, bool conj) {
  typedef typename Split<P>::T T;
  T h[4][8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    Split<P>::split(x[i].x, h[0][i], h[1][i]);
    Split<P>::split(conj ? -x[i].y : x[i].y, h[2][i], h[3][i]);
  }
#pragma unroll
  for (int pl = 0; pl < 4; ++pl)
#pragma unroll
    for (int i = 0; i < 8; ++i) L.v[pl][r * TileLds<P, R>::STRIDE + k0 + i] = h[pl][i];
}

// One (64 MR) x 64 complex tile of C = op(A) * B with split operands; operand
// addressing as in tile_gemm; dynamic LDS of tile_mx_lds<P, MR>() bytes.  zero_head: B[0][0] := 0 when the tile holds it
// (the q = 0 head is added in FP64 elsewhere).
// B_PRE: B comes already split, as Bp[n][plane][k] (row stride 4 ldk, planes
// re hi, re lo, im hi, im lo; zero for k >= K up to a multiple of 32), and is
// copied to LDS without conversion (B, ldb, B_T and zero_head unused).
// A_PRE: the same for A, Ap[m][plane][k] (already conjugated if it is to be;
// A, lda, A_T and CONJ_A unused).
template <int P, bool CONJ_A, bool B_T, bool A_T = false, bool B_PRE = false, bool A_PRE = false, int MR = 1>
__device__ __forceinline__ void tile_gemm_mx(const double2* __restrict__ A, int lda, int a_off, int a_lim,
                                             const double2* __restrict__ B, int ldb, int b_off, int b_lim, int K,
                                             bool zero_head, f4 (&cre)[2 * MR][2], f4 (&cim)[2 * MR][2],
                                             const typename Split<P>::T* __restrict__ Bp = nullptr, int ldk = 0,
                                             const typename Split<P>::T* __restrict__ Ap = nullptr) {
  static_assert(MR == 1 || MR == 2, "64 or 128 rows per tile");
  extern __shared__ double2 smem_mx_raw[];  // 16-byte aligned dynamic area
  char* smem_mx = reinterpret_cast<char*>(smem_mx_raw);
  TileLds<P, 64 * MR>& As = *reinterpret_cast<TileLds<P, 64 * MR>*>(smem_mx);
  TileLds<P>& Bs = *reinterpret_cast<TileLds<P>*>(smem_mx + sizeof(TileLds<P, 64 * MR>));
  constexpr int ST = TileLds<P>::STRIDE;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int i = 0; i < 2 * MR; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cre[i][j] = f4{0, 0, 0, 0};
      cim[i][j] = f4{0, 0, 0, 0};
    }
  const int r = t >> 2, kq = (t & 3) * 8;
  // the next chunk's operands are loaded while the MFMAs consume the current
  // one; out-of-range elements are read from the array start and zeroed
  typedef typename Split<P>::T T;
  constexpr int QW = sizeof(T) * 8 / 16;  // 16-byte words per plane row segment of 8 k
  double2 xa[A_PRE ? 1 : 8 * MR], xb[B_PRE ? 1 : 8];
  uint4 xp[B_PRE ? 4 * QW : 1], xq[A_PRE ? 4 * QW * MR : 1];
  auto load = [&](int k0) {
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      const int gr = a_off + r + 64 * m;
      if constexpr (A_PRE) {
        const bool ok = gr < a_lim;
        const T* row = Ap + (ok ? (size_t)gr * 4 * ldk : 0) + k0 + kq;
#pragma unroll
        for (int pl = 0; pl < 4; ++pl)
#pragma unroll
          for (int w4 = 0; w4 < QW; ++w4) {
            const uint4 v = gld16(reinterpret_cast<const uint4*>(row + (size_t)pl * ldk) + w4);
            xq[(m * 4 + pl) * QW + w4] = ok ? v : make_uint4(0u, 0u, 0u, 0u);
          }
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int k = k0 + kq + i;
          const bool ok = gr < a_lim && k < K;
          const size_t idx = A_T ? (size_t)k * lda + gr : (size_t)gr * lda + k;
          const double2 v = gld(A, ok ? idx : 0);
          xa[m * 8 + i] = make_double2(ok ? v.x : 0.0, ok ? v.y : 0.0);
        }
      }
    }
    if constexpr (B_PRE) {
      const bool ok = b_off + r < b_lim;
      const T* row = Bp + (ok ? (size_t)(b_off + r) * 4 * ldk : 0) + k0 + kq;
#pragma unroll
      for (int pl = 0; pl < 4; ++pl)
#pragma unroll
        for (int w4 = 0; w4 < QW; ++w4) {
          const uint4 v = gld16(reinterpret_cast<const uint4*>(row + (size_t)pl * ldk) + w4);
          xp[pl * QW + w4] = ok ? v : make_uint4(0u, 0u, 0u, 0u);
        }
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + kq + i;
        const bool ok = b_off + r < b_lim && k < K && !(zero_head && k == 0 && b_off + r == 0);
        const size_t idx = B_T ? (size_t)(b_off + r) * ldb + k : (size_t)k * ldb + b_off + r;
        const double2 v = gld(B, ok ? idx : 0);
        xb[i] = make_double2(ok ? v.x : 0.0, ok ? v.y : 0.0);
      }
    }
  };
  if (K > 0) load(0);
  for (int k0 = 0; k0 < K; k0 += MKC) {
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      if constexpr (A_PRE) {
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) {
          const T* src = reinterpret_cast<const T*>(&xq[(m * 4 + pl) * QW]);
#pragma unroll
          for (int i = 0; i < 8; ++i) As.v[pl][(r + 64 * m) * ST + kq + i] = src[i];
        }
      } else {
        put8<P>(As, r + 64 * m, kq, xa + 8 * m, CONJ_A);
      }
    }
    if constexpr (B_PRE) {
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) {
        const T* src = reinterpret_cast<const T*>(&xp[pl * QW]);
#pragma unroll
        for (int i = 0; i < 8; ++i) Bs.v[pl][r * ST + kq + i] = src[i];
      }
    } else {
      put8<P>(Bs, r, kq, xb, false);
    }
    __syncthreads();
    if (k0 + MKC < K) load(k0 + MKC);
    if constexpr (P == BSE_BF16X3) {
      s8 a[2 * MR][4], b[2][4];
#pragma unroll
      for (int i = 0; i < 2 * MR; ++i)
#pragma unroll
        for (int pl = 0; pl < 4; ++pl)
          a[i][pl] =
              *reinterpret_cast<const s8*>(&As.v[pl][(wr * 32 * MR + i * 16 + (lane & 15)) * ST + 8 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int pl = 0; pl < 4; ++pl)
          b[i][pl] = *reinterpret_cast<const s8*>(&Bs.v[pl][(wc * 32 + i * 16 + (lane & 15)) * ST + 8 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < 2 * MR; ++i) {
        s8 nih = a[i][2] ^ (short)0x8000, nil = a[i][3] ^ (short)0x8000;  // -Im(a) parts
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          f4 cr = cre[i][j], ci = cim[i][j];
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][0], cr, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][1], cr, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], b[j][0], cr, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, b[j][2], cr, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, b[j][3], cr, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nil, b[j][2], cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][2], ci, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][3], ci, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], b[j][2], ci, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], b[j][0], ci, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], b[j][1], ci, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][3], b[j][0], ci, 0, 0, 0);
          cre[i][j] = cr;
          cim[i][j] = ci;
        }
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < MKC; kk += 4) {
        float a[2 * MR][4], b[2][4];
#pragma unroll
        for (int i = 0; i < 2 * MR; ++i)
#pragma unroll
          for (int pl = 0; pl < 4; ++pl)
            a[i][pl] = As.v[pl][(wr * 32 * MR + i * 16 + (lane & 15)) * ST + kk + (lane >> 4)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int pl = 0; pl < 4; ++pl)
            b[i][pl] = Bs.v[pl][(wc * 32 + i * 16 + (lane & 15)) * ST + kk + (lane >> 4)];
#pragma unroll
        for (int i = 0; i < 2 * MR; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            f4 cr = cre[i][j], ci = cim[i][j];
            cr = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][0], b[j][0], cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][0], b[j][1], cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][1], b[j][0], cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[i][2], b[j][2], cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[i][2], b[j][3], cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[i][3], b[j][2], cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][0], b[j][2], ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][0], b[j][3], ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][1], b[j][2], ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][2], b[j][0], ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][2], b[j][1], ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][3], b[j][0], ci, 0, 0, 0);
            cre[i][j] = cr;
            cim[i][j] = ci;
          }
      }
    }
    __syncthreads();
  }
}

// f32 MFMA accumulator layout: lane l, register r holds D[4 (l/16) + r][l % 16]
__device__ __forceinline__ int acc_row(int lane, int r) { return 4 * (lane >> 4) + r; }


}  // namespace bse
