// Mixed-precision versions of the exchange and direct-term contractions.
// Every FP64 operand x is split as x = hi + lo with hi = round(x) and
// lo = round(x - hi) in the narrow type; a product a*b is taken as
// hi*hi + hi*lo + lo*hi (the lo*lo term is dropped) with FP32 accumulation:
//   BSE_SPLIT_FP32: FP32 parts, v_mfma_f32_16x16x4_f32
//   BSE_BF16X3:     BF16 parts, v_mfma_f32_16x16x32_bf16
// The q = 0 head of W, the transition-energy diagonal and the final update of
// H stay FP64.
#include "../../include/bse.h"
#include "bse_internal.h"
#include "gemm_tiles.h"
#include "kernels.h"

namespace bse {

template <int P>
__global__ __launch_bounds__(256) void k_exchange_mx(const GemmArgs* __restrict__ gs, const HTile* __restrict__ tiles) {
  const HTile tl = tiles[blockIdx.x];
  const GemmArgs g = gs[tl.sys];
  const int r0 = tl.i * MTM, c0 = tl.j * MTN;
  f4 cre[2][2], cim[2][2];
  tile_gemm_mx<P, true, true>(g.X, g.ng_max, r0, g.ns, g.X, g.ng_max, c0, g.ns, g.ngx, false, cre, cim);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
  const double s = 2.0 * g.cpref;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + wr * 32 + i * 16 + acc_row(lane, r);
        const int col = c0 + wc * 32 + j * 16 + (lane & 15);
        if (row < g.ns && col < g.ns)
          gst(g.H, (size_t)row * g.ldh + col, make_double2(s * (double)cre[i][j][r], s * (double)cim[i][j][r]));
      }
}

// 128-row tiles (MR = 2) for BF16 parts only: with FP32 parts they do not fit
// two waves per SIMD without spilling.
template <int P, int MR>
__global__ __launch_bounds__(256, MR == 1 ? 1 : 2) void k_direct_s1_mx(const GemmArgs* __restrict__ gs,
                                                                       const S1Tile* __restrict__ tiles) {
  static_assert(MR == 1 || P == BSE_BF16X3, "128-row tiles with BF16 parts only");
  const S1Tile tl = tiles[blockIdx.x];
  const GemmArgs g = gs[tl.sys];
  const int nv2 = g.rv_rows;
  const int row_base = (gbl(g.qstart)[tl.iq] - g.p0) * nv2;  // rows of the chunk
  const int rows = (gbl(g.qstart)[tl.iq + 1] - gbl(g.qstart)[tl.iq]) * nv2;
  const int K = gbl(g.ng)[tl.iq];
  const double2* A = g.RV + (size_t)row_base * g.ng_max;
  const double2* Wq = g.W + (size_t)tl.iq * g.ng_max * g.ng_max;
  f4 cre[2 * MR][2], cim[2 * MR][2];
  const int r0 = tl.mt * MTM * MR, c0 = tl.nt * MTN;
  typedef typename Split<P>::T T;
  const T* Wsq = reinterpret_cast<const T*>(g.Ws) + (size_t)tl.iq * g.ng_max * 4 * g.kpad;
  const T* RVs = reinterpret_cast<const T*>(g.RVs) + (size_t)row_base * 4 * g.kpad;
  tile_gemm_mx<P, true, false, false, true, true, MR>(A, g.ng_max, r0, rows, Wq, g.ng_max, c0, K, K, false, cre,
                                                      cim, Wsq, g.kpad, RVs);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
  double2* Z = g.Z + (size_t)row_base * g.ng_max;
#pragma unroll
  for (int i = 0; i < 2 * MR; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + wr * 32 * MR + i * 16 + acc_row(lane, r);
        const int col = c0 + wc * 32 + j * 16 + (lane & 15);
        if (row < rows && col < K)
          gst(Z, (size_t)row * g.ng_max + col, make_double2((double)cre[i][j][r], (double)cim[i][j][r]));
      }
}

// W(q) split once per build and transposed so that the stage-1 tiles read
// their B operand k-contiguous without converting it: one 32 x 32 tile of
// (k, n) per workgroup through LDS.
// W of the irreducible q points (wmap): W(q) is gathered from its source
// matrix through the sphere map and conjugated where the map says so.
template <int P>
__global__ __launch_bounds__(256) void k_split_w(const double2* __restrict__ W, const int* __restrict__ ng,
                                                 const int* __restrict__ wsrc, const int* __restrict__ wmap, int nk,
                                                 int ng_max, int kpad, int head, typename Split<P>::T* __restrict__ Ws) {
  __shared__ double2 tile[32][33];
  const int n0 = blockIdx.x * 32, k0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int q = blockIdx.z; q < nk; q += gridDim.z) {
  const int ngq = ng[q];
  const int src = wmap ? wsrc[2 * q] : q;
  const bool cj = wmap && wsrc[2 * q + 1];
  const int* mq = wmap ? wmap + (size_t)q * ng_max : nullptr;
  __syncthreads();  // the previous q's tile is read
  for (int r = ty; r < 32; r += 8) {
    const int k = k0 + r, n = n0 + tx;
    double2 v = make_double2(0.0, 0.0);
    if (k < ngq && n < ngq && !(head && q == 0 && k == 0 && n == 0)) {
      const int ks = mq ? mq[k] : k, ns = mq ? mq[n] : n;
      v = W[((size_t)src * ng_max + ks) * ng_max + ns];
      if (cj) v.y = -v.y;
    }
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int n = n0 + r, k = k0 + tx;
    if (n >= ng_max || k >= kpad) continue;
    const double2 v = tile[tx][r];
    typename Split<P>::T h[4];
    Split<P>::split(v.x, h[0], h[1]);
    Split<P>::split(v.y, h[2], h[3]);
    typename Split<P>::T* row = Ws + ((size_t)q * ng_max + n) * 4 * kpad + k;
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) row[(size_t)pl * kpad] = h[pl];
  }
  }
}

// The valence pair-density rows of a chunk split, conjugated, into
// RVs[row][part][kpad] (the A operand of stage 1): one thread per (row, k); a
// row of pair p holds ng(q_p) values, the rest (and k >= ng_max) is written as
// zero, whatever the row's tail in RV holds.  `pairs` starts at the chunk's
// first pair.
template <int P>
__global__ __launch_bounds__(256) void k_split_rv(const double2* __restrict__ RV, const int4* __restrict__ pairs,
                                                  const int* __restrict__ ng, size_t nrows, int rows_per_pair,
                                                  int ld, int kpad, typename Split<P>::T* __restrict__ Xs) {
  const size_t n = nrows * (size_t)kpad;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const size_t row = i / kpad;
    const int k = (int)(i - row * kpad);
    const int valid = ng[pairs[row / rows_per_pair].z];
    const double2 v = k < valid ? RV[row * ld + k] : make_double2(0.0, 0.0);
    typename Split<P>::T h[4];
    Split<P>::split(v.x, h[0], h[1]);
    Split<P>::split(-v.y, h[2], h[3]);
    typename Split<P>::T* o = Xs + row * 4 * kpad + k;
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) o[(size_t)pl * kpad] = h[pl];
  }
}

hipError_t launch_split_rv(const double2* RV, const int4* pairs, const int* ng, size_t nrows, int rows_per_pair,
                           int ld, int kpad, int precision, void* RVs, hipStream_t st) {
  if (nrows == 0) return hipSuccess;
  const dim3 grid(8192), blk(256);
  if (precision == BSE_BF16X3)
    hipLaunchKernelGGL(k_split_rv<BSE_BF16X3>, grid, blk, 0, st, RV, pairs, ng, nrows, rows_per_pair, ld, kpad,
                       reinterpret_cast<unsigned short*>(RVs));
  else
    hipLaunchKernelGGL(k_split_rv<BSE_SPLIT_FP32>, grid, blk, 0, st, RV, pairs, ng, nrows, rows_per_pair, ld, kpad,
                       reinterpret_cast<float*>(RVs));
  return hipGetLastError();
}

hipError_t launch_split_w(const double2* W, const int* ng, const int* wsrc, const int* wmap, int nk, int ng_max,
                          int kpad, int head, int precision, void* Ws, hipStream_t st) {
  if (nk <= 0) return hipSuccess;
  const dim3 grid((ng_max + 31) / 32, kpad / 32, nk < 4096 ? nk : 4096);
  if (precision == BSE_BF16X3)
    hipLaunchKernelGGL(k_split_w<BSE_BF16X3>, grid, dim3(256), 0, st, W, ng, wsrc, wmap, nk, ng_max, kpad, head,
                       reinterpret_cast<unsigned short*>(Ws));
  else
    hipLaunchKernelGGL(k_split_w<BSE_SPLIT_FP32>, grid, dim3(256), 0, st, W, ng, wsrc, wmap, nk, ng_max, kpad, head,
                       reinterpret_cast<float*>(Ws));
  return hipGetLastError();
}

template <int P>
static hipError_t launch_ex(const GemmArgs* gs, const HTile* tiles, int ntiles, hipStream_t st) {
  const size_t lds = 2 * sizeof(TileLds<P>);
  hipError_t e = hipFuncSetAttribute((const void*)k_exchange_mx<P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_exchange_mx<P>, dim3(ntiles), dim3(256), lds, st, gs, tiles);
  return hipGetLastError();
}

template <int P, int MR>
static hipError_t launch_s1(const GemmArgs* gs, const S1Tile* tiles, int ntiles, hipStream_t st) {
  const size_t lds = tile_mx_lds<P, MR>();
  void (*k)(const GemmArgs*, const S1Tile*) = k_direct_s1_mx<P, MR>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(ntiles), dim3(256), lds, st, gs, tiles);
  return hipGetLastError();
}

hipError_t launch_exchange_mx(const GemmArgs* gs, const HTile* tiles, int ntiles, int precision, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  return precision == BSE_BF16X3 ? launch_ex<BSE_BF16X3>(gs, tiles, ntiles, st)
                                 : launch_ex<BSE_SPLIT_FP32>(gs, tiles, ntiles, st);
}

hipError_t launch_direct_s1_mx(const GemmArgs* gs, const S1Tile* tiles, int ntiles, int precision, int rows,
                               hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (rows == 128)
    return precision == BSE_BF16X3 ? launch_s1<BSE_BF16X3, 2>(gs, tiles, ntiles, st) : hipErrorInvalidValue;
  return precision == BSE_BF16X3 ? launch_s1<BSE_BF16X3, 1>(gs, tiles, ntiles, st)
                                 : launch_s1<BSE_SPLIT_FP32, 1>(gs, tiles, ntiles, st);
}


}  // namespace bse
