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
          gst(g.H, (size_t)row * g.ns + col, make_double2(s * (double)cre[i][j][r], s * (double)cim[i][j][r]));
      }
}

template <int P>
__global__ __launch_bounds__(256) void k_direct_s1_mx(const GemmArgs* __restrict__ gs, const S1Tile* __restrict__ tiles) {
  const S1Tile tl = tiles[blockIdx.x];
  const GemmArgs g = gs[tl.sys];
  const int nv2 = g.nv * g.nv;
  const int row_base = gbl(g.qstart)[tl.iq] * nv2;
  const int rows = (gbl(g.qstart)[tl.iq + 1] - gbl(g.qstart)[tl.iq]) * nv2;
  const int K = gbl(g.ng)[tl.iq];
  const double2* A = g.RV + (size_t)row_base * g.ng_max;
  const double2* Wq = g.W + (size_t)tl.iq * g.ng_max * g.ng_max;
  f4 cre[2][2], cim[2][2];
  const int r0 = tl.mt * MTM, c0 = tl.nt * MTN;
  tile_gemm_mx<P, true, false>(A, g.ng_max, r0, rows, Wq, g.ng_max, c0, K, K, tl.iq == 0 && g.w_head_fp64,
                              cre, cim);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
  double2* Z = g.Z + (size_t)row_base * g.ng_max;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + wr * 32 + i * 16 + acc_row(lane, r);
        const int col = c0 + wc * 32 + j * 16 + (lane & 15);
        if (row < rows && col < K)
          gst(Z, (size_t)row * g.ng_max + col, make_double2((double)cre[i][j][r], (double)cim[i][j][r]));
      }
}

// Stage 2 per k pair: D[vv'][cc'] = sum_g Z[vv'][g] RC[cc'][g] (no conjugate),
// operands split in registers.  The q = 0 head conj(rho_vv'(0)) W_00 rho_cc'(0)
// is added in FP64.
template <int P>
__global__ __launch_bounds__(256) void k_direct_s2_mx(const GemmArgs* __restrict__ gs, const int* __restrict__ d2off,
                                                      int nsys, int nitems) {
  const int lane = threadIdx.x & 63;
  const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= nitems) return;
  const int sys = item_system(d2off, nsys, item);
  const GemmArgs g = gs[sys];
  const int nv2 = g.nv * g.nv, nc2 = g.nc * g.nc;
  const int tiles_i = (nv2 + 15) / 16, tiles_j = (nc2 + 15) / 16;
  const int loc = item - d2off[sys];
  const int per = tiles_i * tiles_j;
  const int p = loc / per, ti = (loc % per) / tiles_j, tj = loc % tiles_j;
  const int4 pr = gld(g.pairs, p);
  const int ka = pr.x, kb = pr.y;
  const int K = gbl(g.ng)[pr.z];
  const int ia = ti * 16 + (lane & 15), jb = tj * 16 + (lane & 15);
  const bool va = ia < nv2, vb = jb < nc2;
  const double2* zr = g.Z + ((size_t)p * nv2 + (va ? ia : 0)) * g.ng_max;
  const double2* cr = g.RC + ((size_t)p * nc2 + (vb ? jb : 0)) * g.ng_max;
  f4 dre = {0, 0, 0, 0}, dim = {0, 0, 0, 0};
  if constexpr (P == BSE_BF16X3) {
    for (int k0 = 0; k0 < K; k0 += 32) {
      s8 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + 8 * (lane >> 4) + i;
        const double2 x = (va && k < K) ? gld(zr, k) : make_double2(0.0, 0.0);
        const double2 y = (vb && k < K) ? gld(cr, k) : make_double2(0.0, 0.0);
        unsigned short h, l;
        Split<P>::split(x.x, h, l); a[0][i] = (short)h; a[1][i] = (short)l;
        Split<P>::split(x.y, h, l); a[2][i] = (short)h; a[3][i] = (short)l;
        Split<P>::split(y.x, h, l); b[0][i] = (short)h; b[1][i] = (short)l;
        Split<P>::split(y.y, h, l); b[2][i] = (short)h; b[3][i] = (short)l;
      }
      const s8 nih = a[2] ^ (short)0x8000, nil = a[3] ^ (short)0x8000;
      dre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], dre, 0, 0, 0);
      dre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], dre, 0, 0, 0);
      dre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], dre, 0, 0, 0);
      dre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, b[2], dre, 0, 0, 0);
      dre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, b[3], dre, 0, 0, 0);
      dre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nil, b[2], dre, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], dim, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[3], dim, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[2], dim, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], dim, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[1], dim, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[3], b[0], dim, 0, 0, 0);
    }
  } else {
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + (lane >> 4);
      const double2 x = (va && k < K) ? gld(zr, k) : make_double2(0.0, 0.0);
      const double2 y = (vb && k < K) ? gld(cr, k) : make_double2(0.0, 0.0);
      float a[4], b[4];
      Split<P>::split(x.x, a[0], a[1]);
      Split<P>::split(x.y, a[2], a[3]);
      Split<P>::split(y.x, b[0], b[1]);
      Split<P>::split(y.y, b[2], b[3]);
      dre = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], dre, 0, 0, 0);
      dre = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[1], dre, 0, 0, 0);
      dre = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[0], dre, 0, 0, 0);
      dre = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[2], b[2], dre, 0, 0, 0);
      dre = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[2], b[3], dre, 0, 0, 0);
      dre = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[3], b[2], dre, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[2], dim, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[3], dim, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[2], dim, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[0], dim, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[1], dim, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[0], dim, 0, 0, 0);
    }
  }
  // FP64 head of W at q = 0 (left out of both mixed GEMMs)
  const bool head = pr.z == 0 && g.w_head_fp64;
  const double2 w00 = head ? gld(g.W, 0) : make_double2(0.0, 0.0);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = ti * 16 + acc_row(lane, r);
    const int j = tj * 16 + (lane & 15);
    if (i < nv2 && j < nc2) {
      double dr = (double)dre[r], di = (double)dim[r];
      if (head) {
        const double2 rv0 = gld(g.RV, ((size_t)p * nv2 + i) * g.ng_max);
        const double2 rc0 = gld(g.RC, ((size_t)p * nc2 + j) * g.ng_max);
        const double2 hw = cmul(cconjmul(rv0, w00), rc0);
        dr += hw.x;
        di += hw.y;
      }
      const int v = i / g.nv, v2 = i % g.nv, c = j / g.nc, c2 = j % g.nc;
      const size_t S = ((size_t)ka * g.nv + v) * g.nc + c;
      const size_t S2 = ((size_t)kb * g.nv + v2) * g.nc + c2;
      double2 h = gld(g.H, S * g.ns + S2);
      h.x -= g.cpref * dr;
      h.y -= g.cpref * di;
      if (S == S2) h.x += gbl(g.eps)[(size_t)ka * g.nb + g.nv + c] - gbl(g.eps)[(size_t)ka * g.nb + v];
      gst(g.H, S * g.ns + S2, h);
    }
  }
}

template <int P>
static hipError_t launch_ex(const GemmArgs* gs, const HTile* tiles, int ntiles, hipStream_t st) {
  const size_t lds = 2 * sizeof(TileLds<P>);
  hipError_t e = hipFuncSetAttribute((const void*)k_exchange_mx<P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_exchange_mx<P>, dim3(ntiles), dim3(256), lds, st, gs, tiles);
  return hipGetLastError();
}

template <int P>
static hipError_t launch_s1(const GemmArgs* gs, const S1Tile* tiles, int ntiles, hipStream_t st) {
  const size_t lds = 2 * sizeof(TileLds<P>);
  hipError_t e = hipFuncSetAttribute((const void*)k_direct_s1_mx<P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_direct_s1_mx<P>, dim3(ntiles), dim3(256), lds, st, gs, tiles);
  return hipGetLastError();
}

hipError_t launch_exchange_mx(const GemmArgs* gs, const HTile* tiles, int ntiles, int precision, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  return precision == BSE_BF16X3 ? launch_ex<BSE_BF16X3>(gs, tiles, ntiles, st)
                                 : launch_ex<BSE_SPLIT_FP32>(gs, tiles, ntiles, st);
}

hipError_t launch_direct_s1_mx(const GemmArgs* gs, const S1Tile* tiles, int ntiles, int precision, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  return precision == BSE_BF16X3 ? launch_s1<BSE_BF16X3>(gs, tiles, ntiles, st)
                                 : launch_s1<BSE_SPLIT_FP32>(gs, tiles, ntiles, st);
}

hipError_t launch_direct_s2_mx(const GemmArgs* gs, const int* d2off, int nsys, int nitems, int precision,
                               hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  if (precision == BSE_BF16X3)
    hipLaunchKernelGGL(k_direct_s2_mx<BSE_BF16X3>, dim3((nitems + 3) / 4), dim3(256), 0, st, gs, d2off, nsys, nitems);
  else
    hipLaunchKernelGGL(k_direct_s2_mx<BSE_SPLIT_FP32>, dim3((nitems + 3) / 4), dim3(256), 0, st, gs, d2off, nsys,
                       nitems);
  return hipGetLastError();
}

}  // namespace bse
