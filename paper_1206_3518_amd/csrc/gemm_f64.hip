// FP64 MFMA contractions of the Hamiltonian (Sec. II.C of the paper):
//   exchange  H[S][S'] = 2c sum_g conj(X[S][g]) X[S'][g]     (X scaled by sqrt v(G), G = 0 left out)
//   direct 1  Z[r][n]  = sum_g conj(RV[r][g]) W_q[g][n]       (rows r: band pairs vv' of the k pairs of q)
//   direct 2  H[(k v c),(k' v' c')] -= c sum_g Z[(kk' vv')][g] RC[(kk' cc')][g], plus e_ck - e_vk on the diagonal
//   mirror    lower k blocks = conjugate transpose of the upper ones (plain transpose
//             for the symmetric coupling block of the beyond-TDA matrix)
// Complex products run as four real v_mfma_f64_16x16x4 products per step.
// Every launch covers a batch of systems: tiles and items name their system.
#include <algorithm>

#include "../../include/bse.h"
#include "bse_internal.h"
#include "gemm_tiles.h"
#include "kernels.h"

namespace bse {

// ------------------------------------------------------------------ exchange

__global__ __launch_bounds__(256, 2) void k_exchange(const GemmArgs* __restrict__ gs, const HTile* __restrict__ tiles) {
  const HTile tl = tiles[blockIdx.x];
  const GemmArgs g = gs[tl.sys];
  const int r0 = tl.i * TM, c0 = tl.j * TN;
  d4 cre[2][2], cim[2][2];
  tile_gemm<true, true, false, true, false, 1, true>(g.X, g.ng_max, r0, g.ns, g.Xb ? g.Xb : g.X, g.ng_max, c0, g.ns,
                                                     g.ngx, cre, cim);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
  const double s = 2.0 * g.cpref;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + wr * 32 + i * 16 + 4 * r + (lane >> 4);
        const int col = c0 + wc * 32 + j * 16 + (lane & 15);
        if (row < g.ns && col < g.ns) gst(g.H, (size_t)row * g.ldh + col, make_double2(s * cre[i][j][r], s * cim[i][j][r]));
      }
}

hipError_t launch_exchange(const GemmArgs* gs, const HTile* tiles, int ntiles, int precision, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (precision != BSE_FP64) return launch_exchange_mx(gs, tiles, ntiles, precision, st);
  hipLaunchKernelGGL(k_exchange, dim3(ntiles), dim3(256), 0, st, gs, tiles);
  return hipGetLastError();
}

// ------------------------------------------------------------------ direct, stage 1

// MAP: some system of the batch gives W at the irreducible q points only; its
// W(q) is read from the source matrix through the sphere map of q (Sec. III.A),
// conjugated for the time-reversed images.  64-row tiles in the three-product
// form (a quarter fewer MFMAs; its three accumulators hold the tile at two
// waves per SIMD).
template <bool MAP>
__global__ __launch_bounds__(256, 2) void k_direct_s1(const GemmArgs* __restrict__ gs,
                                                      const S1Tile* __restrict__ tiles) {
  const S1Tile tl = tiles[blockIdx.x];
  const GemmArgs g = gs[tl.sys];
  const int nv2 = g.rv_rows;
  const int row_base = (gbl(g.qstart)[tl.iq] - g.p0) * nv2;  // rows of the chunk
  const int rows = (gbl(g.qstart)[tl.iq + 1] - gbl(g.qstart)[tl.iq]) * nv2;
  const int K = gbl(g.ng)[tl.iq];
  const double2* A = g.RV + (size_t)row_base * g.ng_max;
  d4 cre[2][2], cim[2][2];
  const int r0 = tl.mt * TM, c0 = tl.nt * TN;
  if constexpr (MAP) {  // systems without maps take the same path with a null map
    const bool m = g.wmap != nullptr;
    const int src = m ? gbl(g.wsrc)[2 * tl.iq] : tl.iq, cj = m ? gbl(g.wsrc)[2 * tl.iq + 1] : 0;
    tile_gemm<true, false, false, true, true, 1, true>(A, g.ng_max, r0, rows,
                                                       g.W + (size_t)src * g.ng_max * g.ng_max, g.ng_max, c0, K, K,
                                                       cre, cim, m ? g.wmap + (size_t)tl.iq * g.ng_max : nullptr,
                                                       cj != 0);
  } else {
    const double2* Wq = g.W + (size_t)tl.iq * g.ng_max * g.ng_max;
    tile_gemm<true, false, false, true, false, 1, true>(A, g.ng_max, r0, rows, Wq, g.ng_max, c0, K, K, cre, cim);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
  double2* Z = g.Z + (size_t)row_base * g.ng_max;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + wr * 32 + i * 16 + 4 * r + (lane >> 4);
        const int col = c0 + wc * 32 + j * 16 + (lane & 15);
        if (row < rows && col < K) gst(Z, (size_t)row * g.ng_max + col, make_double2(cre[i][j][r], cim[i][j][r]));
      }
}

// rows: tile rows, 64 in FP64 (128 only for the BF16 parts).
hipError_t launch_direct_s1(const GemmArgs* gs, const S1Tile* tiles, int ntiles, int precision, int mapped,
                            int rows, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (rows != 64 && rows != 128) return hipErrorInvalidValue;
  if (precision != BSE_FP64) return launch_direct_s1_mx(gs, tiles, ntiles, precision, rows, st);
  if (rows != 64) return hipErrorInvalidValue;
  void (*k)(const GemmArgs*, const S1Tile*) = mapped ? k_direct_s1<true> : k_direct_s1<false>;
  hipLaunchKernelGGL(k, dim3(ntiles), dim3(256), 0, st, gs, tiles);
  return hipGetLastError();
}

// ------------------------------------------------------------------ direct, stage 2 + assembly

// One wave per item (pair p of the chunk of system s, 16 x 16 tile (ti, tj) of
// vv' x cc').
__global__ __launch_bounds__(256) void k_direct_s2(const GemmArgs* __restrict__ gs, const int* __restrict__ d2off,
                                                   int nsys, int nitems) {
  const int lane = threadIdx.x & 63;
  const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= nitems) return;
  const int sys = item_system(d2off, nsys, item);
  const GemmArgs g = gs[sys];
  const int nv2 = g.rv_rows, nc2 = g.rc_rows;
  const int tiles_i = (nv2 + 15) / 16, tiles_j = (nc2 + 15) / 16;
  const int loc = item - d2off[sys];
  const int per = tiles_i * tiles_j;
  const int p = loc / per, ti = (loc % per) / tiles_j, tj = loc % tiles_j;  // p: pair of the chunk
  const int4 pr = gld(g.pairs, (size_t)g.p0 + p);
  const int ka = pr.x, kb = pr.y;
  const int K = gbl(g.ng)[pr.z];
  const int ia = ti * 16 + (lane & 15), jb = tj * 16 + (lane & 15);
  const double2* zr = g.Z + ((size_t)p * nv2 + (ia < nv2 ? ia : 0)) * g.ng_max;
  const double2* cr = g.RC + ((size_t)p * nc2 + (jb < nc2 ? jb : 0)) * g.ng_max;
  d4 cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
  // four K steps of loads in flight before their MFMAs (the same products in
  // the same order as one step at a time)
  constexpr int U = 4;
  for (int k0 = 0; k0 < K; k0 += 4 * U) {
    double2 a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + 4 * u + (lane >> 4);
      a[u] = (ia < nv2 && k < K) ? gld(zr, k) : make_double2(0.0, 0.0);
      b[u] = (jb < nc2 && k < K) ? gld(cr, k) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cre = mfma64(a[u].x, b[u].x, cre);
      cre = mfma64(-a[u].y, b[u].y, cre);
      cim = mfma64(a[u].x, b[u].y, cim);
      cim = mfma64(a[u].y, b[u].x, cim);
    }
  }
  // mixed precisions: the q = 0 head of W, left out of their stage 1, in FP64
  const bool head = pr.z == 0 && g.w_head_fp64;
  const double2 w00 = head ? gld(g.W0, 0) : make_double2(0.0, 0.0);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = ti * 16 + 4 * r + (lane >> 4);
    const int j = tj * 16 + (lane & 15);
    if (i < nv2 && j < nc2) {
      double dr = cre[r], di = cim[r];
      if (head) {
        const double2 rv0 = gld(g.RV, ((size_t)p * nv2 + i) * g.ng_max);
        const double2 rc0 = gld(g.RC, ((size_t)p * nc2 + j) * g.ng_max);
        const double2 hw = cmul(cconjmul(rv0, w00), rc0);
        dr += hw.x;
        di += hw.y;
      }
      // direct term: rows (v, v') and (c, c'); coupling block: rows (v, c') and (c, v')
      const int v = g.coupling ? i / g.nc : i / g.nv, v2 = g.coupling ? j % g.nv : i % g.nv;
      const int c = g.coupling ? j / g.nv : j / g.nc, c2 = g.coupling ? i % g.nc : j % g.nc;
      const size_t S = ((size_t)ka * g.nv + v) * g.nc + c;
      const size_t S2 = ((size_t)kb * g.nv + v2) * g.nc + c2;
      double2 h = gld(g.H, S * g.ldh + S2);
      h.x -= g.cpref * dr;
      h.y -= g.cpref * di;
      if (S == S2 && !g.coupling) {  // e_{c,k+Q} - e_{v,k}
        const int kc = g.kq ? gbl(g.kq)[ka] : ka;
        h.x += gbl(g.eps)[(size_t)kc * g.nb + g.nv + c] - gbl(g.eps)[(size_t)ka * g.nb + v];
      }
      gst(g.H, S * g.ldh + S2, h);
    }
  }
}

// Stage 2 reads each Z and rho_cc' row once (HBM-bound), so it runs in FP64
// in every precision mode.
hipError_t launch_direct_s2(const GemmArgs* gs, const int* d2off, int nsys, int nitems, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_direct_s2, dim3((nitems + 3) / 4), dim3(256), 0, st, gs, d2off, nsys, nitems);
  return hipGetLastError();
}

// ------------------------------------------------------------------ mirror

// Destination tile (i, j), i >= j, of 32 x 32: lower-k-block entries become the
// conjugate of the transposed source tile (j, i).
__global__ __launch_bounds__(256) void k_mirror(const GemmArgs* __restrict__ gs, const HTile* __restrict__ tiles) {
  __shared__ double2 tile[32][33];
  const HTile tl = tiles[blockIdx.x];
  const GemmArgs g = gs[tl.sys];
  double2* H = g.H;
  const int ns = g.ns, nt = g.nt;
  const size_t ld = g.ldh;
  const int bi = tl.i, bj = tl.j;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
#pragma unroll
  for (int r = ty; r < 32; r += 8) {
    const int sr = bj * 32 + r, sc = bi * 32 + tx;
    tile[r][tx] = (sr < ns && sc < ns) ? gld(H, (size_t)sr * ld + sc) : make_double2(0.0, 0.0);
  }
  __syncthreads();
#pragma unroll
  for (int r = ty; r < 32; r += 8) {
    const int dr = bi * 32 + r, dc = bj * 32 + tx;
    if (dr < ns && dc < ns && dr / nt > dc / nt) {
      const double2 v = tile[tx][r];
      gst(H, (size_t)dr * ld + dc, make_double2(v.x, g.mirror_plain ? v.y : -v.y));
    }
  }
}

hipError_t launch_mirror(const GemmArgs* gs, const HTile* tiles, int ntiles, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mirror, dim3(ntiles), dim3(256), 0, st, gs, tiles);
  return hipGetLastError();
}

// ------------------------------------------------------------------ beyond Tamm-Dancoff

// Exchange B operand of the coupling block: the h-e densities n_{ck,vk}(G) =
// conj(n_{vk,ck}(-G)), scaled like X (v is even in G).
__global__ void k_xbar(const double2* __restrict__ X, const int* __restrict__ inv, int ns, int ng0, int ng_max,
                       double2* __restrict__ Xb) {
  const size_t n = (size_t)ns * ng_max;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
    const int g = (int)(id % ng_max);
    double2 v = make_double2(0.0, 0.0);
    if (g < ng0) {
      const double2 x = gld(X, id - g + gbl(inv)[g]);
      v = make_double2(x.x, -x.y);
    }
    gst(Xb, id, v);
  }
}

hipError_t launch_xbar(const double2* X, const int* inv, int ns, int ng0, int ng_max, double2* Xb, hipStream_t st) {
  hipLaunchKernelGGL(k_xbar, dim3(4096), dim3(256), 0, st, X, inv, ns, ng0, ng_max, Xb);
  return hipGetLastError();
}

// Lower half of H2 = [[A, B], [-B^H, -conj(A)]] (the h-e rows of Sec. II.C's
// basis carry the opposite occupation factor; with Hermitian,
// time-reversal-consistent W the h-e kernel blocks are those of the e-h rows
// conjugated).  32 x 32 tiles through LDS for the transposed block.
__global__ __launch_bounds__(256) void k_full_lower(double2* __restrict__ H2, int ns) {
  __shared__ double2 tile[32][33];
  const int T = (ns + 31) / 32;
  const int bi = blockIdx.x / T, bj = blockIdx.x % T;
  const size_t ld = 2 * (size_t)ns;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // -conj(A) into the bottom-right block
#pragma unroll
  for (int r = ty; r < 32; r += 8) {
    const int i = bi * 32 + r, j = bj * 32 + tx;
    if (i < ns && j < ns) {
      const double2 a = gld(H2, (size_t)i * ld + j);
      gst(H2, (size_t)(ns + i) * ld + ns + j, make_double2(-a.x, a.y));
    }
  }
  // -B^H into the bottom-left block: element (i, j) from B[j][i]
#pragma unroll
  for (int r = ty; r < 32; r += 8) {
    const int sr = bj * 32 + r, sc = bi * 32 + tx;
    tile[r][tx] = (sr < ns && sc < ns) ? gld(H2, (size_t)sr * ld + ns + sc) : make_double2(0.0, 0.0);
  }
  __syncthreads();
#pragma unroll
  for (int r = ty; r < 32; r += 8) {
    const int i = bi * 32 + r, j = bj * 32 + tx;
    if (i < ns && j < ns) {
      const double2 b = tile[tx][r];
      gst(H2, (size_t)(ns + i) * ld + j, make_double2(-b.x, b.y));
    }
  }
}

hipError_t launch_full_lower(double2* H2, int ns, hipStream_t st) {
  const int T = (ns + 31) / 32;
  hipLaunchKernelGGL(k_full_lower, dim3(T * T), dim3(256), 0, st, H2, ns);
  return hipGetLastError();
}

// ------------------------------------------------------------------ sqrt v(G)

// The short-range exchange of Eq. V_eh leaves out G = 0 (entry g0 of the
// sphere of the exciton momentum; -1 when that sphere does not hold it).
__global__ void k_vscale(const double* __restrict__ vx, int ngx, int ng_max, int g0, double* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < ng_max) out[g] = (g == g0 || g >= ngx) ? 0.0 : sqrt(vx[g]);
}

hipError_t launch_vscale(const double* vx, int ngx, int ng_max, int g0, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_vscale, dim3((ng_max + 255) / 256), dim3(256), 0, st, vx, ngx, ng_max, g0, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ counters

__global__ void k_zero_u32(unsigned* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

__global__ void k_zero_f64(double* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

hipError_t launch_zero_f64(double* p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace bse
