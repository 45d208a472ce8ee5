// Adjoint of the Hamiltonian build (the map (W, eps) -> H of Sec. II.C with
// the upper k blocks computed and the lower ones mirrored).
//
// With Gbar = dL/dRe H + i dL/dIm H and dL = Re sum conj(Gbar) dH, an upper
// block (k <= k') enters through Gbar_eff = Gbar + Gbar^H (k < k': the mirrored
// lower block adds its conjugate transpose) or Gbar (k = k'), and
//   T[(kk' vv')][g']   = sum_{cc'} Gbar_eff[(k v c),(k' v' c')] conj(rho_cc'(g'))   (k_adj_T)
//   dL/dW_q[g][g']     = -c sum_{pairs of q, vv'} rho_vv'(g) T[(kk' vv')][g']       (k_adj_dW, MFMA)
//   dL/de_c(k+Q) = sum_v Re Gbar_SS,  dL/de_vk = -sum_c Re Gbar_SS, S = (k v c)      (k_adj_deps)
// Optionally dW is projected onto Hermitian, time-reversal symmetric W by the
// group average over (g g') -> conj(g' g) and (q g g') -> conj(qbar, t-g, t-g')
// (Sec. III.A with T = 1).
#include "bse_internal.h"
#include "gemm_tiles.h"
#include "kernels.h"

namespace bse {

// The recomputed pair densities hold one chunk of k pairs at a time (rows of
// pair p of the chunk start at (p - p0) * nv^2); dW is accumulated over the
// chunks.
//
// T for one k pair and one 16-row block of vv', all g'.  f64 MFMA: A = Gbar_eff
// block (16 x 16 over vv' x cc'), B[cc'][g'] = conj(rho_cc'(g')).
__global__ __launch_bounds__(256) void k_adj_T(AdjArgs a, int tiles_i, int nitems) {
  const int lane = threadIdx.x & 63;
  const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= nitems) return;
  const int p = item / tiles_i, ti = item % tiles_i;  // p: pair of the chunk
  const int4 pr = a.pairs[a.p0 + p];
  const int ka = pr.x, kb = pr.y;
  const int K = a.ng[pr.z];
  const int nv = a.nv, nc = a.nc, nv2 = nv * nv, nc2 = nc * nc, ns = a.ns;
  const int i = ti * 16 + (lane & 15);  // vv' row of the A operand
  double2* T = a.T + (size_t)p * nv2 * a.ng_max;
  for (int n0 = 0; n0 < a.ng_max; n0 += 16) {
    d4 cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
    for (int kc = 0; kc < nc2; kc += 4) {
      const int j = kc + (lane >> 4);  // cc'
      double2 g = make_double2(0.0, 0.0);
      if (i < nv2 && j < nc2) {
        const int v = i / nv, v2 = i % nv, c = j / nc, c2 = j % nc;
        const size_t S = ((size_t)ka * nv + v) * nc + c;
        const size_t S2 = ((size_t)kb * nv + v2) * nc + c2;
        g = a.dH[S * ns + S2];
        if (ka != kb) {
          const double2 h = a.dH[S2 * ns + S];
          g.x += h.x;
          g.y -= h.y;
        }
      }
      const int n = n0 + (lane & 15);
      double2 b = make_double2(0.0, 0.0);
      if (j < nc2 && n < K) {
        const double2 r = a.RC[((size_t)p * nc2 + j) * a.ng_max + n];
        b = make_double2(r.x, -r.y);
      }
      // B operand of lane l: B[k = l/16][n = l%16]; A operand: A[i = l%16][k = l/16]
      cre = mfma64(g.x, b.x, cre);
      cre = mfma64(-g.y, b.y, cre);
      cim = mfma64(g.x, b.y, cim);
      cim = mfma64(g.y, b.x, cim);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = ti * 16 + 4 * r + (lane >> 4);
      const int col = n0 + (lane & 15);
      if (row < nv2 && col < a.ng_max)
        T[(size_t)row * a.ng_max + col] = col < K ? make_double2(cre[r], cim[r]) : make_double2(0.0, 0.0);
    }
  }
}

// dW_q tile += -c RV_q^T T_q over the chunk's pairs of q (A transposed:
// A[g][r] = RV[r][g]).  In the mixed precisions the q = 0 head entry is left
// to k_adj_head (FP64).
template <int P>
__global__ __launch_bounds__(256) void k_adj_dW(AdjArgs a) {
  const int4 tl = a.dwtiles[blockIdx.x];
  const int q = tl.x;
  const int nv2 = a.nv * a.nv;
  const int row_base = (a.qstart[q] - a.p0) * nv2;
  const int K = (a.qstart[q + 1] - a.qstart[q]) * nv2;
  const int ngq = a.ng[q];
  const double2* A = a.RV + (size_t)row_base * a.ng_max;
  const double2* Bm = a.T + (size_t)row_base * a.ng_max;
  const int r0 = tl.y * 64, c0 = tl.z * 64;
  double2* out = a.dWout + (size_t)q * a.ng_max * a.ng_max;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
  if constexpr (P == BSE_FP64) {
    d4 cre[2][2], cim[2][2];
    tile_gemm<false, false, true>(A, a.ng_max, r0, ngq, Bm, a.ng_max, c0, ngq, K, cre, cim);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + wr * 32 + i * 16 + 4 * r + (lane >> 4);
          const int col = c0 + wc * 32 + j * 16 + (lane & 15);
          if (row < a.ng_max && col < a.ng_max) {
            double2 o = out[(size_t)row * a.ng_max + col];
            o.x -= a.cpref * cre[i][j][r];
            o.y -= a.cpref * cim[i][j][r];
            out[(size_t)row * a.ng_max + col] = o;
          }
        }
  } else {
    f4 cre[2][2], cim[2][2];
    tile_gemm_mx<P, false, false, true>(A, a.ng_max, r0, ngq, Bm, a.ng_max, c0, ngq, K, false, cre, cim);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + wr * 32 + i * 16 + acc_row(lane, r);
          const int col = c0 + wc * 32 + j * 16 + (lane & 15);
          if (row < a.ng_max && col < a.ng_max && !(q == 0 && row == 0 && col == 0)) {
            double2 o = out[(size_t)row * a.ng_max + col];
            o.x -= a.cpref * (double)cre[i][j][r];
            o.y -= a.cpref * (double)cim[i][j][r];
            out[(size_t)row * a.ng_max + col] = o;
          }
        }
  }
}

// FP64 head entry dW_0[0][0] (mixed precision): one workgroup reduction over
// the chunk's pairs of q = 0, added to the entry.
__global__ __launch_bounds__(256) void k_adj_head(AdjArgs a) {
  __shared__ double sre[256], sim[256];
  const int nv2 = a.nv * a.nv;
  const int rows = (a.qstart[1] - a.qstart[0]) * nv2;
  const double2* A = a.RV + (size_t)(a.qstart[0] - a.p0) * nv2 * a.ng_max;
  const double2* Bm = a.T + (size_t)(a.qstart[0] - a.p0) * nv2 * a.ng_max;
  double re = 0.0, im = 0.0;
  for (int r = threadIdx.x; r < rows; r += 256) {
    const double2 x = A[(size_t)r * a.ng_max], y = Bm[(size_t)r * a.ng_max];
    re += x.x * y.x - x.y * y.y;
    im += x.x * y.y + x.y * y.x;
  }
  sre[threadIdx.x] = re;
  sim[threadIdx.x] = im;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sre[threadIdx.x] += sre[threadIdx.x + s];
      sim[threadIdx.x] += sim[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double2 o = a.dWout[0];
    o.x -= a.cpref * sre[0];
    o.y -= a.cpref * sim[0];
    a.dWout[0] = o;
  }
}

__global__ void k_adj_deps(AdjArgs a) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  const int nb = a.nv + a.nc;
  if (id >= a.nk * nb) return;
  const int k = id / nb, b = id % nb;
  double s = 0.0;
  if (b >= a.nv) {
    // the electron at k is that of the states whose hole sits at k - Q
    const int k1 = k / (a.kn[1] * a.kn[2]), k2 = (k / a.kn[2]) % a.kn[1], k3 = k % a.kn[2];
    const int kh = (((k1 - a.qe[0] + a.kn[0]) % a.kn[0]) * a.kn[1] + (k2 - a.qe[1] + a.kn[1]) % a.kn[1]) * a.kn[2] +
                   (k3 - a.qe[2] + a.kn[2]) % a.kn[2];
    const int c = b - a.nv;
    for (int v = 0; v < a.nv; ++v) {
      const size_t S = ((size_t)kh * a.nv + v) * a.nc + c;
      s += a.dH[S * a.ns + S].x;
    }
  } else {
    for (int c = 0; c < a.nc; ++c) {
      const size_t S = ((size_t)k * a.nv + b) * a.nc + c;
      s -= a.dH[S * a.ns + S].x;
    }
  }
  a.deps[id] = s;
}

// Orthogonal projection onto Hermitian, time-reversal symmetric W.
__global__ void k_adj_project(AdjArgs a, const double2* __restrict__ raw, double2* __restrict__ out) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t per = (size_t)a.ng_max * a.ng_max;
  if (id >= per * a.nk) return;
  const int q = (int)(id / per);
  const int g = (int)((id % per) / a.ng_max), h = (int)(id % a.ng_max);
  const int n = a.ng[q];
  if (g >= n || h >= n) {
    out[id] = make_double2(0.0, 0.0);
    return;
  }
  const int qb = a.qbar[q];
  const int gb = a.trmap[(size_t)q * a.ng_max + g], hb = a.trmap[(size_t)q * a.ng_max + h];
  const double2 x0 = raw[id];
  const double2 x1 = raw[(size_t)q * per + (size_t)h * a.ng_max + g];
  const double2 x2 = raw[(size_t)qb * per + (size_t)gb * a.ng_max + hb];
  const double2 x3 = raw[(size_t)qb * per + (size_t)hb * a.ng_max + gb];
  out[id] = make_double2(0.25 * (x0.x + x1.x + x2.x + x3.x), 0.25 * (x0.y - x1.y - x2.y + x3.y));
}

// ---------------------------------------------------------------- pair-density gradients
// With dL = Re sum conj(Gbar) dH and Geff as above (Gbar + Gbar^H on k < k',
// Gbar on k = k'), the densities of the upper pairs get
//   dL/drho_cc'(g') = -c sum_vv' Geff_SS' conj(Z_vv'(g')),  Z = conj(rho_vv')^T W  (= conj(W^H rho_vv'))
//   dL/drho_vv'(g)  = -c (W conj(T_vv'))(g),                 T = Geff conj(rho_cc')
// and the exchange densities (every block of H depends on them directly)
//   dL/dn_S(m)      = 2c sqrt v(m) [(conj(Gbar) + Gbar^T) Xs](S, m),  Xs = sqrt v n.

// One k pair and one 16-row block of cc', all g'.  f64 MFMA: A[cc'][vv'] =
// Geff_SS', B[vv'][g'] = conj(Z).
__global__ __launch_bounds__(256) void k_adj_drc(AdjArgs a, int tiles_i, int nitems) {
  const int lane = threadIdx.x & 63;
  const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= nitems) return;
  const int p = item / tiles_i, ti = item % tiles_i;  // p: pair of the chunk
  const int4 pr = a.pairs[a.p0 + p];
  const int ka = pr.x, kb = pr.y;
  const int K = a.ng[pr.z];
  const int nv = a.nv, nc = a.nc, nv2 = nv * nv, nc2 = nc * nc, ns = a.ns;
  const int i = ti * 16 + (lane & 15);  // cc' row of the A operand
  const double2* Z = a.Z + (size_t)p * nv2 * a.ng_max;
  double2* out = a.drc + (size_t)a.plex[a.p0 + p] * nc2 * a.ng_max;
  for (int n0 = 0; n0 < a.ng_max; n0 += 16) {
    d4 cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
    for (int kc = 0; kc < nv2; kc += 4) {
      const int j = kc + (lane >> 4);  // vv'
      double2 g = make_double2(0.0, 0.0);
      if (i < nc2 && j < nv2) {
        const int c = i / nc, c2 = i % nc, v = j / nv, v2 = j % nv;
        const size_t S = ((size_t)ka * nv + v) * nc + c;
        const size_t S2 = ((size_t)kb * nv + v2) * nc + c2;
        g = a.dH[S * ns + S2];
        if (ka != kb) {
          const double2 h = a.dH[S2 * ns + S];
          g.x += h.x;
          g.y -= h.y;
        }
      }
      const int n = n0 + (lane & 15);
      double2 b = make_double2(0.0, 0.0);
      if (j < nv2 && n < K) {
        const double2 z = Z[(size_t)j * a.ng_max + n];
        b = make_double2(z.x, -z.y);
      }
      cre = mfma64(g.x, b.x, cre);
      cre = mfma64(-g.y, b.y, cre);
      cim = mfma64(g.x, b.y, cim);
      cim = mfma64(g.y, b.x, cim);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = ti * 16 + 4 * r + (lane >> 4);
      const int col = n0 + (lane & 15);
      if (row < nc2 && col < a.ng_max)
        out[(size_t)row * a.ng_max + col] =
            col < K ? make_double2(-a.cpref * cre[r], -a.cpref * cim[r]) : make_double2(0.0, 0.0);
    }
  }
}

// dL/drho_vv' tile of a q group: C = conj(T) W_q^T (A = T rows of the group,
// B transposed), every column up to ng_max written.
__global__ __launch_bounds__(256) void k_adj_drv(AdjArgs a) {
  const int4 tl = a.rvtiles[blockIdx.x];
  const int q = tl.x;
  const int nv2 = a.nv * a.nv;
  const int row_base = (a.qstart[q] - a.p0) * nv2;  // rows of the chunk
  const int rows = (a.qstart[q + 1] - a.qstart[q]) * nv2;
  const int K = a.ng[q];
  const double2* A = a.T + (size_t)row_base * a.ng_max;
  const double2* Wq = a.W + (size_t)q * a.ng_max * a.ng_max;
  const int r0 = tl.y * 64, c0 = tl.z * 64;
  d4 cre[2][2], cim[2][2];
  tile_gemm<true, true>(A, a.ng_max, r0, rows, Wq, a.ng_max, c0, K, K, cre, cim);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + wr * 32 + i * 16 + 4 * r + (lane >> 4);
        const int col = c0 + wc * 32 + j * 16 + (lane & 15);
        if (row < rows && col < a.ng_max) {
          const int p = a.qstart[q] + row / nv2;
          double2* o = a.drv + ((size_t)a.plex[p] * nv2 + row % nv2) * a.ng_max;
          o[col] = col < K ? make_double2(-a.cpref * cre[i][j][r], -a.cpref * cim[i][j][r]) : make_double2(0.0, 0.0);
        }
      }
}

// dL/dn_S(m) tile (64 S x 64 m): conj(Gbar) Xs + Gbar^T Xs, K = NS.
__global__ __launch_bounds__(256) void k_adj_dx(AdjArgs a) {
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  d4 cre[2][2], cim[2][2];
  tile_gemm<true, false, false, true>(a.dH, a.ns, r0, a.ns, a.Xs, a.ng_max, c0, a.ngx, a.ns, cre, cim);
  tile_gemm<false, false, true, false>(a.dH, a.ns, r0, a.ns, a.Xs, a.ng_max, c0, a.ngx, a.ns, cre, cim);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + wr * 32 + i * 16 + 4 * r + (lane >> 4);
        const int col = c0 + wc * 32 + j * 16 + (lane & 15);
        if (row < a.ns && col < a.ng_max) {
          const double s = col < a.ngx ? 2.0 * a.cpref * a.vs[col] : 0.0;
          a.dX[(size_t)row * a.ng_max + col] = make_double2(s * cre[i][j][r], s * cim[i][j][r]);
        }
      }
}

hipError_t launch_adj_drc(const AdjArgs& a, hipStream_t st) {
  const int ti = (a.nc * a.nc + 15) / 16;
  const int nitems = a.npairs * ti;
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_drc, dim3((nitems + 3) / 4), dim3(256), 0, st, a, ti, nitems);
  return hipGetLastError();
}

hipError_t launch_adj_drv(const AdjArgs& a, int ntiles, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_drv, dim3(ntiles), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_adj_dx(const AdjArgs& a, hipStream_t st) {
  const dim3 grid((a.ng_max + 63) / 64, (a.ns + 63) / 64);
  hipLaunchKernelGGL(k_adj_dx, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_adjoint(const AdjArgs& a, int precision, int ndw_tiles, bool has_q0, hipStream_t st) {
  const int ti = (a.nv * a.nv + 15) / 16;
  const int nitems = a.npairs * ti;
  if (nitems > 0) {
    hipLaunchKernelGGL(k_adj_T, dim3((nitems + 3) / 4), dim3(256), 0, st, a, ti, nitems);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (a.dWout && ndw_tiles > 0) {
    if (precision == BSE_FP64) {
      hipLaunchKernelGGL(k_adj_dW<BSE_FP64>, dim3(ndw_tiles), dim3(256), 0, st, a);
    } else {
      const size_t lds = precision == BSE_BF16X3 ? 2 * sizeof(TileLds<BSE_BF16X3>) : 2 * sizeof(TileLds<BSE_SPLIT_FP32>);
      auto k = precision == BSE_BF16X3 ? k_adj_dW<BSE_BF16X3> : k_adj_dW<BSE_SPLIT_FP32>;
      hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, dim3(ndw_tiles), dim3(256), lds, st, a);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      if (has_q0) hipLaunchKernelGGL(k_adj_head, dim3(1), dim3(256), 0, st, a);
    }
  }
  return hipGetLastError();
}

hipError_t launch_adjoint_finish(const AdjArgs& a, bool project, hipStream_t st) {
  if (a.dWout && project) {
    const size_t n = (size_t)a.nk * a.ng_max * a.ng_max;
    hipLaunchKernelGGL(k_adj_project, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, a.dWout, a.dWfinal);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (a.deps) {
    const int n = a.nk * (a.nv + a.nc);
    hipLaunchKernelGGL(k_adj_deps, dim3((n + 255) / 256), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ W at the irreducible q points

// W(q) at every q from the matrices at the irreducible points (Sec. III.A):
// Wf[q][g][h] = W[src][map g][map h], conjugated for time-reversed images,
// zero past ng(q).
__global__ void k_unfold_w(const double2* __restrict__ W, const int* __restrict__ wsrc, const int* __restrict__ wmap,
                           const int* __restrict__ ng, int nk, int ng_max, double2* __restrict__ Wf) {
  const size_t per = (size_t)ng_max * ng_max;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < per * nk;
       id += (size_t)gridDim.x * blockDim.x) {
    const int q = (int)(id / per);
    const int g = (int)((id % per) / ng_max), h = (int)(id % ng_max);
    double2 v = make_double2(0.0, 0.0);
    if (g < ng[q] && h < ng[q]) {
      const int* mq = wmap + (size_t)q * ng_max;
      v = W[(size_t)wsrc[2 * q] * per + (size_t)mq[g] * ng_max + mq[h]];
      if (wsrc[2 * q + 1]) v.y = -v.y;
    }
    Wf[id] = v;
  }
}

// The adjoint of the unfolding: dW[s][a][b] = sum over the q that map to s (in
// increasing q: qlist[csr[s]] .. qlist[csr[s+1]-1]) of dWf[q][inv a][inv b],
// conjugated for time-reversed images (PyTorch convention: conj(W) has the
// conjugate gradient); zero past the source's sphere.
__global__ void k_fold_dw(const double2* __restrict__ dWf, const int* __restrict__ csr, const int* __restrict__ qlist,
                          const int* __restrict__ wsrc, const int* __restrict__ winv, const int* __restrict__ ngirr,
                          int nirr, int ng_max, double2* __restrict__ dW) {
  const size_t per = (size_t)ng_max * ng_max;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < per * nirr;
       id += (size_t)gridDim.x * blockDim.x) {
    const int sidx = (int)(id / per);
    const int a = (int)((id % per) / ng_max), b = (int)(id % ng_max);
    double2 acc = make_double2(0.0, 0.0);
    if (a < ngirr[sidx] && b < ngirr[sidx]) {
      for (int t = csr[sidx]; t < csr[sidx + 1]; ++t) {
        const int q = qlist[t];
        const int* iq = winv + (size_t)q * ng_max;
        const double2 v = dWf[(size_t)q * per + (size_t)iq[a] * ng_max + iq[b]];
        acc.x += v.x;
        acc.y += wsrc[2 * q + 1] ? -v.y : v.y;
      }
    }
    dW[id] = acc;
  }
}

hipError_t launch_unfold_w(const double2* W, const int* wsrc, const int* wmap, const int* ng, int nk, int ng_max,
                           double2* Wf, hipStream_t st) {
  hipLaunchKernelGGL(k_unfold_w, dim3(8192), dim3(256), 0, st, W, wsrc, wmap, ng, nk, ng_max, Wf);
  return hipGetLastError();
}

hipError_t launch_fold_dw(const double2* dWf, const int* csr, const int* qlist, const int* wsrc, const int* winv,
                          const int* ngirr, int nirr, int ng_max, double2* dW, hipStream_t st) {
  hipLaunchKernelGGL(k_fold_dw, dim3(8192), dim3(256), 0, st, dWf, csr, qlist, wsrc, winv, ngirr, nirr, ng_max, dW);
  return hipGetLastError();
}

}  // namespace bse
