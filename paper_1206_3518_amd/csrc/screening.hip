// Static RPA screened interaction W(q) from the wave functions (Eq. chi0_GG
// at omega = 0, Eq. epsilon_-1 with the RPA kernel, Sec. III.A for W):
//   chi0_GG'(q) = (2/Omega) sum_k sum_{occupied n, empty n' (both orders)}
//                 (f_nk - f_n'k+q) n(G) conj(n(G')) / (e_nk - e_n'k+q)
//   eps = 1 - v^1/2 chi0 v^1/2 = 1 + sum_r Y_r Y_r^H,
//   Y_r(G) = n_r(G) sqrt(2 / (Omega D_r)) sqrt(v(q+G)),  D_r = e_empty - e_occupied > 0
//   W = v^1/2 eps^-1 v^1/2
// The pair densities n_r come from the pair-density kernel (ordered pairs
// (k, k+q), occupied x empty and empty x occupied band blocks).
//   k_rpa_scale   Y rows from the pair densities, in place
//   k_rpa_init    eps(q) = identity on the sphere (zero padding)
//   k_rpa_herk    eps(q) += conj(Y^H Y) over the chunk's rows of q (FP64 MFMA),
//                 64 x 64 tiles on and above the diagonal
//   k_rpa_mirror  the tiles below the diagonal as the conjugate transpose
//   k_rpa_invert  eps(q)^-1 in place by Gauss-Jordan elimination (Hermitian
//                 positive definite: no pivoting)
//   k_rpa_w       W = v^1/2 eps^-1 v^1/2, the q = 0 head set, wings zero
// The output holds one matrix per slot, slot i for q = qof[i] (every q, or
// only the irreducible q points of Sec. III.A).
//   k_rpa_fill    the empty x occupied rows of (k, k+q) from the occupied x
//                 empty rows of (k+q, k), whose transfer is qbar = -q - t:
//                 n_{ck, v k+q}(G) = conj(n_{v k+q, c k}(t - G)) (conjugating
//                 the integrand exchanges the states and reverses the transfer)
#include "bse_internal.h"
#include "gemm_tiles.h"
#include "kernels.h"

namespace bse {

// One workgroup per k pair of the chunk: 2 nv nc rows (occupied x empty, then
// empty x occupied) scaled in place.
__global__ __launch_bounds__(256) void k_rpa_scale(RpaArgs a) {
  const int p = blockIdx.x;  // pair of the chunk: (q_local, k)
  const int4 pk = a.pk[p];   // (k, k + q, q, -)
  const int k = pk.x, kq = pk.y, q = pk.z;
  const int nv = a.nv, nc = a.nc, nb = nv + nc, ngm = a.ng_max;
  const int ngq = a.ng[q];
  const int per = nv * nc;
  double2* Y = a.Y + (size_t)p * 2 * per * ngm;
  for (int e = threadIdx.x; e < 2 * per * ngm; e += blockDim.x) {
    const int r = e / ngm, g = e - r * ngm;
    double d;
    if (r < per) {  // occupied v at k, empty c at k + q: row v nc + c
      const int v = r / nc, c = r % nc;
      d = a.eps[(size_t)kq * nb + nv + c] - a.eps[(size_t)k * nb + v];
    } else {  // empty c at k, occupied v at k + q: row c nv + v
      const int c = (r - per) / nv, v = (r - per) % nv;
      d = a.eps[(size_t)k * nb + nv + c] - a.eps[(size_t)kq * nb + v];
    }
    const double dh = d * (1.0 / 27.211386245988);
    double s = 0.0;
    if (g < ngq && !(q == 0 && g == 0)) s = sqrt(2.0 / (a.omega * dh) * a.vq[(size_t)q * ngm + g]);
    const double2 x = Y[e];
    Y[e] = make_double2(x.x * s, x.y * s);
  }
}

// One workgroup per item (destination row base, source row base, q): the nc nv
// rows (c, v) from the source's nv nc rows (v, c), raw densities (before
// k_rpa_scale); entries past ng(q) are zero.
__global__ __launch_bounds__(256) void k_rpa_fill(double2* __restrict__ Y, const int4* __restrict__ items,
                                                  const int* __restrict__ trmap, const int* __restrict__ ng, int nv,
                                                  int nc, int ng_max) {
  const int4 it = items[blockIdx.x];
  const int q = it.z, ngq = ng[q];
  const int* map = trmap + (size_t)q * ng_max;
  double2* dst = Y + (size_t)it.x * ng_max;
  const double2* src = Y + (size_t)it.y * ng_max;
  const int total = nv * nc * ng_max;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int r = e / ng_max, g = e - r * ng_max;  // r = c nv + v
    const int c = r / nv, v = r - c * nv;
    double2 x = make_double2(0.0, 0.0);
    if (g < ngq) {
      x = src[(size_t)(v * nc + c) * ng_max + map[g]];
      x.y = -x.y;
    }
    dst[(size_t)r * ng_max + g] = x;
  }
}

__global__ void k_rpa_init(double2* __restrict__ M, const int* __restrict__ ng, const int* __restrict__ qof,
                           int nslot, int ng_max) {
  const size_t per = (size_t)ng_max * ng_max;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < per * nslot;
       id += (size_t)gridDim.x * blockDim.x) {
    const int q = qof[id / per];
    const int g = (int)((id % per) / ng_max), h = (int)(id % ng_max);
    M[id] = make_double2((g == h && g < ng[q]) ? 1.0 : 0.0, 0.0);
  }
}

// Tile (slot, i, j) of 64 x 64: M_q[G][G'] += conj(sum_r conj(Y_r(G)) Y_r(G'))
// over the rows of q = qof[slot] in the chunk (A transposed: A[G][r] = Y[r][G]).
// Three waves per SIMD: the upper tiles of every q of a chunk then run in one
// round of workgroups (each sums over all rows of its q, so rounds dominate).
// A chunk of few q splits the row sum into nsplit slices (a tile per slice):
// slice s writes its partial sum to part[s][q_local], and k_rpa_reduce adds
// the slices to eps in slice order.
__global__ __launch_bounds__(256, 3) void k_rpa_herk(RpaArgs a, const int4* __restrict__ tiles) {
  const int4 tl = tiles[blockIdx.x];  // (slot, row tile | slice << 8, column tile, q_local)
  const int slot = tl.x, q = a.qof[slot], ql = tl.w, sl = tl.y >> 8;
  const int ngm = a.ng_max, ngq = a.ng[q];
  const int rows = a.nk * 2 * a.nv * a.nc;
  const int rs = (rows + 16 * a.nsplit - 1) / (16 * a.nsplit) * 16;  // rows per slice
  const int rb = min(rows, sl * rs), re = min(rows, rb + rs);
  const double2* Yq = a.Y + ((size_t)ql * rows + rb) * ngm;
  const int r0 = (tl.y & 255) * 64, c0 = tl.z * 64;
  d4 cre[2][2], cim[2][2];
  tile_gemm<true, false, true>(Yq, ngm, r0, ngq, Yq, ngm, c0, ngq, re - rb, cre, cim);
  const bool split = a.nsplit > 1;
  double2* M = split ? a.part + ((size_t)sl * a.part_q + ql) * ngm * ngm : a.M + (size_t)slot * ngm * ngm;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + wr * 32 + i * 16 + 4 * r + (lane >> 4);
        const int col = c0 + wc * 32 + j * 16 + (lane & 15);
        if (row < ngq && col < ngq) {
          double2 m = split ? make_double2(0.0, 0.0) : M[(size_t)row * ngm + col];
          m.x += cre[i][j][r];
          m.y -= cim[i][j][r];
          M[(size_t)row * ngm + col] = m;
        }
      }
}

// eps of the chunk's q (cslot: slot of each q_local) += the nsplit partial
// sums, slice after slice, on the tiles on and above the diagonal.
__global__ void k_rpa_reduce(RpaArgs a, const int* __restrict__ cslot, int nql) {
  const int ngm = a.ng_max;
  const size_t per = (size_t)ngm * ngm;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < per * nql;
       id += (size_t)gridDim.x * blockDim.x) {
    const int ql = (int)(id / per);
    const int g = (int)((id % per) / ngm), h = (int)(id % ngm);
    const int slot = cslot[ql], n = a.ng[a.qof[slot]];
    if (g >= n || h >= n || (g >> 6) > (h >> 6)) continue;
    double2 m = a.M[(size_t)slot * per + (size_t)g * ngm + h];
    for (int sl = 0; sl < a.nsplit; ++sl) {
      const double2 v = a.part[((size_t)sl * a.part_q + ql) * per + (size_t)g * ngm + h];
      m.x += v.x;
      m.y += v.y;
    }
    a.M[(size_t)slot * per + (size_t)g * ngm + h] = m;
  }
}

hipError_t launch_rpa_reduce(const RpaArgs& a, const int* cslot, int nql, hipStream_t st) {
  if (nql <= 0 || a.nsplit <= 1) return hipSuccess;
  hipLaunchKernelGGL(k_rpa_reduce, dim3(4096), dim3(256), 0, st, a, cslot, nql);
  return hipGetLastError();
}

// Entries in 64 x 64 tiles below the diagonal: M[h][g] = conj(M[g][h]).
__global__ void k_rpa_mirror(double2* __restrict__ M, const int* __restrict__ ng, const int* __restrict__ qof,
                             int nslot, int ng_max) {
  const size_t per = (size_t)ng_max * ng_max;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < per * nslot;
       id += (size_t)gridDim.x * blockDim.x) {
    const size_t slot = id / per;
    const int h = (int)((id % per) / ng_max), g = (int)(id % ng_max);
    const int n = ng[qof[slot]];
    if (h >= n || g >= n || (h >> 6) <= (g >> 6)) continue;
    const double2 v = M[slot * per + (size_t)g * ng_max + h];
    M[id] = make_double2(v.x, -v.y);
  }
}

// In-place inverse of the Hermitian positive definite M_q (n = ng(q), leading
// dimension ng_max), one workgroup per q.  Step k: with the pivot p = M[k][k],
// row k becomes M[k][j] / p (entry k: 1 / p) and every other row i loses
// M[i][k] times the new row k (entry k: -M[i][k] / p).
constexpr int kRpaMaxG = 1024;
__global__ __launch_bounds__(1024) void k_rpa_invert(double2* __restrict__ M, const int* __restrict__ ng,
                                                     const int* __restrict__ qof, int ng_max) {
  __shared__ double2 col[kRpaMaxG], row[kRpaMaxG];
  const int slot = blockIdx.x, n = ng[qof[slot]];
  double2* A = M + (size_t)slot * ng_max * ng_max;
  for (int k = 0; k < n; ++k) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      col[i] = A[(size_t)i * ng_max + k];
      row[i] = A[(size_t)k * ng_max + i];
    }
    __syncthreads();
    const double2 p = col[k];
    const double den = p.x * p.x + p.y * p.y;
    const double2 pinv = make_double2(p.x / den, -p.y / den);
    for (size_t e = threadIdx.x; e < (size_t)n * n; e += blockDim.x) {
      const int i = (int)(e / n), j = (int)(e - (size_t)i * n);
      const double2 rk = j == k ? pinv : cmul(row[j], pinv);  // new row k, entry j
      double2 v;
      if (i == k) {
        v = rk;
      } else {
        const double2 f = col[i];
        v = j == k ? make_double2(-(f.x * rk.x - f.y * rk.y), -(f.x * rk.y + f.y * rk.x))
                   : csub(A[(size_t)i * ng_max + j], cmul(f, rk));
      }
      A[(size_t)i * ng_max + j] = v;
    }
    __syncthreads();
  }
}

__global__ void k_rpa_w(double2* __restrict__ M, const int* __restrict__ ng, const int* __restrict__ qof,
                        const double* __restrict__ vq, int nslot, int ng_max, double head) {
  const size_t per = (size_t)ng_max * ng_max;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < per * nslot;
       id += (size_t)gridDim.x * blockDim.x) {
    const int q = qof[id / per];
    const int g = (int)((id % per) / ng_max), h = (int)(id % ng_max);
    const int n = ng[q];
    double2 w = make_double2(0.0, 0.0);
    if (g < n && h < n) {
      if (q == 0 && (g == 0 || h == 0)) {
        w = make_double2(g == 0 && h == 0 ? head : 0.0, 0.0);
      } else {
        const double s = sqrt(vq[(size_t)q * ng_max + g] * vq[(size_t)q * ng_max + h]);
        const double2 m = M[id];
        w = make_double2(s * m.x, s * m.y);
      }
    }
    M[id] = w;
  }
}

hipError_t launch_rpa_scale(const RpaArgs& a, int npairs, hipStream_t st) {
  if (npairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rpa_scale, dim3(npairs), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_rpa_fill(double2* Y, const int4* items, int nitems, const int* trmap, const int* ng, int nv, int nc,
                          int ng_max, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rpa_fill, dim3(nitems), dim3(256), 0, st, Y, items, trmap, ng, nv, nc, ng_max);
  return hipGetLastError();
}

hipError_t launch_rpa_init(double2* M, const int* ng, const int* qof, int nslot, int ng_max, hipStream_t st) {
  hipLaunchKernelGGL(k_rpa_init, dim3(8192), dim3(256), 0, st, M, ng, qof, nslot, ng_max);
  return hipGetLastError();
}

hipError_t launch_rpa_herk(const RpaArgs& a, const int4* tiles, int ntiles, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rpa_herk, dim3(ntiles), dim3(256), 0, st, a, tiles);
  return hipGetLastError();
}

hipError_t launch_rpa_mirror(double2* M, const int* ng, const int* qof, int nslot, int ng_max, hipStream_t st) {
  hipLaunchKernelGGL(k_rpa_mirror, dim3(8192), dim3(256), 0, st, M, ng, qof, nslot, ng_max);
  return hipGetLastError();
}

hipError_t launch_rpa_invert(double2* M, const int* ng, const int* qof, int nslot, int ng_max, hipStream_t st) {
  if (ng_max > kRpaMaxG) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rpa_invert, dim3(nslot), dim3(1024), 0, st, M, ng, qof, ng_max);
  return hipGetLastError();
}

hipError_t launch_rpa_w(double2* M, const int* ng, const int* qof, const double* vq, int nslot, int ng_max,
                        double head, hipStream_t st) {
  hipLaunchKernelGGL(k_rpa_w, dim3(8192), dim3(256), 0, st, M, ng, qof, vq, nslot, ng_max, head);
  return hipGetLastError();
}

}  // namespace bse
