// Pair densities of k pairs that are time-reversal images of computed ones
// (Sec. III.A, the transformation of the pair density with T the identity
// combined with time reversal).  With u_{n,kbar} = exp(-i K.r) conj(u_{n,k})
// for kbar the mesh point of -k (-k = kbar - K):
//   pair (kbar, kbar') with kbar <= kbar':  n_{a kbar, b kbar'}(G) =
//     conj(n_{a k, b k'}(G'')), q + G'' = -(qbar + G) -- the sphere map of W;
//   pair (kbar', kbar) with kbar' < kbar:   n_{a kbar', b kbar}(G) = n_{b k, a k'}(G),
//     the same q and sphere, bands exchanged.
// Both are gathers over rows of ng(q) values: HBM-bound, a small fraction of
// the transforms they replace.
// The coupling block of the beyond-TDA matrix needs no symmetry of u: for any
// ordered pair, conjugating the integrand of the pair density exchanges the
// two states and reverses the momentum transfer, so
//   n_{c k, v' k'}(G) = conj(n_{v' k', c k}(G'')),  G'' = t - G,  -q = qbar + t,
// the same sphere map; the (c, v') rows of (k, k') come from the (v', c) rows
// of (k', k).
#include "bse_internal.h"
#include "kernels.h"

namespace bse {

// One workgroup per item: every band pair row of the destination pair (both
// pairs of the current chunk).  kind 1: valence rows, 2: conduction rows (time
// reversal); 3: coupling rows, destination (c, v') rows of it.x (nc x nv) from
// source (v, c') rows of it.y (nv x nc).
__global__ void __launch_bounds__(256) k_tr_fill(const TrArgs* __restrict__ as, const int4* __restrict__ items,
                                                 int kind) {
  const int4 it = items[blockIdx.x];
  const TrArgs a = as[it.w];
  const int n = kind == 1 ? a.nv : a.nc;
  const int ngm = a.ng_max;
  const int q = it.z >> 1, mode = kind == 3 ? 2 : it.z & 1;
  const int ngq = gbl(a.ng)[q];
  const size_t rows = kind == 3 ? (size_t)a.nv * a.nc : (size_t)n * n;
  const double2* src = (kind == 2 ? a.rc : a.rv) + (size_t)it.y * rows * ngm;
  double2* dst = (kind == 1 ? a.rv : a.rc) + (size_t)it.x * rows * ngm;
  const auto* map = gbl(a.trmap + (size_t)q * ngm);
  const int total = (int)rows * ngq;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int r = e / ngq, g = e - r * ngq;
    double2 v;
    if (mode == 2) {  // row (c, v') <- conj of row (v', c) at t - G
      const int c = r / a.nv, vp = r - c * a.nv;
      v = gld(src, (size_t)(vp * a.nc + c) * ngm + map[g]);
      v.y = -v.y;
    } else if (mode == 0) {
      v = gld(src, (size_t)r * ngm + map[g]);
      v.y = -v.y;
    } else {
      const int ra = r / n, rb = r - ra * n;
      v = gld(src, (size_t)(rb * n + ra) * ngm + g);
    }
    gst(dst, (size_t)r * ngm + g, v);
  }
}

hipError_t launch_tr_fill(const TrArgs* as, const int4* items, int nitems, int kind, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tr_fill, dim3(nitems), dim3(256), 0, st, as, items, kind);
  return hipGetLastError();
}

}  // namespace bse
