// Input checks of BSE_VALIDATE: non-finite values in the inputs, and the
// symmetries the build relies on: W(q) Hermitian and, where the spheres are
// closed under time reversal, W_{t-G,t-G'}(qbar) = conj(W_GG'(q)) (Sec. III.A
// with T = 1).  Deviations are reduced to maxima with 64-bit atomics on the
// bit patterns of non-negative doubles (their order is that of the values).
#include "bse_internal.h"
#include "kernels.h"

namespace bse {

__device__ __forceinline__ void amax(unsigned long long* p, double v) {
  atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

__global__ void k_scan_finite(const double* __restrict__ x, size_t n, unsigned* __restrict__ bad) {
  unsigned found = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    found |= isfinite(x[i]) ? 0u : 1u;
  if (found) atomicOr(bad, 1u);
}

// One thread per (q, g, h) with g, h < ng(q): max |W|, max Hermiticity and
// time-reversal deviations.
__global__ void k_scan_W(const double2* __restrict__ W, const int* __restrict__ ng, const int* __restrict__ qbar,
                         const int* __restrict__ trmap, int nk, int ng_max, int check_tr,
                         unsigned long long* __restrict__ out) {
  const size_t per = (size_t)ng_max * ng_max;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < per * nk;
       id += (size_t)gridDim.x * blockDim.x) {
    const int q = (int)(id / per);
    const int g = (int)((id % per) / ng_max), h = (int)(id % ng_max);
    const int n = ng[q];
    if (g >= n || h >= n) continue;
    const double2 w = W[id];
    const double2 wt = W[(size_t)q * per + (size_t)h * ng_max + g];
    double m = fabs(w.x) + fabs(w.y);
    double dh = fabs(w.x - wt.x) + fabs(w.y + wt.y);
    double dt = 0.0;
    if (check_tr) {
      const int qb = qbar[q];
      const int gb = trmap[(size_t)q * ng_max + g], hb = trmap[(size_t)q * ng_max + h];
      const double2 wr = W[(size_t)qb * per + (size_t)gb * ng_max + hb];
      dt = fabs(w.x - wr.x) + fabs(w.y + wr.y);
    }
    if (!isfinite(m) || !isfinite(dh) || !isfinite(dt)) {
      m = dh = dt = INFINITY;
    }
    amax(out + 0, m);
    amax(out + 1, dh);
    amax(out + 2, dt);
  }
}

// One thread per element of u at points k with kbar != k: max |u| and max
// deviation from the time-reversal image of the partner point.
__global__ void k_scan_u_tr(const double2* __restrict__ u, const int* __restrict__ ktr, int nk, int nb, int N1,
                            int N2, int N3, unsigned long long* __restrict__ out) {
  const size_t nr = (size_t)N1 * N2 * N3, per = nr * nb;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < per * nk;
       id += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(id / per);
    const size_t rest = id % per;
    const int j = (int)(rest % nr);
    const int j1 = j / (N2 * N3), j2 = (j / N3) % N2, j3 = j % N3;
    const int t = ktr[k];
    const int kb = t & 0xffffff;
    if (kb == k) continue;  // no relation is assumed at a point that is its own partner
    const double f = ((t >> 24) & 1) * (double)j1 / N1 + ((t >> 25) & 1) * (double)j2 / N2 +
                     ((t >> 26) & 1) * (double)j3 / N3;
    double s, c;
    sincospi(-2.0 * f, &s, &c);
    const double2 a = u[id];
    const double2 b = u[(size_t)kb * per + rest];
    // exp(-i K.r) conj(a)
    const double ex = c * a.x + s * a.y, ey = s * a.x - c * a.y;
    double m = fabs(a.x) + fabs(a.y);
    double d = fabs(b.x - ex) + fabs(b.y - ey);
    if (!isfinite(m) || !isfinite(d)) m = d = INFINITY;
    amax(out + 3, m);
    amax(out + 4, d);
  }
}

hipError_t launch_validate_u_tr(const double2* u, const int* ktr, int nk, int nb, int N1, int N2, int N3,
                                unsigned long long* wstat, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_u_tr, dim3(2048), dim3(256), 0, st, u, ktr, nk, nb, N1, N2, N3, wstat);
  return hipGetLastError();
}

hipError_t launch_validate(const double* u, size_t nu, const double* eps, size_t ne, const double* vx, size_t nvx,
                           const double2* W, const int* ng, const int* qbar, const int* trmap, int nk, int ng_max,
                           int check_tr, unsigned* bad, unsigned long long* wstat, hipStream_t st) {
  const dim3 blk(256), grid(2048);
  hipLaunchKernelGGL(k_scan_finite, grid, blk, 0, st, u, nu, bad + 0);
  hipLaunchKernelGGL(k_scan_finite, grid, blk, 0, st, eps, ne, bad + 1);
  hipLaunchKernelGGL(k_scan_finite, grid, blk, 0, st, vx, nvx, bad + 2);
  hipLaunchKernelGGL(k_scan_W, grid, blk, 0, st, W, ng, qbar, trmap, nk, ng_max, check_tr, wstat);
  return hipGetLastError();
}

}  // namespace bse
