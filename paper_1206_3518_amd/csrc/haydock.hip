// Absorption spectrum from the resolvent of H without its eigenpairs: the
// Haydock recursion (Lanczos three-term recurrence from the dipole vector,
// then a continued fraction), for Hamiltonians too large to diagonalise.
// The spectral representation of the appendix (Eq. resolvent, Tamm-Dancoff
// so the overlap matrix is the identity) gives
//   sum_l |t_l|^2 eta / ((w - E_l)^2 + eta^2) = -Im v^H (w + i eta - H)^-1 v,
//   t_l = sum_S A[S][l] d_S,  v = conj(d),
// and m recurrence steps from v / |v| give (w + i eta - H)^-1 in that state
// as the continued fraction of the tridiagonal (a_j, b_j).
//   k_hy_init     q_0 = conj(d) / |d| per polarisation, q_-1 = 0
//   k_hy_hemv<NQ> Y = H Q for NQ vectors at once: one pass over H, HBM-bound
//   k_hy_step     a_j, the three-term update, b_j and q_{j+1} per polarisation
//   k_hy_eps2     the continued fractions on the frequency grid
#include "bse_internal.h"
#include "kernels.h"

namespace bse {

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

// Sum over the 1024 threads of a workgroup (16 waves).
__device__ double group_sum(double x, double* red) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();  // red may still be read from the previous call
  if (lane == 0) red[w] = x;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

// One workgroup per polarisation p: V0[p] = conj(d_p) / |d_p|, V1[p] = 0,
// norm2[p] = |d_p|^2.
__global__ __launch_bounds__(1024) void k_hy_init(const double2* __restrict__ d, int ns, double2* __restrict__ V0,
                                                  double2* __restrict__ V1, double* __restrict__ norm2) {
  __shared__ double red[16];
  const int p = blockIdx.x;
  const double2* dp = d + (size_t)p * ns;
  double s = 0.0;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    const double2 x = dp[i];
    s += x.x * x.x + x.y * x.y;
  }
  s = group_sum(s, red);
  const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    const double2 x = dp[i];
    V0[(size_t)p * ns + i] = make_double2(x.x * inv, -x.y * inv);
    V1[(size_t)p * ns + i] = make_double2(0.0, 0.0);
  }
  if (threadIdx.x == 0) norm2[p] = s;
}

// Y[p][r] = sum_c H[r][c] Q[p][c] for the NQ vectors Q[p] (p < nq; the rest
// of the NQ slots are zero).  A workgroup takes 4 kHyRows rows (kHyRows per
// wave); column chunks of 256 of Q go through LDS as [c][p]; lane l of a wave
// reads columns c0 + l + 64 i of its rows, 1 KB per row and load instruction.
constexpr int kHyCols = 256, kHyRows = 2;
template <int NQ>
__global__ __launch_bounds__(256) void k_hy_hemv(const double2* __restrict__ H, int ns, const double2* __restrict__ Q,
                                                 int nq, double2* __restrict__ Y) {
  __shared__ double2 qs[kHyCols][NQ];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = blockIdx.x * 4 * kHyRows + wave * kHyRows;
  double2 acc[kHyRows][NQ];
#pragma unroll
  for (int i = 0; i < kHyRows; ++i)
#pragma unroll
    for (int p = 0; p < NQ; ++p) acc[i][p] = make_double2(0.0, 0.0);
  for (int c0 = 0; c0 < ns; c0 += kHyCols) {
    __syncthreads();  // the previous chunk is consumed
    for (int e = threadIdx.x; e < kHyCols * NQ; e += blockDim.x) {
      const int p = e / kHyCols, c = e - p * kHyCols;
      qs[c][p] = (p < nq && c0 + c < ns) ? gld(Q, (size_t)p * ns + c0 + c) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    double2 h[kHyRows][kHyCols / 64];
#pragma unroll
    for (int i = 0; i < kHyRows; ++i) {
      const int r = r0 + i < ns ? r0 + i : 0;
#pragma unroll
      for (int t = 0; t < kHyCols / 64; ++t) {
        const int c = c0 + lane + 64 * t;
        h[i][t] = gld(H, (size_t)r * ns + (c < ns ? c : 0));
      }
    }
#pragma unroll
    for (int t = 0; t < kHyCols / 64; ++t) {
      double2 qv[NQ];
#pragma unroll
      for (int p = 0; p < NQ; ++p) qv[p] = qs[lane + 64 * t][p];  // zero past ns
#pragma unroll
      for (int i = 0; i < kHyRows; ++i)
#pragma unroll
        for (int p = 0; p < NQ; ++p) acc[i][p] = cfma(h[i][t], qv[p], acc[i][p]);
    }
  }
#pragma unroll
  for (int i = 0; i < kHyRows; ++i)
#pragma unroll
    for (int p = 0; p < NQ; ++p) {
      const double re = wave_sum(acc[i][p].x), im = wave_sum(acc[i][p].y);
      if (lane == 0 && r0 + i < ns && p < nq) gst(Y, (size_t)p * ns + r0 + i, make_double2(re, im));
    }
}

// Step j of the recurrence for polarisation p (one workgroup each):
//   w = Y - b_{j-1} q_{j-1};  a_j = Re q_j^H w;  w -= a_j q_j;  b_j = |w|;
//   q_{j+1} = w / b_j (zero once b_j vanishes: the Krylov space is exhausted
//   and the continued fraction ends there)
// Qc holds q_j, Qp holds q_{j-1} and receives q_{j+1}; coef[p][j] = (a_j, b_j).
__global__ __launch_bounds__(1024) void k_hy_step(const double2* __restrict__ Y, const double2* __restrict__ Qc,
                                                  double2* __restrict__ Qp, int ns, int j, int niter,
                                                  double* __restrict__ coef) {
  __shared__ double red[16];
  const int p = blockIdx.x;
  const double2* y = Y + (size_t)p * ns;
  const double2* qc = Qc + (size_t)p * ns;
  double2* qp = Qp + (size_t)p * ns;
  double* cp = coef + (size_t)p * niter * 2;
  const double bprev = j > 0 ? cp[2 * (j - 1) + 1] : 0.0;
  double s = 0.0;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    const double2 q = qc[i], yy = y[i], o = qp[i];
    // Re conj(q) (y - bprev o)
    s += q.x * (yy.x - bprev * o.x) + q.y * (yy.y - bprev * o.y);
  }
  const double a = group_sum(s, red);
  double n2 = 0.0;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    const double2 q = qc[i], yy = y[i], o = qp[i];
    const double2 w = make_double2(yy.x - bprev * o.x - a * q.x, yy.y - bprev * o.y - a * q.y);
    qp[i] = w;  // q_{j-1} is no longer needed
    n2 += w.x * w.x + w.y * w.y;
  }
  const double b = sqrt(group_sum(n2, red));
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    const double2 w = qp[i];
    qp[i] = make_double2(w.x * inv, w.y * inv);
  }
  if (threadIdx.x == 0) {
    cp[2 * j] = a;
    cp[2 * j + 1] = b;
  }
}

// eps2(w_i) = 8 pi / (Nk Omega_cell) (1/nq) sum_p |d_p|^2 (-Im g_p(w_i + i eta)),
// g(z) = 1 / (z - a_0 - b_0^2 / (z - a_1 - ... / (z - a_{m-1}))), every energy
// converted from eV to Hartree.
__global__ void k_hy_eps2(const double* __restrict__ coef, const double* __restrict__ norm2, int nq, int niter,
                          double nk_omega, int nw, double w0, double dw, double eta, double* __restrict__ eps2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nw) return;
  constexpr double ha = 1.0 / 27.211386245988;
  const double zr = w0 + dw * i, zi = eta;
  double s = 0.0;
  for (int p = 0; p < nq; ++p) {
    const double* c = coef + (size_t)p * niter * 2;
    // t = 1 / (z - a_{m-1}), then t = 1 / (z - a_j - b_j^2 t) down to j = 0
    double tr = 0.0, ti = 0.0;
    for (int j = niter - 1; j >= 0; --j) {
      const double a = c[2 * j] * ha;
      const double b2 = j < niter - 1 ? (c[2 * j + 1] * ha) * (c[2 * j + 1] * ha) : 0.0;
      const double dr = zr - a - b2 * tr, di = zi - b2 * ti;
      const double den = dr * dr + di * di;
      tr = dr / den;
      ti = -di / den;
    }
    s += norm2[p] * (-ti);
  }
  eps2[i] = 8.0 * 3.14159265358979323846 / nk_omega * s / nq;
}

hipError_t launch_haydock(int ns, const double2* H, const double2* d, int nq, int niter, double nk_omega, int nw,
                          double w0, double w1, double eta, double* eps2, double* coef, double2* V0, double2* V1,
                          double2* Y, double* norm2, hipStream_t st) {
  if (nq < 1 || nq > kMaxQhat || niter < 1 || ns < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_hy_init, dim3(nq), dim3(1024), 0, st, d, ns, V0, V1, norm2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid((ns + 4 * kHyRows - 1) / (4 * kHyRows)), blk(256);
  for (int j = 0; j < niter; ++j) {
    double2* Qc = (j & 1) ? V1 : V0;
    double2* Qp = (j & 1) ? V0 : V1;
    switch (nq) {
      case 1: hipLaunchKernelGGL(k_hy_hemv<1>, grid, blk, 0, st, H, ns, Qc, nq, Y); break;
      case 2: hipLaunchKernelGGL(k_hy_hemv<2>, grid, blk, 0, st, H, ns, Qc, nq, Y); break;
      case 3: hipLaunchKernelGGL(k_hy_hemv<3>, grid, blk, 0, st, H, ns, Qc, nq, Y); break;
      case 4: hipLaunchKernelGGL(k_hy_hemv<4>, grid, blk, 0, st, H, ns, Qc, nq, Y); break;
      default: hipLaunchKernelGGL(k_hy_hemv<8>, grid, blk, 0, st, H, ns, Qc, nq, Y); break;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hy_step, dim3(nq), dim3(1024), 0, st, Y, Qc, Qp, ns, j, niter, coef);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  constexpr double ha = 1.0 / 27.211386245988;
  const double dw = nw > 1 ? (w1 - w0) / (nw - 1) : 0.0;
  hipLaunchKernelGGL(k_hy_eps2, dim3((nw + 255) / 256), dim3(256), 0, st, coef, norm2, nq, niter, nk_omega, nw,
                     w0 * ha, dw * ha, eta * ha, eps2);
  return hipGetLastError();
}

}  // namespace bse
