// Optical spectrum from the spectral representation of the irreducible
// response (Sec. II.C, Tamm-Dancoff: overlap matrix = identity), and the k.p
// matrix elements <u_vk|grad|u_ck> it needs (Sec. II.B, q -> 0 limit of the
// pair density).
//   k_fft_axis     batched in-place DFT of full grids along one axis
//   k_grad         S_d = sum_m m_d conj(U_v(m)) U_c(m), Nyquist planes dropped,
//                  <u_v|grad|u_c> = (i / N_r) sum_d S_d b_d
//   k_dipole_project  d_S = qhat . <u_vk|grad|u_ck> / (e_ck - e_vk), Hartree units
//   k_spec_t       t_l = sum_S A[S][l] d[S], |t_l|^2 averaged over polarisations
//   k_spec_eps2    eps2(w) = 8 pi / (Nk Omega_cell) sum_l |t_l|^2 eta / ((w - E_l)^2 + eta^2)
#include "bse_internal.h"
#include "fft_row.h"
#include "kernels.h"

namespace bse {

// One wave = 64 / L lines of length N; line i of the batch starts at
// line_base(i) and has stride `stride`.  AX: 3 = contiguous axis (lines are
// consecutive rows), otherwise lines with consecutive j3 sit in consecutive
// lane groups so that loads coalesce across j3.
template <int N>
__global__ __launch_bounds__(256) void k_fft_axis(double2* __restrict__ data, int nlines, int N1, int N2, int N3,
                                                  int axis) {
  constexpr int L = Split<N>::L, M = Split<N>::M;
  __shared__ double2 tw[N];
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    double s, c;
    sincospi(2.0 * t / N, &s, &c);
    tw[t] = make_double2(c, -s);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave_global = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int line = wave_global * (64 / L) + lane / L;
  const int l = lane % L;
  const bool ok = line < nlines;
  size_t base = 0, stride = 1;
  const int li = ok ? line : 0;
  if (axis == 3) {  // line = (b, j1, j2)
    base = (size_t)li * N3;
    stride = 1;
  } else if (axis == 2) {  // line = (b, j1, j3)
    const int j3 = li % N3, r = li / N3;
    base = (size_t)r * N2 * N3 + j3;
    stride = N3;
  } else {  // line = (b, j2, j3)
    const int j23 = li % (N2 * N3), b = li / (N2 * N3);
    base = (size_t)b * N1 * N2 * N3 + j23;
    stride = (size_t)N2 * N3;
  }
  double2 x[M];
#pragma unroll
  for (int s = 0; s < M; ++s) x[s] = ok ? data[base + (size_t)(l + L * s) * stride] : make_double2(0.0, 0.0);
  row_fft<N, L, M>(x, l, tw);
  const int br = bitrev<L>(l);
  if (ok) {
    static_for<0, M>([&](auto fc) {
      constexpr int f = decltype(fc)::value;
      data[base + (size_t)(f + M * br) * stride] = x[fft_pos<M>(f)];
    });
  }
}

static hipError_t launch_fft_axis(double2* data, int batch, int N1, int N2, int N3, int axis, hipStream_t st) {
  const int N = axis == 1 ? N1 : axis == 2 ? N2 : N3;
  const int nlines = batch * (N1 * N2 * N3 / N);
#define BSE_FFT_CASE(X)                                                                            \
  if (N == X) {                                                                                    \
    const int per_block = 4 * (64 / Split<X>::L);                                                  \
    hipLaunchKernelGGL(k_fft_axis<X>, dim3((nlines + per_block - 1) / per_block), dim3(256), 0, st, \
                       data, nlines, N1, N2, N3, axis);                                           \
    return hipGetLastError();                                                                      \
  }
  BSE_FFT_CASE(8)
  BSE_FFT_CASE(12)
  BSE_FFT_CASE(16)
  BSE_FFT_CASE(24)
  BSE_FFT_CASE(32)
  BSE_FFT_CASE(48)
  BSE_FFT_CASE(64)
  BSE_FFT_CASE(96)
#undef BSE_FFT_CASE
  return hipErrorInvalidValue;
}

bool fft_len_supported(int N) {
  return N == 8 || N == 12 || N == 16 || N == 24 || N == 32 || N == 48 || N == 64 || N == 96;
}

__device__ double block_sum(double x, double* red) {
  red[threadIdx.x] = x;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

constexpr int kGradMaxC = 8;

// One workgroup per (k, v): sums over the grid for every c.
__global__ __launch_bounds__(256) void k_grad(const double2* __restrict__ U, int N1, int N2, int N3, int nv,
                                              int nc, GradCell bc, double2* __restrict__ out) {
  __shared__ double red[256];
  const int k = blockIdx.x / nv, v = blockIdx.x % nv;
  const int nb = nv + nc;
  const size_t Nr = (size_t)N1 * N2 * N3;
  const double2* uv = U + ((size_t)k * nb + v) * Nr;
  double acc[kGradMaxC][3][2];
#pragma unroll
  for (int c = 0; c < kGradMaxC; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) acc[c][d][0] = acc[c][d][1] = 0.0;
  for (size_t m = threadIdx.x; m < Nr; m += blockDim.x) {
    const int m3 = (int)(m % N3), m2 = (int)((m / N3) % N2), m1 = (int)(m / ((size_t)N2 * N3));
    // signed frequency; the Nyquist plane of an even axis contributes nothing
    const double f1 = (2 * m1 == N1) ? 0.0 : (m1 > N1 / 2 ? m1 - N1 : m1);
    const double f2 = (2 * m2 == N2) ? 0.0 : (m2 > N2 / 2 ? m2 - N2 : m2);
    const double f3 = (2 * m3 == N3) ? 0.0 : (m3 > N3 / 2 ? m3 - N3 : m3);
    const double2 a = uv[m];
#pragma unroll
    for (int c = 0; c < kGradMaxC; ++c) {
      if (c < nc) {
        const double2 b = U[((size_t)k * nb + nv + c) * Nr + m];
        const double2 p = cconjmul(a, b);
        acc[c][0][0] += f1 * p.x;
        acc[c][0][1] += f1 * p.y;
        acc[c][1][0] += f2 * p.x;
        acc[c][1][1] += f2 * p.y;
        acc[c][2][0] += f3 * p.x;
        acc[c][2][1] += f3 * p.y;
      }
    }
  }
  for (int c = 0; c < nc && c < kGradMaxC; ++c) {
    double S[3][2];
    for (int d = 0; d < 3; ++d) {
      S[d][0] = block_sum(acc[c][d][0], red);
      S[d][1] = block_sum(acc[c][d][1], red);
    }
    if (threadIdx.x < 3) {
      const int x = threadIdx.x;  // Cartesian component
      double re = 0.0, im = 0.0;
      for (int d = 0; d < 3; ++d) {
        re += S[d][0] * bc.b[d][x];
        im += S[d][1] * bc.b[d][x];
      }
      // times i / N_r
      out[(((size_t)k * nv + v) * nc + c) * 3 + x] = make_double2(-im / (double)Nr, re / (double)Nr);
    }
  }
}

hipError_t launch_grad(const double2* u, double2* scratch, int nk, int nb, int nv, int nc, int N1, int N2, int N3,
                       const GradCell& bc, double2* out, hipStream_t st) {
  const size_t n = (size_t)nk * nb * N1 * N2 * N3;
  hipError_t e = hipMemcpyAsync(scratch, u, n * sizeof(double2), hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  for (int axis = 3; axis >= 1; --axis) {
    e = launch_fft_axis(scratch, nk * nb, N1, N2, N3, axis, st);
    if (e != hipSuccess) return e;
  }
  if (nc > kGradMaxC) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_grad, dim3(nk * nv), dim3(256), 0, st, scratch, N1, N2, N3, nv, nc, bc, out);
  return hipGetLastError();
}

// Transition dipoles of nq polarisations:
//   d[q][S] = qhat_q . D[S] / ((e_ck - e_vk) / E_h),   D[S] = <u_vk|grad|u_ck> (bohr^-1)
// (Sec. II.B: the q -> 0 limit of n_{vk,ck}(0) divided by -i q, in Hartree
// atomic units).
__global__ void k_dipole_project(const double2* __restrict__ D, const double* __restrict__ eps, Qhats qh,
                                 int nq, int nk, int nv, int nc, double2* __restrict__ d) {
  const int ns = nk * nv * nc;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns * nq) return;
  const int q = i / ns, S = i - q * ns;
  const int k = S / (nv * nc), v = (S / nc) % nv, c = S % nc;
  const int nb = nv + nc;
  const double de = (eps[(size_t)k * nb + nv + c] - eps[(size_t)k * nb + v]) * (1.0 / 27.211386245988);
  double re = 0.0, im = 0.0;
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    const double2 g = D[(size_t)S * 3 + x];
    re += qh.v[q][x] * g.x;
    im += qh.v[q][x] * g.y;
  }
  d[i] = make_double2(re / de, im / de);
}

hipError_t launch_dipole_project(const double2* D, const double* eps, const Qhats& qh, int nq, int nk, int nv,
                                 int nc, double2* d, hipStream_t st) {
  const int n = nk * nv * nc * nq;
  if (n <= 0) return hipSuccess;
  if (nq > kMaxQhat) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dipole_project, dim3((n + 255) / 256), dim3(256), 0, st, D, eps, qh, nq, nk, nv, nc, d);
  return hipGetLastError();
}

// t2[l] = (1 / nq) sum_q |sum_S A[S][l] d[q][S]|^2: the oscillator strength of
// exciton l averaged over the polarisations
__global__ void k_spec_t(int ns, int nlam, int nq, const double2* __restrict__ A, const double2* __restrict__ d,
                         double* __restrict__ t2) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nlam) return;
  double acc = 0.0;
  for (int q = 0; q < nq; ++q) {
    const double2* dq = d + (size_t)q * ns;
    double re = 0.0, im = 0.0;
    for (int S = 0; S < ns; ++S) {
      const double2 a = A[(size_t)S * nlam + l], x = dq[S];
      re += a.x * x.x - a.y * x.y;
      im += a.x * x.y + a.y * x.x;
    }
    acc += re * re + im * im;
  }
  t2[l] = acc / nq;
}

// eps2(w) = 8 pi / (Nk Omega_cell) sum_l t2_l eta / ((w - E_l)^2 + eta^2), w and
// eta in Hartree (Sec. II.C; spin 2, Tamm-Dancoff overlap = identity)
__global__ void k_spec_eps2(int nlam, const double* __restrict__ E, const double* __restrict__ t2, double nk_omega,
                            int nw, double w0, double dw, double eta, double* __restrict__ eps2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nw) return;
  const double w = w0 + dw * i;
  double s = 0.0;
  for (int l = 0; l < nlam; ++l) {
    const double x = w - E[l] * (1.0 / 27.211386245988);
    s += t2[l] / (x * x + eta * eta);
  }
  eps2[i] = 8.0 * 3.14159265358979323846 / nk_omega * eta * s;
}

hipError_t launch_spectrum(int ns, int nlam, int nq, const double* E, const double2* A, const double2* d,
                           double nk_omega, int nw, double w0, double w1, double eta, double* t2, double* eps2,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_spec_t, dim3((nlam + 255) / 256), dim3(256), 0, st, ns, nlam, nq, A, d, t2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double ha = 1.0 / 27.211386245988;
  const double dw = nw > 1 ? (w1 - w0) / (nw - 1) : 0.0;
  hipLaunchKernelGGL(k_spec_eps2, dim3((nw + 255) / 256), dim3(256), 0, st, nlam, E, t2, nk_omega, nw, w0 * ha,
                     dw * ha, eta * ha, eps2);
  return hipGetLastError();
}

}  // namespace bse
