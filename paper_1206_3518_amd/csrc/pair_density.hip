// Pair densities n_{ak,bk'}(G) = sum_r conj(u_ak(r)) u_bk'(r) exp(-i (G - G0).r)
// on the plane-wave sphere of q (charge density matrix, Sec. II.B of the paper).
//
// One workgroup (4 waves) takes a job: one ordered k pair (k, k') and a block
// of nA x nB band pairs.  Each wave takes band pairs one at a time and sweeps
// the real-space planes j1 of the grid:
//   pass 1  product conj(u_a) u_b on the plane, FFT along j3 (register FFT of
//           M3 points per lane, then an L3-point DFT across lanes), keep the
//           F3 frequencies of the output window -> LDS T1[f3][j2];
//   pass 2  FFT along j2 of the F3 columns, keep F2 -> LDS T2[f2][f3];
//   pass 3  every lane owns sphere points g and accumulates
//           T2[f2_g][f3_g] * exp(-2 pi i f1_g j1 / N1) over the planes.
// Nothing but the pruned F2 x F3 window of a plane ever leaves registers, and
// the sphere values are written once at the end.
#include "bse_internal.h"
#include "kernels.h"

namespace bse {

template <int N>
struct Split;  // N = L * M: L lanes per row, M points per lane (register FFT)
template <> struct Split<8>  { static constexpr int L = 2, M = 4; };
template <> struct Split<12> { static constexpr int L = 2, M = 6; };
template <> struct Split<16> { static constexpr int L = 4, M = 4; };
template <> struct Split<24> { static constexpr int L = 4, M = 6; };
template <> struct Split<32> { static constexpr int L = 4, M = 8; };
template <> struct Split<48> { static constexpr int L = 4, M = 12; };
template <> struct Split<64> { static constexpr int L = 8, M = 8; };
template <> struct Split<96> { static constexpr int L = 8, M = 12; };

template <int L>
__device__ __forceinline__ int bitrev(int l) {
  if constexpr (L == 1) return 0;
  if constexpr (L == 2) return l;
  if constexpr (L == 4) return ((l & 1) << 1) | (l >> 1);
  if constexpr (L == 8) return ((l & 1) << 2) | (l & 2) | (l >> 2);
}

// L-point DFT across the L lanes of a row group, for each of the M values a
// lane holds.  Radix-2 decimation in frequency with xor shuffles; afterwards
// lane l holds output index bitrev(l).  tw[t] = exp(-2 pi i t / N), L | N.
template <int L, int M>
__device__ __forceinline__ void cross_lane_dft(double2 (&x)[M], int l, const double2* tw, int N) {
#pragma unroll
  for (int h = L / 2; h >= 1; h >>= 1) {
    const int p = l & (2 * h - 1);
    const bool upper = p >= h;
    const double2 w = tw[(p & (h - 1)) * (N / (2 * h))];
#pragma unroll
    for (int f = 0; f < M; ++f) {
      double2 o = shfl_xor2(x[f], h);
      x[f] = upper ? cmul(csub(o, x[f]), w) : cadd(x[f], o);
    }
  }
}

// Full row transform: x holds samples l + L*s (s < M) of a length-N row;
// afterwards x[f'] holds output f' + M * bitrev(l).
template <int N, int M>
__device__ __forceinline__ void row_fft(double2 (&x)[M], int l, const double2* tw) {
  constexpr int L = Split<N>::L;
  RegFFT<M>::run(x, 0);
#pragma unroll
  for (int f = 1; f < M; ++f) x[f] = cmul(x[f], tw[(l * f) % N]);
  cross_lane_dft<L, M>(x, l, tw, N);
}

template <int N2, int N3>
__global__ __launch_bounds__(256) void k_pair_density(PdArgs a) {
  constexpr int L3 = Split<N3>::L, M3 = Split<N3>::M, R1 = 64 / L3;
  constexpr int L2 = Split<N2>::L, M2 = Split<N2>::M, C2 = 64 / L2;
  constexpr int I1 = (N2 + R1 - 1) / R1;
  extern __shared__ double2 smem[];
  const int N1 = a.N1, F2 = a.F2, F3 = a.F3, ngm = a.ng_max;
  // LDS: twiddles | per wave (T1, T2, acc) | gather table
  double2* tw1 = smem;
  double2* tw2 = tw1 + N1;
  double2* tw3 = tw2 + N2;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int per_wave = F3 * N2 + F2 * F3 + ngm;
  double2* T1 = tw3 + N3 + wave * per_wave;
  double2* T2 = T1 + F3 * N2;
  double2* acc = T2 + F2 * F3;
  int2* gtab = reinterpret_cast<int2*>(tw3 + N3 + 4 * per_wave);

  for (int t = threadIdx.x; t < N1 + N2 + N3; t += blockDim.x) {
    const int n = t < N1 ? N1 : (t < N1 + N2 ? N2 : N3);
    const int k = t < N1 ? t : (t < N1 + N2 ? t - N1 : t - N1 - N2);
    double s, c;
    sincospi(2.0 * k / n, &s, &c);
    smem[t] = make_double2(c, -s);
  }
  const PdJob job = a.jobs[blockIdx.x];
  const int nA = job.nab & 255, nB = job.nab >> 8;
  int m01, m02, m03;
  unpack_m(job.m0p, m01, m02, m03);
  const int ngq = a.ng[job.iq];
  const int* gq = a.gpack + (size_t)job.iq * ngm;
  // sphere point g: offset of (f2, f3) in the plane window and f1 mod N1
  for (int g = threadIdx.x; g < ngq; g += blockDim.x) {
    int m1, m2, m3;
    unpack_m(gq[g], m1, m2, m3);
    gtab[g] = make_int2((m2 - m02 - a.lo2) * F3 + (m3 - m03 - a.lo3), imod(m1 - m01, N1));
  }
  __syncthreads();
  const float inv_n1 = 1.0f / (float)N1;

  const size_t Nr = (size_t)N1 * N2 * N3;
  for (int p = wave; p < nA * nB; p += 4) {
    const int ia = p / nB, ib = p % nB;
    const double2* ua = a.u + ((size_t)job.ka * a.nb + job.a0 + ia) * Nr;
    const double2* ub = a.u + ((size_t)job.kb * a.nb + job.b0 + ib) * Nr;
    for (int g = lane; g < ngq; g += 64) acc[g] = make_double2(0.0, 0.0);
    for (int j1 = 0; j1 < N1; ++j1) {
      // pass 1: rows of the plane
#pragma unroll 1
      for (int it = 0; it < I1; ++it) {
        const int j2 = it * R1 + lane / L3, l = lane % L3;
        const bool ok = j2 < N2;
        const size_t base = ((size_t)j1 * N2 + (ok ? j2 : 0)) * N3 + l;
        double2 x[M3];
#pragma unroll
        for (int s = 0; s < M3; ++s)
          x[s] = ok ? cconjmul(ua[base + L3 * s], ub[base + L3 * s]) : make_double2(0.0, 0.0);
        row_fft<N3, M3>(x, l, tw3);
        const int br = bitrev<L3>(l);
#pragma unroll
        for (int f = 0; f < M3; ++f) {
          const int a3 = imod(f + M3 * br - a.lo3, N3);
          if (ok && a3 < F3) T1[a3 * N2 + j2] = x[f];
        }
      }
      wave_sync();
      // pass 2: columns of the kept j3 frequencies
      for (int it = 0; it * C2 < F3; ++it) {
        const int col = it * C2 + lane / L2, l = lane % L2;
        const bool ok = col < F3;
        double2 x[M2];
#pragma unroll
        for (int s = 0; s < M2; ++s) x[s] = ok ? T1[col * N2 + l + L2 * s] : make_double2(0.0, 0.0);
        row_fft<N2, M2>(x, l, tw2);
        const int br = bitrev<L2>(l);
#pragma unroll
        for (int f = 0; f < M2; ++f) {
          const int a2 = imod(f + M2 * br - a.lo2, N2);
          if (ok && a2 < F2) T2[a2 * F3 + col] = x[f];
        }
      }
      wave_sync();
      // pass 3: direct sum over planes at the sphere points
      for (int g = lane; g < ngq; g += 64) {
        const int2 e = gtab[g];
        int r = e.y * j1;  // < 2^24, exact in float
        r -= N1 * (int)((float)r * inv_n1);
        r += r < 0 ? N1 : 0;
        r -= r >= N1 ? N1 : 0;
        acc[g] = cfma(T2[e.x], tw1[r], acc[g]);
      }
      wave_sync();
    }
    double2* o = a.out + (size_t)(job.row0 + p) * ngm;
    for (int g = lane; g < ngm; g += 64) {
      if (g < ngq) {
        const double sc = a.vscale ? a.vscale[g] : 1.0;
        const double2 v = acc[g];
        o[g] = make_double2(v.x * sc, v.y * sc);
      } else {
        o[g] = make_double2(0.0, 0.0);
      }
    }
    wave_sync();
  }
}

size_t pd_lds_bytes(int N1, int N2, int N3, int F2, int F3, int ng_max) {
  return sizeof(double2) * ((size_t)N1 + N2 + N3 + 4 * ((size_t)F3 * N2 + (size_t)F2 * F3 + ng_max)) +
         sizeof(int2) * (size_t)ng_max;
}

template <int N2, int N3>
static hipError_t launch_grid(const PdArgs& a, int njobs, hipStream_t st) {
  const size_t lds = pd_lds_bytes(a.N1, N2, N3, a.F2, a.F3, a.ng_max);
  auto k = k_pair_density<N2, N3>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(njobs), dim3(256), lds, st, a);
  return hipGetLastError();
}

bool pd_grid_supported(int N2, int N3) {
  return (N2 == N3 && (N2 == 8 || N2 == 12 || N2 == 16 || N2 == 24 || N2 == 32 || N2 == 48 || N2 == 64 ||
                       N2 == 96)) ||
         (N2 == 24 && N3 == 96) || (N2 == 12 && N3 == 16) || (N2 == 16 && N3 == 24);
}


hipError_t launch_pair_density(const PdArgs& a, int N2, int N3, int njobs, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
#define BSE_PD_CASE(X, Y) \
  if (N2 == X && N3 == Y) return launch_grid<X, Y>(a, njobs, st);
  BSE_PD_CASE(8, 8)
  BSE_PD_CASE(12, 12)
  BSE_PD_CASE(16, 16)
  BSE_PD_CASE(24, 24)
  BSE_PD_CASE(32, 32)
  BSE_PD_CASE(48, 48)
  BSE_PD_CASE(64, 64)
  BSE_PD_CASE(96, 96)
  BSE_PD_CASE(24, 96)
  BSE_PD_CASE(12, 16)
  BSE_PD_CASE(16, 24)
#undef BSE_PD_CASE
  return hipErrorInvalidValue;
}

}  // namespace bse
