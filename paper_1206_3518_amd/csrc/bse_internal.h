// Internal helpers shared by the HIP kernels of the BSE Hamiltonian builder.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace bse {

// ---------------------------------------------------------------- complex

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// acc + a * b
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}

// ---------------------------------------------------------------- roots of unity
// cos(2 pi k / 48) on the first quadrant; every twiddle of a register FFT of
// length dividing 48 is one of these up to sign.
constexpr double kCosQ48[13] = {
    1.0,
    9.91444861373810411145e-1,
    9.6592582628906828675e-1,
    9.23879532511286756128e-1,
    8.66025403784438646764e-1,
    7.9335334029123516458e-1,
    7.07106781186547524401e-1,
    6.08761429008720639416e-1,
    5.0e-1,
    3.82683432365089771728e-1,
    2.58819045102520762349e-1,
    1.30526192220051591548e-1,
    0.0};

constexpr double cos48(int k) {
  k = ((k % 48) + 48) % 48;
  return k <= 12 ? kCosQ48[k] : k <= 24 ? -kCosQ48[24 - k] : k <= 36 ? -kCosQ48[k - 24] : kCosQ48[48 - k];
}
constexpr double sin48(int k) { return cos48(k - 12); }

// exp(-2 pi i k / M) for M dividing 48
template <int M>
__device__ __forceinline__ double2 root(int k) {
  static_assert(48 % M == 0, "register FFT length must divide 48");
  return make_double2(cos48(k * (48 / M)), -sin48(k * (48 / M)));
}

// ---------------------------------------------------------------- register FFT
// In-place forward DFT (exp(-2 pi i)) of M points held by one lane, natural
// order in and out.  Decimation in time on radix 2 and 3.

template <int M, int S = 1>
struct RegFFT;

template <int S>
struct RegFFT<1, S> {
  template <int N>
  __device__ __forceinline__ static void run(double2 (&)[N], int) {}
};

template <int M, int S>
struct RegFFT {
  // operates on x[off + S*i], i < M
  template <int N>
  __device__ __forceinline__ static void run(double2 (&x)[N], int off) {
    if constexpr (M % 2 == 0) {
      constexpr int H = M / 2;
      RegFFT<H, 2 * S>::run(x, off);      // even samples
      RegFFT<H, 2 * S>::run(x, off + S);  // odd samples
      double2 t[M];
#pragma unroll
      for (int k = 0; k < H; ++k) {
        double2 e = x[off + 2 * S * k];
        double2 o = cmul(x[off + 2 * S * k + S], root<M>(k));
        t[k] = cadd(e, o);
        t[k + H] = csub(e, o);
      }
#pragma unroll
      for (int k = 0; k < M; ++k) x[off + S * k] = t[k];
    } else {
      static_assert(M % 3 == 0, "register FFT radices are 2 and 3");
      constexpr int T = M / 3;
      RegFFT<T, 3 * S>::run(x, off);
      RegFFT<T, 3 * S>::run(x, off + S);
      RegFFT<T, 3 * S>::run(x, off + 2 * S);
      double2 t[M];
      constexpr double c3 = -0.5;                         // cos(2 pi / 3)
      constexpr double s3 = 8.66025403784438646764e-1;    // sin(2 pi / 3)
#pragma unroll
      for (int k = 0; k < T; ++k) {
        double2 a = x[off + 3 * S * k];
        double2 b = cmul(x[off + 3 * S * k + S], root<M>(k));
        double2 c = cmul(x[off + 3 * S * k + 2 * S], root<M>(2 * k));
        double2 sbc = cadd(b, c), dbc = csub(b, c);
        double2 m = make_double2(a.x + c3 * sbc.x, a.y + c3 * sbc.y);
        // -i * s3 * (b - c) for the exp(-2 pi i/3) branch
        double2 r = make_double2(s3 * dbc.y, -s3 * dbc.x);
        t[k] = cadd(a, sbc);
        t[k + T] = cadd(m, r);
        t[k + 2 * T] = csub(m, r);
      }
#pragma unroll
      for (int k = 0; k < M; ++k) x[off + S * k] = t[k];
    }
  }
};

// ---------------------------------------------------------------- wave utilities

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double2 shfl_xor2(double2 v, int mask) {
  return make_double2(__shfl_xor(v.x, mask, 64), __shfl_xor(v.y, mask, 64));
}

// ---------------------------------------------------------------- packed Miller indices
// (m1, m2, m3) with |m_d| < 512 packed into one int.
__host__ __device__ __forceinline__ int pack_m(int m1, int m2, int m3) {
  return ((m1 + 512) << 20) | ((m2 + 512) << 10) | (m3 + 512);
}
__host__ __device__ __forceinline__ void unpack_m(int p, int& m1, int& m2, int& m3) {
  m1 = ((p >> 20) & 1023) - 512;
  m2 = ((p >> 10) & 1023) - 512;
  m3 = (p & 1023) - 512;
}

__host__ __device__ __forceinline__ int imod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

}  // namespace bse
