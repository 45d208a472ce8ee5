// Internal helpers shared by the HIP kernels of the BSE Hamiltonian builder.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

namespace bse {

// Global-memory access through pointers read from a table in memory (rather
// than from the kernel arguments): the compiler treats those as generic and
// emits flat accesses, which also wait on the LDS counter.  These casts give
// global loads and stores.  gbl() is for scalar element types; complex
// elements go through gld()/gst() on a builtin two-double vector.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gbl(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
typedef double gd2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 gld(const double2* p, size_t i) {
  const gd2 v = ((const __attribute__((address_space(1))) gd2*)p)[i];
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void gst(double2* p, size_t i, double2 x) {
  gd2 v;
  v.x = x.x;
  v.y = x.y;
  ((__attribute__((address_space(1))) gd2*)p)[i] = v;
}
__device__ __forceinline__ int4 gld(const int4* p, size_t i) {
  const int* q = reinterpret_cast<const int*>(p) + 4 * i;
  return make_int4(gbl(q)[0], gbl(q)[1], gbl(q)[2], gbl(q)[3]);
}
// one 16-byte global load (p 16-byte aligned)
typedef unsigned gu4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 gld16(const void* p) {
  const gu4 v = *(const __attribute__((address_space(1))) gu4*)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}

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
// c ? a : b per component (a conditional on the vector class itself would
// select between addresses and push register arrays into scratch memory)
__device__ __forceinline__ double2 csel(bool c, double2 a, double2 b) {
  return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}
// acc + a * b
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}

// The same in single precision (FP32 pair densities).
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconjmul(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 acc) {
  return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y)));
}

// Complex value of the type of C from its parts.
template <class C>
__device__ __forceinline__ C mkc(double re, double im) {
  if constexpr (sizeof(C) == 8)
    return make_float2((float)re, (float)im);
  else
    return make_double2(re, im);
}

// ---------------------------------------------------------------- roots of unity
// cos(2 pi k / 96) on the first quadrant; every twiddle of a transform whose
// length divides 96 is one of these up to sign.
constexpr double kCosQ96[25] = {
    1.0,
    9.97858923238603506738e-1,
    9.91444861373810411145e-1,
    9.80785280403230449126e-1,
    9.6592582628906828675e-1,
    9.46930129495105664256e-1,
    9.23879532511286756128e-1,
    8.96872741532688303894e-1,
    8.66025403784438646764e-1,
    8.31469612302545237079e-1,
    7.9335334029123516458e-1,
    7.51839807478977396408e-1,
    7.07106781186547524401e-1,
    6.59345815100068868425e-1,
    6.08761429008720639416e-1,
    5.55570233019602224743e-1,
    5.0e-1,
    4.42288690219001281995e-1,
    3.82683432365089771728e-1,
    3.21439465303161580701e-1,
    2.58819045102520762349e-1,
    1.95090322016128267848e-1,
    1.30526192220051591548e-1,
    6.54031292301430668153e-2,
    0.0};

constexpr double cos96(int k) {
  k = ((k % 96) + 96) % 96;
  return k <= 24 ? kCosQ96[k] : k <= 48 ? -kCosQ96[48 - k] : k <= 72 ? -kCosQ96[k - 48] : kCosQ96[96 - k];
}
constexpr double sin96(int k) { return cos96(k - 24); }

// Calls f(std::integral_constant<int, I>) for I = B .. E-1, so that loop
// indices are compile-time constants inside f.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// x * exp(-2 pi i K / M), M dividing 96.  Multiples of a quarter and an eighth
// turn need no general complex product.
template <int M, int K, class C>
__device__ __forceinline__ C cmul_root(C x) {
  static_assert(96 % M == 0, "transform length must divide 96");
  using R = decltype(x.x);
  constexpr int k = ((K % M) + M) % M;
  constexpr R r = (R)7.07106781186547524401e-1;
  C y;
  if constexpr (k == 0) {
    return x;
  } else if constexpr (2 * k == M) {
    y.x = -x.x;
    y.y = -x.y;
  } else if constexpr (4 * k == M) {  // -i
    y.x = x.y;
    y.y = -x.x;
  } else if constexpr (4 * k == 3 * M) {  // +i
    y.x = -x.y;
    y.y = x.x;
  } else if constexpr (8 * k == M) {
    y.x = r * (x.x + x.y);
    y.y = r * (x.y - x.x);
  } else if constexpr (8 * k == 3 * M) {
    y.x = r * (x.y - x.x);
    y.y = -r * (x.x + x.y);
  } else if constexpr (8 * k == 5 * M) {
    y.x = -r * (x.x + x.y);
    y.y = r * (x.x - x.y);
  } else if constexpr (8 * k == 7 * M) {
    y.x = r * (x.x - x.y);
    y.y = r * (x.x + x.y);
  } else {
    constexpr R c = (R)cos96(k * (96 / M)), s = (R)-sin96(k * (96 / M));
    y.x = fma(x.x, c, -x.y * s);
    y.y = fma(x.x, s, x.y * c);
  }
  return y;
}

// ---------------------------------------------------------------- register FFT
// In-place forward DFT (exp(-2 pi i)) of M points held by one lane, on
// x[OFF + S*i] for i < M (natural order in).  Decimation in time on radix 2
// and 3 with every butterfly writing back into its own input slots, so no
// temporaries are live; output f ends in slot OFF + S * fft_pos<M>(f).

template <int M>
__host__ __device__ constexpr int fft_pos(int f) {
  if constexpr (M == 1) {
    return 0;
  } else if constexpr (M % 2 == 0) {
    return f < M / 2 ? 2 * fft_pos<M / 2>(f) : 2 * fft_pos<M / 2>(f - M / 2) + 1;
  } else {
    static_assert(M % 3 == 0, "register FFT radices are 2 and 3");
    return 3 * fft_pos<M / 3>(f % (M / 3)) + f / (M / 3);
  }
}

template <int M, int S, int OFF, class C, int N>
__device__ __forceinline__ void reg_fft(C (&x)[N]) {
  using R = decltype(x[0].x);
  if constexpr (M == 1) {
    return;
  } else if constexpr (M % 2 == 0) {
    constexpr int H = M / 2;
    reg_fft<H, 2 * S, OFF>(x);      // even samples
    reg_fft<H, 2 * S, OFF + S>(x);  // odd samples
    static_for<0, H>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr int pe = OFF + 2 * S * fft_pos<H>(k);  // E_k; O_k sits S further
      const C e = x[pe];
      const C o = cmul_root<M, k>(x[pe + S]);
      x[pe] = cadd(e, o);      // output k
      x[pe + S] = csub(e, o);  // output k + H
    });
  } else {
    static_assert(M % 3 == 0, "register FFT radices are 2 and 3");
    constexpr int T = M / 3;
    reg_fft<T, 3 * S, OFF>(x);
    reg_fft<T, 3 * S, OFF + S>(x);
    reg_fft<T, 3 * S, OFF + 2 * S>(x);
    constexpr R c3 = (R)-0.5;                        // cos(2 pi / 3)
    constexpr R s3 = (R)8.66025403784438646764e-1;  // sin(2 pi / 3)
    static_for<0, T>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr int pa = OFF + 3 * S * fft_pos<T>(k);
      const C a = x[pa];
      const C b = cmul_root<M, k>(x[pa + S]);
      const C c = cmul_root<M, 2 * k>(x[pa + 2 * S]);
      const C sbc = cadd(b, c), dbc = csub(b, c);
      C m, r;
      m.x = fma(c3, sbc.x, a.x);
      m.y = fma(c3, sbc.y, a.y);
      r.x = s3 * dbc.y;  // -i s3 (b - c)
      r.y = -s3 * dbc.x;
      x[pa] = cadd(a, sbc);         // output k
      x[pa + S] = cadd(m, r);       // output k + T
      x[pa + 2 * S] = csub(m, r);   // output k + 2T
    });
  }
}

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
