// Pair densities n_{ak,bk'}(G) = sum_r conj(u_ak(r)) u_bk'(r) exp(-i (G - G0).r)
// on the plane-wave sphere of q (charge density matrix, Sec. II.B of the paper).
//
// One workgroup (4 waves) takes a job: one ordered k pair (k, k') and a block
// of nA x nB band pairs.  A wave takes PW band pairs at a time and sweeps the
// real-space planes j1 of the grid; per plane and band pair:
//   pass 1  conj(u_a) u_b on the plane and an FFT along j3 (register FFT of M3
//           points per lane, then an L3-point DFT across lanes with DPP /
//           swizzle exchanges); the F3 kept frequencies go to LDS T1[f3][j2];
//   pass 2  FFT along j2 of the F3 kept columns; the F2 kept outputs are
//           written column-major over the columns already read (T2);
//   pass 3  every lane owns sphere points g = lane + 64 t and accumulates
//           T2[f3_g][f2_g] * exp(-2 pi i f1_g j1 / N1) in registers.
// Only the pruned window of a plane touches LDS; global memory sees the wave
// functions (read) and the sphere values (written once).
#include "bse_internal.h"
#include "fft_row.h"
#include "kernels.h"

namespace bse {

// Geometry of the two in-plane passes.  The plane is N2 x N3 (j3 fastest).
// Pass 1 transforms axis A straight from global memory, pass 2 the other axis
// B out of LDS.  AX = 2: columns (A = j2) in the layout lane = (column c,
// sub-lane l), sample s at row l + L*s, so one load instruction covers L whole
// rows; AX = 3: rows (A = j3), lane = (row r, sub-lane l), sample s at column
// l + L*s, which coalesces when L is large.
template <int N2, int N3>
struct PlaneGeo {
  static constexpr int AX = (N3 * Split<N2>::L <= 64) ? 2 : 3;
  static constexpr int NA = AX == 2 ? N2 : N3;   // pass-1 length
  static constexpr int NB = AX == 2 ? N3 : N2;   // pass-2 length (lines of pass 1)
  static constexpr int LA = Split<NA>::L, MA = Split<NA>::M;
  static constexpr int LB = SplitB<NB>::L, MB = SplitB<NB>::M;
  static constexpr int LINES = 64 / LA;          // pass-1 lines per iteration
  static constexpr int IA = (NB + LINES - 1) / LINES;
  static constexpr int SA = NB + 1;              // padded T1 row stride
  static constexpr int PW = 1;  // band pairs per wave
  // element (line, sample index i along A) of the plane
  __device__ static constexpr int at(int line, int i) { return AX == 2 ? i * N3 + line : line * N3 + i; }
};

// TG sphere points per lane (64 * TG >= ng_max).  EXCH: exchange set (rows
// scaled by sqrt v); a separate instantiation so that the direct-term
// launches form one kernel in traces.
template <int N2, int N3, int TG, bool EXCH>
__device__ __forceinline__ void pd_general_job(const PdArgs& a, const PdJob& job) {
  using G = PlaneGeo<N2, N3>;
  constexpr int LA = G::LA, MA = G::MA, LB = G::LB, MB = G::MB, NA = G::NA, NB = G::NB;
  constexpr int PW = G::PW, SA = G::SA;
  constexpr int LP = 64 / PW;  // lanes per band pair in pass 2
  constexpr int CB = LP / LB;  // pass-2 lines per iteration
  extern __shared__ double2 smem[];
  const int N1 = a.N1, ngm = a.ng_max;
  // window along the pass-1 axis (A) and the pass-2 axis (B)
  const int loA = G::AX == 2 ? a.lo2 : a.lo3, FA = G::AX == 2 ? a.F2 : a.F3;
  const int loB = G::AX == 2 ? a.lo3 : a.lo2, FB = G::AX == 2 ? a.F3 : a.F2;
  double2* tw1 = smem;
  double2* twA = tw1 + N1;
  double2* twB = twA + NA;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int per_pd = FA * SA;
  double2* T1 = twB + NB + wave * PW * per_pd;
  int2* gtab = reinterpret_cast<int2*>(twB + NB + 4 * PW * per_pd);

  for (int t = threadIdx.x; t < N1 + NA + NB; t += blockDim.x) {
    const int n = t < N1 ? N1 : (t < N1 + NA ? NA : NB);
    const int k = t < N1 ? t : (t < N1 + NA ? t - N1 : t - N1 - NA);
    double s, c;
    sincospi(2.0 * k / n, &s, &c);
    smem[t] = make_double2(c, -s);
  }
  const int nA = job.nab & 255, nB = (job.nab >> 8) & 255;
  int m01, m02, m03;
  unpack_m(job.m0p, m01, m02, m03);
  const int ngq = gbl(a.ng)[job.iq];
  const auto* gq = gbl(a.gpack + (size_t)job.iq * ngm);
  // sphere point g: offset of (fA, fB) in the column-major window, f1 mod N1
  for (int g = threadIdx.x; g < ngq; g += blockDim.x) {
    int m1, m2, m3;
    unpack_m(gq[g], m1, m2, m3);
    const int f2 = m2 - m02 - a.lo2, f3 = m3 - m03 - a.lo3;
    gtab[g] = make_int2(G::AX == 2 ? f2 * FB + f3 : f3 * FB + f2, imod(m1 - m01, N1));
  }
  __syncthreads();
  const float inv_n1 = 1.0f / (float)N1;

  // pass-1 lane geometry: outputs f' + MA * bitrev(lA) along A
  const int lA = lane % LA;
  const int bA = imod(MA * bitrev<LA>(lA) - loA, NA);
  // pass-2 lane geometry
  const int sub = PW == 2 ? lane >> 5 : 0;
  const int ll = PW == 2 ? lane & 31 : lane;
  const int lB = ll % LB;
  const int bB = imod(MB * bitrev<LB>(lB) - loB, NB);

  const int Nr = N1 * N2 * N3;
  const int npd = nA * nB;
  // band pairs of this wave: p = wave + 4 i; the PW pairs of one sweep share
  // the right operand when nB = 4
  for (int p0 = wave; p0 < npd; p0 += 4 * PW) {
    const int p1 = p0 + 4;
    const bool live1 = PW == 2 && p1 < npd;
    const int q1 = live1 ? p1 : p0;
    const double2* ua0 = a.u + ((size_t)job.ka * a.nb + job.a0 + p0 / nB) * Nr;
    const double2* ub0 = a.u + ((size_t)job.kb * a.nb + job.b0 + p0 % nB) * Nr;
    const double2* ua1 = a.u + ((size_t)job.ka * a.nb + job.a0 + q1 / nB) * Nr;
    const double2* ub1 = a.u + ((size_t)job.kb * a.nb + job.b0 + q1 % nB) * Nr;
    const bool share_b = ub1 == ub0;
    double2 acc[PW][TG];
#pragma unroll
    for (int t = 0; t < TG; ++t)
#pragma unroll
      for (int w = 0; w < PW; ++w) acc[w][t] = make_double2(0.0, 0.0);

    for (int j1 = 0; j1 < N1; ++j1) {
      const int poff = j1 * N2 * N3;
      // ---- pass 1 along A, straight from global memory
#pragma unroll 1
      for (int it = 0; it < G::IA; ++it) {
        const int line = it * G::LINES + lane / LA;
        const bool ok = line < NB;
        const int base = poff + G::at(ok ? line : 0, lA);
        double2 yb[MA];
#pragma unroll
        for (int s = 0; s < MA; ++s) yb[s] = gld(ub0, base + G::at(0, LA * s));
#pragma unroll
        for (int w = 0; w < PW; ++w) {
          const double2* ua = w == 0 ? ua0 : ua1;
          double2 x[MA];
          if (w == 1 && !share_b) {
#pragma unroll
            for (int s = 0; s < MA; ++s) yb[s] = gld(ub1, base + G::at(0, LA * s));
          }
#pragma unroll
          for (int s = 0; s < MA; ++s) x[s] = cconjmul(gld(ua, base + G::at(0, LA * s)), yb[s]);
          row_fft<NA, LA, MA>(x, lA, twA);
          double2* T1w = T1 + w * per_pd;
          static_for<0, MA>([&](auto fc) {
            constexpr int f = decltype(fc)::value;
            int aA = bA + f;
            aA -= aA >= NA ? NA : 0;
            if (ok && aA < FA) T1w[aA * SA + line] = x[fft_pos<MA>(f)];
          });
          // keep the two band pairs' loads and transforms from overlapping,
          // which would double the live registers
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      wave_sync();
      // ---- pass 2 along B (PW band pairs side by side); outputs go
      // column-major over the lines already read, so T2 needs no space of its own
      double2* T1s = T1 + sub * per_pd;
      for (int c0 = 0; c0 < FA; c0 += CB) {
        const int col = c0 + ll / LB;
        const bool ok = col < FA;
        double2 x[MB];
#pragma unroll
        for (int s = 0; s < MB; ++s) x[s] = csel(ok, T1s[col * SA + lB + LB * s], make_double2(0.0, 0.0));
        row_fft<NB, LB, MB>(x, lB, twB);
        wave_sync();
        static_for<0, MB>([&](auto fc) {
          constexpr int f = decltype(fc)::value;
          int aB = bB + f;
          aB -= aB >= NB ? NB : 0;
          if (ok && aB < FB) T1s[col * FB + aB] = x[fft_pos<MB>(f)];
        });
        wave_sync();
      }
      // ---- pass 3: direct sum over planes at the sphere points
#pragma unroll
      for (int t = 0; t < TG; ++t) {
        if (lane + 64 * t < ngq) {
          const int2 e = gtab[lane + 64 * t];
          int r = e.y * j1;  // below 2^24: exact in float
          r -= N1 * (int)((float)r * inv_n1);
          r += r < 0 ? N1 : 0;
          r -= r >= N1 ? N1 : 0;
          const double2 w1 = tw1[r];
#pragma unroll
          for (int w = 0; w < PW; ++w) acc[w][t] = cfma(T1[w * per_pd + e.x], w1, acc[w][t]);
        }
      }
      wave_sync();
    }
#pragma unroll
    for (int w = 0; w < PW; ++w) {
      if (w == 1 && !live1) continue;
      double2* o = a.out + (size_t)(job.row0 + p0 + 4 * w) * ngm;
#pragma unroll
      for (int t = 0; t < TG; ++t) {
        const int g = lane + 64 * t;
        if (g < ngq) {
          const double sc = EXCH ? gbl(a.vscale)[g] : 1.0;
          gst(o, g, make_double2(acc[w][t].x * sc, acc[w][t].y * sc));
        } else if (g < ngm) {
          gst(o, g, make_double2(0.0, 0.0));
        }
      }
    }
  }
}

// Planes of at most 32 x 32 points: one lane owns a whole line, so both
// in-plane transforms are register FFTs with compile-time twiddles and no
// exchange between lanes, and each is pruned to the kept window by
// wave-uniform branches.  A wave takes one band pair and two planes at a time
// (lanes 0-31 plane j1, lanes 32-63 plane j1 + 1):
//   pass 1  lane (h, j3): column j3 of plane j1 + h, product and FFT along j2
//           as two half-length FFTs of the even and odd rows, combined only at
//           the kept f2 -> T1_h[f2][j3];
//   pass 2  lane (h, f2): row f2, the same split along j3 -> T2_h[f2][f3],
//           written over the rows already read;
//   pass 3  sphere point g = lane + 64 t accumulates both planes.
// Element i of a wave-uniform array, addressed by a 32-bit byte offset so that
// the load takes the scalar-base + 32-bit vector-offset form.
__device__ __forceinline__ double2 ldg(const double2* base, unsigned i) {
  const auto* b = gbl(reinterpret_cast<const char*>(base));
  const gd2 v = *(const __attribute__((address_space(1))) gd2*)(b + (size_t)(i * 16u));
  return make_double2(v.x, v.y);
}
typedef float gf2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ldg(const float2* base, unsigned i) {
  const auto* b = gbl(reinterpret_cast<const char*>(base));
  const gf2 v = *(const __attribute__((address_space(1))) gf2*)(b + (size_t)(i * 8u));
  return make_float2(v.x, v.y);
}

// Materialise every value of x here: stops the optimiser from sinking the
// last butterflies into the branches that pick the kept window, which would
// keep their inputs live across all of them.
template <class C, int M>
__device__ __forceinline__ void pin(C (&x)[M]) {
#pragma unroll
  for (int i = 0; i < M; ++i) asm volatile("" : "+v"(x[i].x), "+v"(x[i].y));
}

// C: double2, or float2 for FP32 pair densities (wave functions read from the
// FP32 copy, every pass in FP32, the sphere values written as FP64).
// NP planes per step (2 or 4): with 4, pass 1 runs twice per step and pass 2
// takes the kept rows of all four planes at once (4 F2 <= 64 lanes), which
// halves its issued instructions for windows of up to 16 rows.
template <int N2, int N3, int TG, bool EXCH, class C, bool PF, int NP = 2>
__device__ __forceinline__ void pd_line_job(const PdArgs& a, const PdJob& job) {
  static_assert(NP == 2 || (NP == 4 && !PF), "2 planes per step, or 4 without the prefetch");
  static_assert(N2 <= 32 && N3 <= 32 && N2 % 2 == 0 && N3 % 2 == 0, "lines must fit a half wave");
  constexpr bool F32 = sizeof(C) == 8;
  static_assert(!(F32 && EXCH), "exchange pair densities are FP64");
  constexpr int H2 = N2 / 2, H3 = N3 / 2;
  constexpr int S1 = 33;  // T1 row stride: columns N3..31 of idle lanes land in the padding
  // declared as double2 for its 16-byte alignment: the dynamic area follows
  // the static job word of the persistent loop
  extern __shared__ double2 smem_raw[];
  C* smem = reinterpret_cast<C*>(smem_raw);
  const int N1 = a.N1, ngm = a.ng_max;
  const int F2 = a.F2, F3 = a.F3;
  C* tw1 = smem;
  // wave index made uniform so that band pointers live in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5, c = lane & 31;
  const int per_pl = F2 * S1;
  C* T1 = tw1 + N1 + wave * NP * per_pl;
  int2* gtab = reinterpret_cast<int2*>(tw1 + N1 + 4 * NP * per_pl);

  for (int t = threadIdx.x; t < N1; t += blockDim.x) {
    double s, cs;
    sincospi(2.0 * t / N1, &s, &cs);
    tw1[t] = mkc<C>(cs, -s);
  }
  const int nA = job.nab & 255, nB = (job.nab >> 8) & 255;
  int m01, m02, m03;
  unpack_m(job.m0p, m01, m02, m03);
  const int ngq = gbl(a.ng)[job.iq];
  const auto* gq = gbl(a.gpack + (size_t)job.iq * ngm);
  // sphere point g: offset of (f2, f3) in the window, f1 mod N1
  for (int g = threadIdx.x; g < ngq; g += blockDim.x) {
    int m1, m2, m3;
    unpack_m(gq[g], m1, m2, m3);
    gtab[g] = make_int2((m2 - m02 - a.lo2) * F3 + (m3 - m03 - a.lo3), imod(m1 - m01, N1));
  }
  // kept frequencies as bit masks: f is kept when (f - lo) mod N < F
  unsigned keep2 = 0, keep3 = 0;
  for (int f = 0; f < N2; ++f) keep2 |= (unsigned)(imod(f - a.lo2, N2) < F2) << f;
  for (int f = 0; f < N3; ++f) keep3 |= (unsigned)(imod(f - a.lo3, N3) < F3) << f;
  __syncthreads();
  const float inv_n1 = 1.0f / (float)N1;

  const int Nr = N1 * N2 * N3;
  const int npd = nA * nB;
  C* T1h = T1 + h * per_pl;
  // pass 2 with four planes: lane l takes kept row l mod F2 of plane l / F2
  const bool ok4 = NP == 4 && lane < 4 * F2;
  const int pl4 = ok4 ? lane / F2 : 0, rw4 = ok4 ? lane - pl4 * F2 : 0;
  // with an even number of bands on both sides the four waves of a step take
  // a 2 x 2 block of band pairs (four distinct grids per step instead of five)
  const bool blk = nA % 2 == 0 && nB % 2 == 0;
  for (int p = wave; p < npd; p += 4) {
    int ia = p / nB, ib = p % nB;
    if (blk) {
      const int i = p >> 2, nb2 = nB >> 1;
      ia = 2 * (i / nb2) + (wave >> 1);
      ib = 2 * (i % nb2) + (wave & 1);
    }
    const C* u;
    if constexpr (F32)
      u = a.u32;
    else
      u = a.u;
    const C* ua = u + ((size_t)job.ka * a.nb + job.a0 + ia) * Nr;
    const C* ub = u + ((size_t)job.kb * a.nb + job.b0 + ib) * Nr;
    C acc[TG];
#pragma unroll
    for (int t = 0; t < TG; ++t) acc[t] = mkc<C>(0.0, 0.0);

    // even rows of a plane pair (lane: column c of plane j1 + h): with PF issued
    // one plane pair ahead, so that their latency hides behind pass 3
    const int col = c < N3 ? c : 0;
    C pa[H2], pb[H2];
    auto load_even = [&](int jj) {
      const unsigned o = (unsigned)(col + (jj + 1 < N1 ? jj + h : jj) * (N2 * N3));
#pragma unroll
      for (int s = 0; s < H2; ++s) {
        pa[s] = ldg(ua, o + 2 * s * N3);
        pb[s] = ldg(ub, o + 2 * s * N3);
      }
    };
    if constexpr (PF) load_even(0);
    for (int j1 = 0; j1 < N1; j1 += NP) {
      // window masks and origins re-read per plane: kept loop-invariant they
      // would pin one scalar condition per frequency across the loop
      unsigned k2 = __builtin_amdgcn_readfirstlane(keep2), k3 = __builtin_amdgcn_readfirstlane(keep3);
      int lo2 = __builtin_amdgcn_readfirstlane(a.lo2), lo3 = __builtin_amdgcn_readfirstlane(a.lo3);
      asm volatile("" : "+s"(k2), "+s"(k3), "+s"(lo2), "+s"(lo3));
      // (f - lo) mod N as f + sh with one wrap, sh = N - (lo mod N) in [1, N]
      const int sh2 = N2 - imod(lo2, N2), sh3 = N3 - imod(lo3, N3);
      // ---- pass 1 (idle lanes load a valid column and write padding or a
      // plane that pass 3 skips), once per two planes
#pragma unroll
      for (int hf = 0; hf < NP / 2; ++hf) {
        const int jj = j1 + 2 * hf;
        if (NP > 2 && jj >= N1) break;  // wave-uniform
        if constexpr (!PF) load_even(jj);
        const bool two = jj + 1 < N1;  // the second plane exists
        C* T1w = T1 + (2 * hf + h) * per_pl;
        const unsigned off = (unsigned)(col + (two ? jj + h : jj) * (N2 * N3));
        C E[H2], O[H2];
#pragma unroll
        for (int s = 0; s < H2; ++s) E[s] = cconjmul(pa[s], pb[s]);
        __builtin_amdgcn_sched_barrier(0);
        // half of the odd rows in flight during the even-row FFT, the other
        // half after it: at most half the odd rows sit in raw registers next
        // to the even-row transform
        constexpr int HO = H2 / 2;
        C ra[H2], rb[H2];
#pragma unroll
        for (int s = 0; s < HO; ++s) {
          ra[s] = ldg(ua, off + (2 * s + 1) * N3);
          rb[s] = ldg(ub, off + (2 * s + 1) * N3);
        }
        __builtin_amdgcn_sched_barrier(0);
        reg_fft<H2, 1, 0>(E);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = HO; s < H2; ++s) {
          ra[s] = ldg(ua, off + (2 * s + 1) * N3);
          rb[s] = ldg(ub, off + (2 * s + 1) * N3);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < H2; ++s) O[s] = cconjmul(ra[s], rb[s]);
        __builtin_amdgcn_sched_barrier(0);
        reg_fft<H2, 1, 0>(O);
        pin(E);
        pin(O);
        static_for<0, N2>([&](auto fc) {
          constexpr int f = decltype(fc)::value;
          if (k2 & (1u << f)) {  // wave-uniform
            int r = f + sh2;
            if constexpr ((N2 & (N2 - 1)) == 0) r &= N2 - 1;
            else r -= r >= N2 ? N2 : 0;
            constexpr int q = fft_pos<H2>(f % H2);
            T1w[r * S1 + c] = cadd(E[q], cmul_root<N2, f>(O[q]));
          }
        });
      }
      wave_sync();
      // ---- pass 2
      {
        const bool ok = NP == 4 ? ok4 : c < F2;
        const int rr = NP == 4 ? rw4 : (ok ? c : 0);
        C* T2 = NP == 4 ? T1 + pl4 * per_pl : T1h;
        const int row = rr * S1;
        C E[H3], O[H3];
#pragma unroll
        for (int s = 0; s < H3; ++s) {
          E[s] = T2[row + 2 * s];
          O[s] = T2[row + 2 * s + 1];
        }
        reg_fft<H3, 1, 0>(E);
        reg_fft<H3, 1, 0>(O);
        pin(E);
        pin(O);
        wave_sync();
        static_for<0, N3>([&](auto fc) {
          constexpr int f = decltype(fc)::value;
          if (k3 & (1u << f)) {  // wave-uniform
            int r = f + sh3;
            if constexpr ((N3 & (N3 - 1)) == 0) r &= N3 - 1;
            else r -= r >= N3 ? N3 : 0;
            constexpr int q = fft_pos<H3>(f % H3);
            const C v = cadd(E[q], cmul_root<N3, f>(O[q]));
            if (ok) T2[rr * F3 + r] = v;
          }
        });
      }
      wave_sync();
      // with PF, the next plane pair in flight during pass 3 (issued whether
      // or not one is left, so that the values just consumed are dead; the
      // last pair re-reads a valid plane)
      if constexpr (PF) load_even(j1 + 2 < N1 ? j1 + 2 : j1);
      __builtin_amdgcn_sched_barrier(0);
      // ---- pass 3
#pragma unroll
      for (int t = 0; t < TG; ++t) {
        if (lane + 64 * t < ngq) {
          const int2 e = gtab[lane + 64 * t];
          int r = e.y * j1;  // below 2^24: exact in float
          r -= N1 * (int)((float)r * inv_n1);
          r += r < 0 ? N1 : 0;
          r -= r >= N1 ? N1 : 0;
          acc[t] = cfma(T1[e.x], tw1[r], acc[t]);
#pragma unroll
          for (int pp = 1; pp < NP; ++pp) {
            if (j1 + pp < N1) {
              r += e.y;
              r -= r >= N1 ? N1 : 0;
              acc[t] = cfma(T1[pp * per_pl + e.x], tw1[r], acc[t]);
            }
          }
        }
      }
      wave_sync();
    }
    double2* o = a.out + (size_t)(job.row0 + ia * nB + ib) * ngm;
#pragma unroll
    for (int t = 0; t < TG; ++t) {
      const int g = lane + 64 * t;
      if (g < ngq) {
        const double sc = EXCH ? gbl(a.vscale)[g] : 1.0;
        gst(o, g, make_double2((double)acc[t].x * sc, (double)acc[t].y * sc));
      } else if (g < ngm) {
        gst(o, g, make_double2(0.0, 0.0));
      }
    }
  }
}

// Job order of the pair-density kernels; returns the next job of this
// workgroup, or -1 (uniform).  Static: workgroup b runs job b once.
// Persistent: thread 0 draws from the queue of this workgroup's XCD (b mod 8)
// and then from the other seven in turn, so every workgroup leaves once all
// queues are drained (each draw advances a counter that only grows).
template <bool PERSIST>
__device__ __forceinline__ int next_job(const PdBatch& b, int& round, int& tries, int* s_job) {
  if constexpr (!PERSIST) return (round++ == 0 && (int)blockIdx.x < b.njobs) ? (int)blockIdx.x : -1;
  const int per_q = b.njobs >> 3;
  const int home = blockIdx.x & 7;
  if (threadIdx.x == 0) {
    int got = -1;
    while (tries < 8) {
      const int x = (home + tries) & 7;
      const int t = (int)atomicAdd(&b.cnt[x * kQueueStride], 1u);
      if (t < per_q) {
        got = 8 * t + x;
        break;
      }
      ++tries;
    }
    *s_job = got;
  }
  __syncthreads();
  const int j = __builtin_amdgcn_readfirstlane(*s_job);
  __syncthreads();
  return j;
}

template <int N2, int N3, int TG, bool EXCH, bool PERSIST>
__global__ __launch_bounds__(256, 2) void k_pair_density(PdBatch b) {
  __shared__ int s_job;
  int round = 0, tries = 0;
  for (int j = next_job<PERSIST>(b, round, tries, &s_job); j >= 0; j = next_job<PERSIST>(b, round, tries, &s_job)) {
    const PdJob job = b.jobs[j];
    const PdArgs a = b.sys[job.nab >> 16];
    pd_general_job<N2, N3, TG, EXCH>(a, job);
    __syncthreads();  // LDS of this job is free before the next one fills it
  }
}

template <int N2, int N3, int TG, bool EXCH, bool PERSIST>
__global__ __launch_bounds__(256, 2) void k_pair_density_line(PdBatch b) {
  __shared__ int s_job;
  int round = 0, tries = 0;
  for (int j = next_job<PERSIST>(b, round, tries, &s_job); j >= 0; j = next_job<PERSIST>(b, round, tries, &s_job)) {
    const PdJob job = b.jobs[j];
    const PdArgs a = b.sys[job.nab >> 16];
    pd_line_job<N2, N3, TG, EXCH, double2, true>(a, job);
    __syncthreads();
  }
}

// FP32 variant (valence-valence and conduction-conduction densities of the
// mixed-precision modes): half the registers, so no next-plane prefetch (the
// occupancy hides the load latency instead).  Two planes per step: four
// workgroups per CU under static dispatch, three with the persistent loop,
// which needs more registers.  Four planes per step: three (LDS).
template <int N2, int N3, int TG, bool PERSIST, int NP>
__global__ __launch_bounds__(256, (PERSIST || NP == 4) ? 3 : 4) void k_pair_density_line_f32(PdBatch b) {
  __shared__ int s_job;
  int round = 0, tries = 0;
  for (int j = next_job<PERSIST>(b, round, tries, &s_job); j >= 0; j = next_job<PERSIST>(b, round, tries, &s_job)) {
    const PdJob job = b.jobs[j];
    const PdArgs a = b.sys[job.nab >> 16];
    pd_line_job<N2, N3, TG, false, float2, false, NP>(a, job);
    __syncthreads();
  }
}

template <int N2, int N3>
constexpr bool use_line() {
  return N2 <= 32 && N3 <= 32 && N2 % 2 == 0 && N3 % 2 == 0;
}

static int tg_bucket(int ng_max) {
  const int t = (ng_max + 63) / 64;
  return t <= 4 ? 4 : t <= 5 ? 5 : t <= 8 ? 8 : t <= 13 ? 13 : 16;
}

template <int N2, int N3>
static size_t lds_bytes(int N1, int F2, int F3, int ng_max, int f32_planes) {
  if constexpr (use_line<N2, N3>()) {
    const size_t np = f32_planes == 4 ? 4 : 2;
    return (f32_planes ? sizeof(float2) : sizeof(double2)) * ((size_t)N1 + 4 * np * (size_t)F2 * 33) +
           sizeof(int2) * (size_t)ng_max;
  }
  using G = PlaneGeo<N2, N3>;
  const int FA = G::AX == 2 ? F2 : F3;
  return sizeof(double2) * ((size_t)N1 + N2 + N3 + 4 * (size_t)G::PW * FA * G::SA) + sizeof(int2) * (size_t)ng_max;
}

template <int N2, int N3, int TG>
static hipError_t launch_tg(const PdBatch& b, size_t lds, int grid, bool exch, int f32_planes, hipStream_t st) {
  void (*k)(PdBatch);
  if constexpr (use_line<N2, N3>()) {
    if (f32_planes == 4 && !exch && !b.persist)  // (the persistent loop spills with four planes)
      k = k_pair_density_line_f32<N2, N3, TG, false, 4>;
    else if (f32_planes && !exch)
      k = b.persist ? k_pair_density_line_f32<N2, N3, TG, true, 2> : k_pair_density_line_f32<N2, N3, TG, false, 2>;
    else if (b.persist)
      k = exch ? k_pair_density_line<N2, N3, TG, true, true> : k_pair_density_line<N2, N3, TG, false, true>;
    else
      k = exch ? k_pair_density_line<N2, N3, TG, true, false> : k_pair_density_line<N2, N3, TG, false, false>;
  } else {
    if (b.persist)
      k = exch ? k_pair_density<N2, N3, TG, true, true> : k_pair_density<N2, N3, TG, false, true>;
    else
      k = exch ? k_pair_density<N2, N3, TG, true, false> : k_pair_density<N2, N3, TG, false, false>;
  }
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid), dim3(256), lds, st, b);
  return hipGetLastError();
}

template <int N2, int N3>
static hipError_t launch_grid(const PdBatch& b, int ng_max, size_t lds, int grid, bool exch, int f32_planes,
                              hipStream_t st) {
  switch (tg_bucket(ng_max)) {
    case 4: return launch_tg<N2, N3, 4>(b, lds, grid, exch, f32_planes, st);
    case 5: return launch_tg<N2, N3, 5>(b, lds, grid, exch, f32_planes, st);
    case 8: return launch_tg<N2, N3, 8>(b, lds, grid, exch, f32_planes, st);
    case 13: return launch_tg<N2, N3, 13>(b, lds, grid, exch, f32_planes, st);
    default: return launch_tg<N2, N3, 16>(b, lds, grid, exch, f32_planes, st);
  }
}

bool pd_grid_supported(int N2, int N3) {
  return (N2 == N3 && (N2 == 8 || N2 == 12 || N2 == 16 || N2 == 24 || N2 == 32 || N2 == 48 || N2 == 64 ||
                       N2 == 96)) ||
         (N2 == 24 && N3 == 96) || (N2 == 12 && N3 == 16) || (N2 == 16 && N3 == 24);
}

bool pd_line_grid(int N2, int N3) {
  return pd_grid_supported(N2, N3) && N2 <= 32 && N3 <= 32 && N2 % 2 == 0 && N3 % 2 == 0;
}

// One workgroup per (grid, j1) plane: the N2 x N3 plane through LDS, written
// as rows j2 of the slabs j3.
__global__ __launch_bounds__(256) void k_rotate_axes(const double2* __restrict__ u, double2* __restrict__ ut, int N1,
                                                     int N2, int N3) {
  extern __shared__ double2 tile[];  // [N2][N3 + 1]
  const long long gj = blockIdx.x;
  const long long g = gj / N1;
  const int j1 = (int)(gj % N1);
  const int n = N2 * N3, S = N3 + 1;
  const double2* src = u + (size_t)(g * N1 + j1) * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) tile[(i / N3) * S + i % N3] = src[i];
  __syncthreads();
  double2* dst = ut + (size_t)g * N1 * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int j3 = i / N2, j2 = i % N2;
    dst[((size_t)j3 * N1 + j1) * N2 + j2] = tile[j2 * S + j3];
  }
}

hipError_t launch_rotate_axes(const double2* u, double2* ut, long long ngrids, int N1, int N2, int N3,
                              hipStream_t st) {
  const size_t lds = sizeof(double2) * (size_t)N2 * (N3 + 1);
  if (ngrids <= 0) return hipSuccess;
  if (lds > 160 * 1024 || ngrids * N1 > 0x7fffffffLL) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void*)k_rotate_axes, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rotate_axes, dim3((unsigned)(ngrids * N1)), dim3(256), lds, st, u, ut, N1, N2, N3);
  return hipGetLastError();
}

// FP32 copy of the wave functions for the FP32 pair densities (round to nearest).
__global__ __launch_bounds__(256) void k_to_f32(const double2* __restrict__ u, float2* __restrict__ v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 x = u[i];
    v[i] = make_float2((float)x.x, (float)x.y);
  }
}

hipError_t launch_to_f32(const double2* u, float2* v, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f32, dim3(4096), dim3(256), 0, st, u, v, n);
  return hipGetLastError();
}

size_t pd_lds_bytes(int N1, int N2, int N3, int F2, int F3, int ng_max, int f32_planes) {
#define BSE_PD_LDS(X, Y) \
  if (N2 == X && N3 == Y) return lds_bytes<X, Y>(N1, F2, F3, ng_max, f32_planes);
  BSE_PD_LDS(8, 8)
  BSE_PD_LDS(12, 12)
  BSE_PD_LDS(16, 16)
  BSE_PD_LDS(24, 24)
  BSE_PD_LDS(32, 32)
  BSE_PD_LDS(48, 48)
  BSE_PD_LDS(64, 64)
  BSE_PD_LDS(96, 96)
  BSE_PD_LDS(24, 96)
  BSE_PD_LDS(12, 16)
  BSE_PD_LDS(16, 24)
#undef BSE_PD_LDS
  return ~size_t(0);
}

// exch: the launch computes exchange rows (every system's PdArgs.vscale set).
hipError_t launch_pair_density(const PdBatch& b, int N2, int N3, int ng_max, size_t lds, int grid, bool exch,
                               int f32_planes, hipStream_t st) {
  if (b.njobs <= 0 || grid <= 0) return hipSuccess;
#define BSE_PD_CASE(X, Y) \
  if (N2 == X && N3 == Y) return launch_grid<X, Y>(b, ng_max, lds, grid, exch, f32_planes, st);
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
