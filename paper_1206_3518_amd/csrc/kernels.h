// Launch interfaces of the HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

namespace bse {

// One pair-density job: band block [a0, a0+nA) at k = ka (conjugated operand)
// times [b0, b0+nB) at k' = kb, shift m0 (packed), sphere iq, of system
// nab >> 16 of a batch (nab = nA | nB << 8 | sys << 16).  Output row of band
// pair (ia, ib) is row0 + ia*nB + ib.  nA = nB = 0 marks an empty job.
struct PdJob {
  int ka, kb, m0p, iq, a0, b0, nab, row0;
};

struct PdArgs {
  const double2* u;
  int nb;
  int N1;
  const int* gpack;     // [Nk][ng_max] packed Miller indices
  const int* ng;        // [Nk]
  int ng_max;
  int lo2, lo3;         // lowest kept frequency (m - m0) along axes 2, 3
  int F2, F3;           // kept window widths
  const double* vscale; // [ng_max] output scale (sqrt v) or null
  double2* out;         // rows of ng_max
  const float2* u32;    // FP32 copy of u (FP32 pair densities) or null
};

// Jobs of one pair-density launch over a batch of systems that share N2, N3.
// Static dispatch: workgroup b runs jobs[b].  Persistent dispatch: a grid of
// at most `grid` workgroups; workgroup b serves queue b mod 8 (the XCD it runs
// on), whose t-th job is jobs[8 t + queue], by an atomic counter per queue,
// then takes jobs from the other queues until all are drained.  njobs is a
// multiple of 8 in both modes.
// Queue counters of persistent dispatch sit kQueueStride unsigned apart, each
// on a 256-byte line of its own, so that the queues of different XCDs share
// no cache line.
constexpr int kQueueStride = 64;

struct PdBatch {
  const PdArgs* sys;    // [nsys] per-system arguments (device)
  const PdJob* jobs;    // [njobs]
  int njobs;
  int persist;
  unsigned* cnt;        // queue x at cnt[x * kQueueStride], x < 8, zero at launch (persistent only)
};

bool pd_grid_supported(int N2, int N3);
// planes N2 x N3 that the one-lane-per-line kernel takes (both even, <= 32)
bool pd_line_grid(int N2, int N3);
// ut[g][j3][j1][j2] = u[g][j1][j2][j3] for ngrids grids of N1 x N2 x N3 (N1, N2 <= 32)
hipError_t launch_rotate_axes(const double2* u, double2* ut, long long ngrids, int N1, int N2, int N3, hipStream_t st);
// f32_planes: 0 for FP64, else the planes per step of the FP32 kernel (2 or 4)
size_t pd_lds_bytes(int N1, int N2, int N3, int F2, int F3, int ng_max, int f32_planes);
// v = (float) u, n complex values
hipError_t launch_to_f32(const double2* u, float2* v, size_t n, hipStream_t st);
// ng_max: the largest of the batch; lds: the largest pd_lds_bytes of the
// batch; exch: exchange rows (every system's vscale set); grid: njobs for
// static dispatch, the persistent grid otherwise; f32_planes: 0, or FP32
// transforms from PdArgs.u32 with 2 or 4 planes per step (one-lane-per-line
// planes and non-exchange rows only; 4 needs every F2 <= 16).
hipError_t launch_pair_density(const PdBatch& b, int N2, int N3, int ng_max, size_t lds, int grid, bool exch,
                               int f32_planes, hipStream_t st);
hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t st);

// A GEMM tile of the direct term's first stage: q group iq, tile (mt, nt), system sys.
struct S1Tile {
  int iq, mt, nt, sys;
};
// An exchange tile (64 x 64 block (i, j) of H) or a mirror tile (32 x 32
// destination block (i, j), i >= j) of system sys.
struct HTile {
  int i, j, sys, pad;
};

// The per-pair arrays (RV, RC, Z, RVs) hold one chunk of k pairs at a time:
// row r of pair p of the chunk is row (p - p0) * nv^2 + r (nc^2 for RC).
struct GemmArgs {
  // exchange:   H[S][S'] = cpref2 * sum_g conj(X[S][g]) X[S'][g], upper tiles
  // stage 1:    Z[r][n]  = sum_g conj(RV[r][g]) W[q][g][n], rows r of q group
  // stage 2:    D[vv'][cc'] = sum_g Z[p][vv'][g] RC[p][cc'][g];  H block -= c * D (+ diag)
  const double2* X;
  int ns;
  int ng_max;
  int ngx;              // K of the exchange (= ng(Q), the sphere of the exciton momentum)
  const int* kq;        // [Nk] mesh index of k + Q (null: Q = 0), for the transition energies
  double2* H;
  double cpref;         // E_h / (Nk Omega_cell)
  const double2* RV;
  const double2* RC;
  double2* Z;
  const double2* W;     // W(q) for every q, or (wmap) the matrices of the irreducible q points
  const int* wsrc;      // null, or [Nk][2] (source matrix, conjugate) of W(q)
  const int* wmap;      // null, or [Nk][ng_max]: W_GG'(q) = W[wsrc[q][0]][wmap[q][G]][wmap[q][G']]
  const double2* W0;    // W(q = 0) (its G = 0 entry is the head)
  const int* ng;
  const int* qstart;    // [Nk+1] first pair of each q group of the chunk (global pair index;
                        // the chunk's pairs are sorted by q), qstart[Nk] = end of the chunk
  const int4* pairs;    // (ka, kb, iq, m0p), every pair of the system
  int p0;               // first pair of the chunk
  const double* eps;
  int nv, nc, nb, npairs;
  int nt;               // nv * nc: rows of one k block
  int w_head_fp64;      // mixed precision: q=0 head added separately in FP64
  const void* Ws;       // mixed precision: W split and transposed, [Nk][ng_max][4][kpad] of the
                        // split type (planes re hi, re lo, im hi, im lo), head left out
  int kpad;             // ng_max rounded up to a multiple of 32
  const void* RVs;      // mixed precision: conj(RV) split, [rows][4][kpad] of the split type
  int ldh;              // row stride of H (ns, or 2 ns inside the beyond-TDA matrix)
  int rv_rows, rc_rows; // rows per pair of RV and Z, and of RC (nv^2, nc^2; coupling: nv nc both)
  int coupling;         // coupling block: RV rows (v, c') = n_{vk,c'k'}, RC rows (c, v') = n_{ck,v'k'},
                        // output H[(k v c)][(k' v' c')], no transition energies
  const double2* Xb;    // exchange B operand (coupling: conj(X) at -G); null: X
  int mirror_plain;     // mirror lower blocks as the transpose (symmetric coupling block), not its conjugate
};

// The contractions run over a batch: gs is a device array of per-system
// arguments, every tile names its system.  Stage 2 items are (pair, 16 x 16
// tile) of every system, numbered system after system: d2off[s] is the first
// item of system s (nsys + 1 entries).
// out[g] = sqrt(vx[g]) for g < ngx, zero at g = g0 (G = 0; -1: none) and past ngx
hipError_t launch_vscale(const double* vx, int ngx, int ng_max, int g0, double* out, hipStream_t st);
hipError_t launch_exchange(const GemmArgs* gs, const HTile* tiles, int ntiles, int precision, hipStream_t st);
// mapped: some system reads W through its sphere maps (FP64; the mixed modes
// unfold W while they split it).  rows: 64 or 128 rows per tile, as the tile
// list was made (tile mt covers rows [rows mt, rows (mt + 1))).
hipError_t launch_direct_s1(const GemmArgs* gs, const S1Tile* tiles, int ntiles, int precision, int mapped,
                            int rows, hipStream_t st);
// stage 2 is FP64 in every mode (it adds the FP64 q = 0 head when w_head_fp64)
hipError_t launch_direct_s2(const GemmArgs* gs, const int* d2off, int nsys, int nitems, hipStream_t st);
hipError_t launch_mirror(const GemmArgs* gs, const HTile* tiles, int ntiles, hipStream_t st);
// Xb[S][g] = conj(X[S][inv[g]]) for g < ng0 (inv: position of -G in the q = 0
// sphere), zero past it; ns rows of stride ng_max
hipError_t launch_xbar(const double2* X, const int* inv, int ns, int ng0, int ng_max, double2* Xb, hipStream_t st);
// lower half of the beyond-TDA matrix H2 [2ns][2ns] from its upper half:
// H2[ns+i][ns+j] = -conj(H2[i][j]), H2[ns+i][j] = -conj(H2[j][ns+i])
hipError_t launch_full_lower(double2* H2, int ns, hipStream_t st);
// Ws[q][n][pl][k] = part pl of W[q][k][n] for k, n < ng(q), zero elsewhere up
// to kpad (and at the q = 0 head when head != 0); precision BSE_SPLIT_FP32 or
// BSE_BF16X3 (parts as in the mixed contractions).  With wmap, W[q][k][n] is
// W[wsrc[q][0]][wmap[q][k]][wmap[q][n]], conjugated when wsrc[q][1] != 0.
// RVs[row][pl][k] = part pl of conj(RV[row][k]) for k < ng(q of the row's
// pair), zero up to kpad; rows_per_pair = nv^2.
hipError_t launch_split_rv(const double2* RV, const int4* pairs, const int* ng, size_t nrows, int rows_per_pair,
                           int ld, int kpad, int precision, void* RVs, hipStream_t st);
hipError_t launch_split_w(const double2* W, const int* ng, const int* wsrc, const int* wmap, int nk, int ng_max,
                          int kpad, int head, int precision, void* Ws, hipStream_t st);
// mixed-precision bodies (precision BSE_SPLIT_FP32 or BSE_BF16X3), called by the above
hipError_t launch_exchange_mx(const GemmArgs* gs, const HTile* tiles, int ntiles, int precision, hipStream_t st);
hipError_t launch_direct_s1_mx(const GemmArgs* gs, const S1Tile* tiles, int ntiles, int precision, int rows,
                               hipStream_t st);
// system of stage-2 item `item`: the last s with d2off[s] <= item
__device__ __forceinline__ int item_system(const int* __restrict__ d2off, int nsys, int item) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d2off[mid] <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Adjoint of the build.
struct AdjArgs {
  const double2* dH;   // [NS][NS] dL/dH
  const double2* RV;   // recomputed pair densities (layout of the forward build)
  const double2* RC;
  double2* T;          // [npairs][nv^2][ng_max] scratch
  double2* dWout;      // dW GEMM output (dW itself, or the raw gradient before projection)
  double2* dWfinal;    // projected dW
  double* deps;        // [Nk][nb]
  const int4* pairs;   // every pair of the system
  const int* ng;
  const int* qstart;   // [Nk+1] q groups of the chunk (as in GemmArgs)
  int p0;              // first pair of the chunk; RV, RC, T, Z hold the chunk's rows
  const int4* dwtiles; // (q, row tile, column tile, -)
  const int* qbar;     // [Nk] time-reversal partner of q
  const int* trmap;    // [Nk][ng_max] index of t - m_g in the sphere of qbar
  int nk, nv, nc, ns, ng_max, npairs;
  double cpref;
  int qe[3], kn[3];    // exciton momentum Q and the k mesh (grid-axis triplets of the k index)
  // gradients with respect to the pair densities (nullable outputs)
  const double2* Z;    // forward stage-1 product conj(rho_vv')^T W, rows like RV
  const double2* W;    // [Nk][ng_max][ng_max]
  const double2* Xs;   // exchange densities scaled by sqrt v, [NS][ng_max]
  const double* vs;    // sqrt v on S(0), zero at G = 0
  const int* plex;     // [npairs] lexicographic position of each pair (k <= k')
  const int4* rvtiles; // (q, row tile, column tile, -) over every column of ng_max
  int ngx;             // ng(q = 0)
  double2* dX;         // [NS][ng_max]
  double2* drv;        // [npairs][nv][nv][ng_max], lexicographic pairs
  double2* drc;        // [npairs][nc][nc][ng_max]
};
// Reciprocal vectors (rows b_d, bohr^-1) for the gradient matrix elements.
struct GradCell {
  double b[3][3];
};
// BSE_VALIDATE scans: bad[0..2] get 1 on a non-finite value in u, eps, vx;
// wstat[0..2] (zero on entry) the bit patterns of max |W|, max Hermiticity
// deviation and max time-reversal deviation (abs(re) + abs(im) each).
hipError_t launch_validate(const double* u, size_t nu, const double* eps, size_t ne, const double* vx, size_t nvx,
                           const double2* W, const int* ng, const int* qbar, const int* trmap, int nk, int ng_max,
                           int check_tr, unsigned* bad, unsigned long long* wstat, hipStream_t st);
// Time reversal (BSE_TIME_REVERSAL): ktr[k] = kbar | K0 << 24 | K1 << 25 |
// K2 << 26 with -k = kbar - K (grid axes).  Over the points with kbar != k,
// wstat[3] gets max |u|, wstat[4] max |u_{kbar}(r_j) - exp(-i K.r_j)
// conj(u_k(r_j))| (abs(re) + abs(im)); u in grid order [k][band][j1][j2][j3].
hipError_t launch_validate_u_tr(const double2* u, const int* ktr, int nk, int nb, int N1, int N2, int N3,
                                unsigned long long* wstat, hipStream_t st);

// Pair densities of the time-reversal images of computed k pairs.  Item
// (dst, src, q_dst << 1 | mode, sys), dst and src pairs of the current chunk
// (rows local to it): mode 0, rho_dst[ab][g] = conj(rho_src[ab][trmap[q_dst][g]]);
// mode 1, rho_dst[a nB + b][g] = rho_src[b nB + a][g].  kind 1 fills the
// valence pair densities, kind 2 the conduction ones.
struct TrArgs {
  double2* rv;
  double2* rc;
  const int* ng;
  const int* trmap;
  int ng_max, nv, nc;
};
hipError_t launch_tr_fill(const TrArgs* as, const int4* items, int nitems, int kind, hipStream_t st);
bool fft_len_supported(int N);
hipError_t launch_grad(const double2* u, double2* scratch, int nk, int nb, int nv, int nc, int N1, int N2, int N3,
                       const GradCell& bc, double2* out, hipStream_t st);
// Polarisations of the transition dipoles (Cartesian unit vectors, at most 8).
constexpr int kMaxQhat = 8;
struct Qhats {
  double v[kMaxQhat][3];
};
// d[q][S] = qhat_q . D[S] / ((e_ck - e_vk) / E_h) from D = <u_vk|grad|u_ck> [NS][3]
hipError_t launch_dipole_project(const double2* D, const double* eps, const Qhats& qh, int nq, int nk, int nv,
                                 int nc, double2* d, hipStream_t st);
// eps2 on nw points of [w0, w1] (eV) from nlam excitons and nq polarisation
// rows of d ([nq][ns]); nk_omega = Nk * Omega_cell; t2 scratch of nlam doubles
hipError_t launch_spectrum(int ns, int nlam, int nq, const double* E, const double2* A, const double2* d,
                           double nk_omega, int nw, double w0, double w1, double eta, double* t2, double* eps2,
                           hipStream_t st);

// Static RPA screening (bse_screening).  Y: pair densities of a chunk of q,
// rows ((q_local * nk + k) * 2 + type) * nv * nc + band pair, scaled in place;
// M: [Nk][ng_max][ng_max], eps(q) then W(q); pk: (k, k + q, q, -) per
// (q_local, k); omega = Nk * Omega_cell.
struct RpaArgs {
  double2* Y;
  double2* M;           // [nslot][ng_max][ng_max]: slot i holds q = qof[i]
  const int4* pk;
  const int* ng;
  const int* qof;       // [nslot] q of each output slot
  int nsplit;           // slices of the row sum per HERK tile (1: accumulate into M)
  double2* part;        // nsplit > 1: partial sums [nsplit][part_q][ng_max][ng_max]
  int part_q;           // q_local stride of part
  const double* eps;
  const double* vq;
  int nv, nc, nk, ng_max;
  double omega;
};
hipError_t launch_rpa_scale(const RpaArgs& a, int npairs, hipStream_t st);
hipError_t launch_rpa_init(double2* M, const int* ng, const int* qof, int nslot, int ng_max, hipStream_t st);
// items (destination row base, source row base, q, -): rows (c, v) of the
// destination = conj of rows (v, c) of the source at the sphere map t - G of q
hipError_t launch_rpa_fill(double2* Y, const int4* items, int nitems, const int* trmap, const int* ng, int nv, int nc,
                          int ng_max, hipStream_t st);
// tiles (slot, row tile | slice << 8, column tile, q_local) of 64 x 64 over ng_max x ng_max
hipError_t launch_rpa_herk(const RpaArgs& a, const int4* tiles, int ntiles, hipStream_t st);
// with a.nsplit > 1: eps of the chunk's q (cslot: slot of each q_local) += the partial sums
hipError_t launch_rpa_reduce(const RpaArgs& a, const int* cslot, int nql, hipStream_t st);
// the 64 x 64 tiles below the diagonal of each eps(q) from those above (conjugate transpose)
hipError_t launch_rpa_mirror(double2* M, const int* ng, const int* qof, int nslot, int ng_max, hipStream_t st);
hipError_t launch_rpa_invert(double2* M, const int* ng, const int* qof, int nslot, int ng_max, hipStream_t st);
hipError_t launch_rpa_w(double2* M, const int* ng, const int* qof, const double* vq, int nslot, int ng_max,
                        double head, hipStream_t st);
// Haydock recursion: niter steps of the Lanczos recurrence from conj(d_p)
// for nq <= kMaxQhat polarisations (H [ns][ns] eV, d [nq][ns] Hartree units),
// coefficients into coef [nq][niter][2] (a_j, b_j in eV), then eps2 on nw
// points of [w0, w1] (eV) with half width eta (eV).  V0, V1, Y: nq * ns
// complex each; norm2: nq doubles.
hipError_t launch_haydock(int ns, const double2* H, const double2* d, int nq, int niter, double nk_omega, int nw,
                          double w0, double w1, double eta, double* eps2, double* coef, double2* V0, double2* V1,
                          double2* Y, double* norm2, hipStream_t st);
// T (over Z) and the dW contraction of one chunk, added into dWout (zeroed
// before the first chunk by launch_zero_f64); has_q0: the chunk holds pairs
// of q = 0 (whose FP64 head entry the mixed precisions add separately)
hipError_t launch_adjoint(const AdjArgs& a, int precision, int ndw_tiles, bool has_q0, hipStream_t st);
// after the last chunk: the projection of dW (if asked) and dL/de
hipError_t launch_adjoint_finish(const AdjArgs& a, bool project, hipStream_t st);
hipError_t launch_zero_f64(double* p, size_t n, hipStream_t st);
// W at the irreducible q points: the unfolded W(q) at every q, and the adjoint
// of that unfolding (dW of the nirr matrices from dW at every q)
hipError_t launch_unfold_w(const double2* W, const int* wsrc, const int* wmap, const int* ng, int nk, int ng_max,
                           double2* Wf, hipStream_t st);
hipError_t launch_fold_dw(const double2* dWf, const int* csr, const int* qlist, const int* wsrc, const int* winv,
                          const int* ngirr, int nirr, int ng_max, double2* dW, hipStream_t st);
// dL/drho_cc' from Z (run before launch_adjoint overwrites Z with T)
hipError_t launch_adj_drc(const AdjArgs& a, hipStream_t st);
// dL/drho_vv' from T (after launch_adjoint)
hipError_t launch_adj_drv(const AdjArgs& a, int ntiles, hipStream_t st);
// dL/dn_{vk,ck} from the scaled exchange densities
hipError_t launch_adj_dx(const AdjArgs& a, hipStream_t st);

}  // namespace bse
