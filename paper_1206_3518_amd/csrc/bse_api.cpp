// C ABI of the BSE Hamiltonian builder: argument checks, the host planner
// (k-pair folding, G-sphere tables, FFT windows, GEMM tile lists), workspace
// layout and the kernel sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bse.h"
#include "bse_internal.h"
#include "kernels.h"

using namespace bse;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(BSE_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ------------------------------------------------------------ table uploads
// Plan tables go to the device by asynchronous copies from a pinned staging
// buffer (one per thread, grown as needed, kept for the life of the process),
// so the stream does not stall behind a pageable copy.  Before the buffer is
// rewritten, the copies of the previous call are waited for.
struct Staging {
  char* buf = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};
thread_local Staging g_staging;

// Returns a host buffer of n bytes that no pending copy reads.
int staging_acquire(size_t n, char** out) {
  Staging& S = g_staging;
  if (S.pending) {
    HIP_TRY(hipEventSynchronize(S.done));
    S.pending = false;
  }
  if (!S.done) HIP_TRY(hipEventCreateWithFlags(&S.done, hipEventDisableTiming));
  if (n > S.cap) {
    if (S.buf) HIP_TRY(hipHostFree(S.buf));
    S.buf = nullptr;
    S.cap = 0;
    const size_t want = std::max(n, size_t(1) << 20);
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&S.buf), want, hipHostMallocDefault));
    S.cap = want;
  }
  *out = S.buf;
  return BSE_OK;
}

// Marks the staging buffer as read by the copies just enqueued on st.
int staging_release(hipStream_t st) {
  HIP_TRY(hipEventRecord(g_staging.done, st));
  g_staging.pending = true;
  return BSE_OK;
}

// ------------------------------------------------------------ stage timing
struct ProfRec {
  int stage;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
double g_prof_ms[BSE_NSTAGES] = {0};
long long g_prof_n[BSE_NSTAGES] = {0};

// Runs one launch; with timing on, brackets it with events on the stream.
template <class F>
hipError_t stage(int id, hipStream_t st, F&& launch) {
  bool on;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    on = g_prof_on;
  }
  if (!on) return launch();
  ProfRec r{id, nullptr, nullptr};
  hipError_t e = hipEventCreate(&r.a);
  if (e == hipSuccess) e = hipEventCreate(&r.b);
  if (e == hipSuccess) e = hipEventRecord(r.a, st);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(r.b, st);
  if (e != hipSuccess) {
    if (r.a) (void)hipEventDestroy(r.a);
    if (r.b) (void)hipEventDestroy(r.b);
    return e;
  }
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_pending.push_back(r);
  return hipSuccess;
}

// k' - k = q + G0: q on the k-shaped mesh (componentwise in [0, n)), G0 = m0 . b
// with m0 in {-1, 0} (Sec. III.A: the q mesh has the form of the k mesh).
void fold(const int* n, int ka, int kb, int& iq, int m0[3]) {
  int ta[3] = {ka / (n[1] * n[2]), (ka / n[2]) % n[1], ka % n[2]};
  int tb[3] = {kb / (n[1] * n[2]), (kb / n[2]) % n[1], kb % n[2]};
  int r[3];
  for (int d = 0; d < 3; ++d) {
    const int dd = tb[d] - ta[d];
    r[d] = imod(dd, n[d]);
    m0[d] = (dd - r[d]) / n[d];
  }
  iq = (r[0] * n[1] + r[1]) * n[2] + r[2];
}

// Dispatch order of pair-density jobs.  Workgroup i runs on XCD i mod 8 and
// each XCD keeps about 64 workgroups resident, so the job list is cut into 8
// contiguous chunks (one per XCD) of jobs sorted by system and then by
// ktile x ktile tiles of (k, k'): the resident jobs of an XCD then read the
// wave functions of few k points, which its L2 holds plane by plane.  Chunk x
// is stored at positions 8 t + x (static dispatch hands workgroup 8 t + x to
// XCD x; persistent dispatch uses chunk x as the XCD's queue).  Holes become
// empty jobs.  Tuning choices (order): 0 as above; 1 interleaved, the sorted
// jobs in order, so that the eight XCDs work through the same tiles at once;
// 2 kind-major, the valence-pair jobs of a system before its conduction-pair
// jobs, so that the resident jobs of an XCD read the grids of one band set.
constexpr int kXcds = 8;
// queue counters of the three pair-density kinds, then the validation flags
constexpr size_t kCntBytes = 3 * kXcds * kQueueStride * sizeof(unsigned);

std::vector<PdJob> dispatch_order(std::vector<PdJob> jobs, int ktile, int order = 0) {
  std::stable_sort(jobs.begin(), jobs.end(), [ktile, order](const PdJob& x, const PdJob& y) {
    const int sx = x.nab >> 16, sy = y.nab >> 16;
    if (sx != sy) return sx < sy;
    if (order == 2 && (x.a0 != 0) != (y.a0 != 0)) return x.a0 == 0;  // valence-pair jobs first
    const int tx = x.ka / ktile, ty = y.ka / ktile, ux = x.kb / ktile, uy = y.kb / ktile;
    if (tx != ty) return tx < ty;
    if (ux != uy) return ux < uy;
    if (x.ka != y.ka) return x.ka < y.ka;
    return x.kb < y.kb;
  });
  const size_t n = jobs.size(), c = (n + kXcds - 1) / kXcds;
  if (order == 1) {
    jobs.resize(c * kXcds, PdJob{0, 0, pack_m(0, 0, 0), 0, 0, 0, 0, 0});
    return jobs;
  }
  std::vector<PdJob> out(c * kXcds, PdJob{0, 0, pack_m(0, 0, 0), 0, 0, 0, 0, 0});
  for (size_t x = 0; x < (size_t)kXcds; ++x)
    for (size_t t = 0; t < c && x * c + t < n; ++t) out[t * kXcds + x] = jobs[x * c + t];
  return out;
}

// Workgroup b of a launch runs on XCD b mod 8, so tiles next to each other in
// a list land in eight different L2 caches.  This reorders a tile list so that
// XCD x takes the x-th contiguous segment of it, in order: the column tiles of
// one row block, which read the same rows of the left operand, and the row
// blocks of one q, which read the same W(q), then meet in one L2.  A
// permutation, without holes.
template <class T>
std::vector<T> xcd_segments(const std::vector<T>& in) {
  const size_t n = in.size(), base = n / kXcds, extra = n % kXcds;
  std::vector<T> out(n);
  for (size_t b = 0; b < n; ++b) {
    const size_t x = b % kXcds, s = b / kXcds;
    out[b] = in[x * base + std::min(x, extra) + s];
  }
  return out;
}

// The per-pair arrays of the build (RV, RC, Z and, in the mixed precisions,
// the split copy of conj(RV)) hold one chunk of k pairs at a time.  A batch's
// pairs are cut into chunks of about g_chunk_budget bytes of those arrays (all
// systems together), so the workspace stays bounded as the k mesh grows.  A
// chunk is a range of block rows: the pairs whose first k point falls in a
// range (with time reversal, together with their images), so the dispatch
// order keeps the k tiles whole.
constexpr size_t kChunkBudget = size_t(6) << 30;
std::atomic<size_t> g_chunk_budget{kChunkBudget};

// One system's share of a chunk.
struct Chunk {
  int p0 = 0, np = 0;           // pairs [p0, p0 + np) in the system's pair order
  std::vector<PdJob> jv, jc;    // pairs transformed, rows local to the chunk
  std::vector<int4> fill;       // time-reversal images: (dst, src, q_dst << 1 | mode, sys), local pairs
  std::vector<S1Tile> s1;       // stage-1 tiles (q groups of the chunk)
  int d2items = 0;              // stage-2 items (pairs x 16 x 16 tiles)
  std::vector<int4> dwt, rvt;   // adjoint tiles (q, row tile, column tile, -) of the q groups present
  bool has_q0 = false;          // holds pairs of q = 0
};

struct Plan {
  // N1, N2, N3 and every Miller index, shift and window below are in the
  // pair-density frame: frame axis d is grid axis ax[d].  The frame is the
  // grid itself unless the planes N2 x N3 are too long for the one-lane-per-
  // line kernel while N1 x N2 planes are not; then the axes are rotated,
  // (j1, j2, j3) -> (j3, j1, j2), and the wave functions are transposed once
  // per build into the workspace (o_ut).
  int ax[3] = {0, 1, 2};
  bool rot = false;
  int N1 = 0, N2 = 0, N3 = 0, nk = 0, nv = 0, nc = 0, nb = 0, ng_max = 0, ns = 0, nt = 0;
  int lo[3] = {0, 0, 0}, F[3] = {0, 0, 0};
  std::vector<int> gpack, ng;
  std::vector<PdJob> jx;           // exchange pair densities (k, k+Q), natural order
  int qexc = 0;                    // exciton momentum Q (q-mesh index)
  std::vector<int> kq;             // per k: mesh index of k + Q
  int g0x = 0;                     // position of G = 0 in the sphere of Q (-1: absent)
  // coupling block of the beyond-TDA matrix: every ordered pair, rows (v, c') and (c, v')
  bool coupling = false;
  bool cswap = false;              // coupling: the (c, v') rows of (k, k') gathered from the (v, c') rows of (k', k)
  int ldh = 0;                     // row stride of the output matrix
  int rv_rows = 0, rc_rows = 0;    // rows per pair of RV / Z and of RC
  std::vector<int> inv0;           // coupling: position of -G in the q = 0 sphere
  std::vector<int> qbar, trmap;    // time-reversal partner of q; sphere map t - m
  // W from the irreducible q points: (source, conjugate) per q, the sphere maps, and
  // the sphere size of every source matrix (0: no q maps to it)
  int nirr = 0;
  std::vector<int> wsrc, wmap, ngirr;
  bool tr_closed = true;
  std::vector<int> ktr;            // per k: kbar | K << 24 (grid axes)
  // pairs k <= k', chunk after chunk, sorted by (q, k, k') inside a chunk
  std::vector<int4> pairs;         // (ka, kb, iq, m0p)
  std::vector<int> plex;           // lexicographic position of each pair among k <= k'
  std::vector<int> qs;             // [nchunk][nk + 1] first pair of each q group of the chunk
  std::vector<Chunk> ch;
  int maxcp = 0;                   // pairs of the largest chunk
  std::vector<HTile> xt, mt;       // exchange tiles; mirror tiles
  bool pd32 = false;               // FP32 valence / conduction pair densities
  bool mixed = false;              // split buffers of the mixed precisions reserved
  int kpad = 0;                    // ng_max rounded up to a multiple of 32
  // byte offsets inside the system's region of the workspace
  size_t o_gpack = 0, o_ng = 0, o_pairs = 0, o_qs = 0, o_plex = 0, o_qbar = 0, o_trmap = 0, o_ktr = 0, o_kq = 0;
  size_t o_inv0 = 0, o_Xb = 0;     // coupling only
  size_t o_wsrc = 0, o_wmap = 0, o_ngirr = 0;  // nirr > 0 only
  size_t tables = 0, o_vs = 0, o_X = 0, o_RV = 0, o_RC = 0, o_Z = 0, o_dWraw = 0, total = 0;
  size_t o_ut = 0;   // rotated wave functions (rot only)
  size_t o_u32 = 0;  // FP32 copy of the wave functions in the frame (pd32 only)
  size_t o_Ws = 0;   // W split for the mixed stage 1: [Nk][ng_max][4][kpad] of up to 4 bytes (mixed only)
  size_t o_RVs = 0;  // conj(RV) split for the mixed stage 1: [rows][4][kpad] (mixed only)
};

// need_w: the build's inputs W and vx are required (not by the screening).
int check_system(const bse_system* s, bool need_w = true) {
  if (!s) return fail(BSE_ERR_INVALID_ARG, "system pointer is NULL");
  for (int d = 0; d < 3; ++d) {
    if (s->grid[d] < 1 || s->grid[d] > 4096) return fail(BSE_ERR_SHAPE, "grid[%d] = %d out of range", d, s->grid[d]);
    if (s->kmesh[d] < 1 || s->kmesh[d] > 1024) return fail(BSE_ERR_SHAPE, "kmesh[%d] = %d out of range", d, s->kmesh[d]);
  }
  if (!pd_grid_supported(s->grid[1], s->grid[2]) && !(pd_line_grid(s->grid[0], s->grid[1]) && s->grid[2] <= 256))
    return fail(BSE_ERR_SHAPE, "grid (N2, N3) = (%d, %d) has no FFT kernel", s->grid[1], s->grid[2]);
  if (s->nv < 1 || s->nc < 1 || s->nv > 255 || s->nc > 255) return fail(BSE_ERR_SHAPE, "nv/nc out of range");
  if (s->ng_max < 1 || s->ng_max > 1024) return fail(BSE_ERR_SHAPE, "ng_max = %d out of range (1..1024)", s->ng_max);
  if (!(s->omega_cell > 0.0)) return fail(BSE_ERR_INVALID_ARG, "omega_cell must be positive");
  if (!s->ng || !s->gvec) return fail(BSE_ERR_INVALID_ARG, "ng / gvec host tables are NULL");
  if (!s->u || !s->eps || (need_w && (!s->W || !s->vx)))
    return fail(BSE_ERR_INVALID_ARG, "a device input pointer is NULL");
  const long long nk = (long long)s->kmesh[0] * s->kmesh[1] * s->kmesh[2];
  if (s->qexc < 0 || s->qexc >= nk) return fail(BSE_ERR_INVALID_ARG, "qexc = %d not in 0..Nk-1", s->qexc);
  if (s->nirr < 0 || s->nirr > nk) return fail(BSE_ERR_INVALID_ARG, "nirr = %d not in 0..Nk", s->nirr);
  if (s->nirr > 0 && (!s->wsrc || !s->wmap)) return fail(BSE_ERR_INVALID_ARG, "nirr > 0 needs the wsrc and wmap tables");
  return BSE_OK;
}

// What a batch is planned for besides its systems.
struct BatchOpts {
  bool backward = false;  // room and tiles for the adjoint
  bool project = false;   // backward with the projection of dW (its raw buffer)
  bool tr = false;        // time-reversal images gathered (BSE_TIME_REVERSAL)
  bool pd32 = false;      // FP32 pair densities where the one-lane-per-line kernel applies
  bool mixed = false;     // split buffers of the mixed-precision stage 1
  bool coupling = false;  // the coupling block of the beyond-TDA matrix (FP64, Q = 0)
  int ldh = 0;            // row stride of the output (0: NS)
};

// Frame, spheres, windows, exchange jobs and time-reversal maps of one system.
int make_geometry(const bse_system* s, Plan& P, bool need_w = true) {
  int rc = check_system(s, need_w);
  if (rc) return rc;
  P.rot = !pd_line_grid(s->grid[1], s->grid[2]) && pd_line_grid(s->grid[0], s->grid[1]) && s->grid[2] <= 256;
  if (P.rot) {
    P.ax[0] = 2;
    P.ax[1] = 0;
    P.ax[2] = 1;
  }
  P.N1 = s->grid[P.ax[0]];
  P.N2 = s->grid[P.ax[1]];
  P.N3 = s->grid[P.ax[2]];
  P.nk = s->kmesh[0] * s->kmesh[1] * s->kmesh[2];
  P.nv = s->nv;
  P.nc = s->nc;
  P.nb = s->nv + s->nc;
  P.ng_max = s->ng_max;
  P.nt = s->nv * s->nc;
  const long long ns = (long long)P.nk * P.nt;
  if (ns > (1LL << 20)) return fail(BSE_ERR_SHAPE, "NS = %lld too large", ns);
  P.ns = (int)ns;
  P.ng.assign(s->ng, s->ng + P.nk);
  P.gpack.assign((size_t)P.nk * P.ng_max, pack_m(0, 0, 0));
  int mlo[3] = {1 << 20, 1 << 20, 1 << 20}, mhi[3] = {-(1 << 20), -(1 << 20), -(1 << 20)};
  for (int q = 0; q < P.nk; ++q) {
    if (P.ng[q] < 1 || P.ng[q] > P.ng_max) return fail(BSE_ERR_SHAPE, "ng[%d] = %d not in 1..ng_max", q, P.ng[q]);
    for (int g = 0; g < P.ng[q]; ++g) {
      const int* m = s->gvec + ((size_t)q * P.ng_max + g) * 3;
      for (int d = 0; d < 3; ++d) {
        const int md = m[P.ax[d]];
        if (md < -500 || md > 500) return fail(BSE_ERR_SHAPE, "Miller index out of range");
        mlo[d] = std::min(mlo[d], md);
        mhi[d] = std::max(mhi[d], md);
      }
      P.gpack[(size_t)q * P.ng_max + g] = pack_m(m[P.ax[0]], m[P.ax[1]], m[P.ax[2]]);
    }
  }
  if (s->gvec[0] != 0 || s->gvec[1] != 0 || s->gvec[2] != 0)
    return fail(BSE_ERR_SHAPE, "gvec[0][0] must be G = 0");
  // W of the irreducible q points: every source index, flag and map entry in
  // range (the gathers rely on it), one sphere size per source, maps bijective
  P.nirr = s->nirr;
  P.wsrc.clear();
  P.wmap.clear();
  P.ngirr.clear();
  if (P.nirr > 0) {
    P.wsrc.assign(s->wsrc, s->wsrc + 2 * (size_t)P.nk);
    P.wmap.assign((size_t)P.nk * P.ng_max, 0);
    P.ngirr.assign(P.nirr, 0);
    std::vector<int> seen(P.ng_max);
    for (int q = 0; q < P.nk; ++q) {
      const int src = P.wsrc[2 * q], cj = P.wsrc[2 * q + 1];
      if (src < 0 || src >= P.nirr || (cj != 0 && cj != 1))
        return fail(BSE_ERR_INVALID_ARG, "wsrc[%d] = (%d, %d): source not in 0..nirr-1 or flag not 0/1", q, src, cj);
      if (P.ngirr[src] && P.ngirr[src] != P.ng[q])
        return fail(BSE_ERR_SHAPE, "q = %d maps to W matrix %d with ng %d, another q with ng %d", q, src, P.ng[q],
                    P.ngirr[src]);
      P.ngirr[src] = P.ng[q];
      std::fill(seen.begin(), seen.end(), 0);
      for (int g = 0; g < P.ng[q]; ++g) {
        const int m = s->wmap[(size_t)q * P.ng_max + g];
        if (m < 0 || m >= P.ng[q]) return fail(BSE_ERR_INVALID_ARG, "wmap[%d][%d] = %d not in 0..ng(q)-1", q, g, m);
        if (seen[m]++) return fail(BSE_ERR_SHAPE, "wmap[%d] is not a permutation (entry %d twice)", q, m);
        P.wmap[(size_t)q * P.ng_max + g] = m;
      }
    }
    if (P.wmap[0] != 0) return fail(BSE_ERR_SHAPE, "wmap[0][0] must be 0 (G = 0 of q = 0)");
  }
  // kept frequencies f = m - m0 with m0 in {-1, 0} along axes with more than one k
  const int N[3] = {P.N1, P.N2, P.N3};
  for (int d = 0; d < 3; ++d) {
    P.lo[d] = mlo[d];
    const int hi = mhi[d] + (s->kmesh[P.ax[d]] > 1 ? 1 : 0);
    P.F[d] = hi - P.lo[d] + 1;
    if (P.F[d] > N[d])
      return fail(BSE_ERR_SHAPE, "G-sphere window %d exceeds grid %d along axis %d", P.F[d], N[d], d);
  }
  // exciton momentum: the electron of S = (k, v, c) sits at k + Q, so the
  // exchange densities pair (k, k + Q) on the sphere of Q
  P.qexc = s->qexc;
  P.kq.resize(P.nk);
  {
    const int* n = s->kmesh;
    const int Q = P.qexc, q1 = Q / (n[1] * n[2]), q2 = (Q / n[2]) % n[1], q3 = Q % n[2];
    for (int k = 0; k < P.nk; ++k) {
      const int a = (k / (n[1] * n[2]) + q1) % n[0], b = ((k / n[2]) % n[1] + q2) % n[1], c = (k % n[2] + q3) % n[2];
      P.kq[k] = (a * n[1] + b) * n[2] + c;
    }
  }
  P.g0x = -1;
  for (int g = 0; g < P.ng[P.qexc]; ++g) {
    const int* m = s->gvec + ((size_t)P.qexc * P.ng_max + g) * 3;
    if (m[0] == 0 && m[1] == 0 && m[2] == 0) {
      P.g0x = g;
      break;
    }
  }
  P.jx.resize(P.nk);
  for (int k = 0; k < P.nk; ++k) {
    int iq, m0[3];
    fold(s->kmesh, k, P.kq[k], iq, m0);
    P.jx[k] = PdJob{k, P.kq[k], pack_m(m0[P.ax[0]], m0[P.ax[1]], m0[P.ax[2]]), iq, 0, P.nv, P.nv | (P.nc << 8),
                    k * P.nt};
  }

  // time reversal on the q mesh: qbar = -q mod n, and the index of t - m_g in
  // the sphere of qbar (-q = qbar + t)
  P.qbar.assign(P.nk, 0);
  P.trmap.assign((size_t)P.nk * P.ng_max, 0);
  P.tr_closed = true;
  {
    std::vector<std::vector<std::pair<int, int>>> sorted(P.nk);
    for (int q = 0; q < P.nk; ++q) {
      sorted[q].resize(P.ng[q]);
      for (int g = 0; g < P.ng[q]; ++g) sorted[q][g] = {P.gpack[(size_t)q * P.ng_max + g], g};
      std::sort(sorted[q].begin(), sorted[q].end());
    }
    const int* n = s->kmesh;
    for (int q = 0; q < P.nk; ++q) {
      const int iv[3] = {q / (n[1] * n[2]), (q / n[2]) % n[1], q % n[2]};
      int qb[3], tt[3];
      for (int d = 0; d < 3; ++d) {
        qb[d] = imod(-iv[d], n[d]);
        tt[d] = (-iv[d] - qb[d]) / n[d];
      }
      const int iqb = (qb[0] * n[1] + qb[1]) * n[2] + qb[2];
      P.qbar[q] = iqb;
      for (int g = 0; g < P.ng[q]; ++g) {
        int m1, m2, m3;
        unpack_m(P.gpack[(size_t)q * P.ng_max + g], m1, m2, m3);
        const int want = pack_m(tt[P.ax[0]] - m1, tt[P.ax[1]] - m2, tt[P.ax[2]] - m3);
        const auto& sv = sorted[iqb];
        const auto it = std::lower_bound(sv.begin(), sv.end(), std::make_pair(want, -1));
        const int found = (it != sv.end() && it->first == want) ? it->second : -1;
        if (found < 0) P.tr_closed = false;
        P.trmap[(size_t)q * P.ng_max + g] = found < 0 ? 0 : found;
      }
    }
  }
  // time reversal on the k mesh: -k = kbar - K
  P.ktr.assign(P.nk, 0);
  {
    const int* n = s->kmesh;
    for (int k = 0; k < P.nk; ++k) {
      const int iv[3] = {k / (n[1] * n[2]), (k / n[2]) % n[1], k % n[2]};
      int kb[3], bits = 0;
      for (int d = 0; d < 3; ++d) {
        kb[d] = imod(-iv[d], n[d]);
        bits |= ((kb[d] + iv[d]) / n[d]) << (24 + d);
      }
      P.ktr[k] = ((kb[0] * n[1] + kb[1]) * n[2] + kb[2]) | bits;
    }
  }
  return BSE_OK;
}

// Bytes of the per-pair arrays of one pair.
size_t pair_bytes(const bse_system* s, bool mixed, bool coupling = false) {
  const size_t ngm = (size_t)s->ng_max, kpad = (ngm + 31) / 32 * 32;
  if (coupling) return sizeof(double2) * ngm * 3 * (size_t)s->nv * s->nc;  // RV, RC and Z rows
  size_t b = sizeof(double2) * ngm * (2 * (size_t)s->nv * s->nv + (size_t)s->nc * s->nc);
  if (mixed) b += (size_t)s->nv * s->nv * 4 * kpad * sizeof(float);
  return b;
}

// The pairs k <= k' cut into at most `nchunk` chunks, their jobs and tiles,
// and the workspace layout.  `sys` tags the jobs and fill items.
int plan_pairs(const bse_system* s, Plan& P, const BatchOpts& opt, int nchunk, int sys, int s1_rows) {
  const int nk = P.nk, nv = P.nv, nc = P.nc;
  P.coupling = opt.coupling;
  P.ldh = opt.ldh > 0 ? opt.ldh : P.ns;
  P.rv_rows = P.coupling ? nv * nc : nv * nv;
  P.rc_rows = P.coupling ? nc * nv : nc * nc;
  // the coupling block has no symmetry between (k, k') and (k', k): every ordered pair
  const long long npl = P.coupling ? (long long)nk * nk : (long long)nk * (nk + 1) / 2;
  if (npl > (1LL << 30)) return fail(BSE_ERR_SHAPE, "too many k pairs (%lld)", npl);
  const int np = (int)npl;
  // lexicographic pairs (ka, kb), ka <= kb (coupling: every kb)
  auto lex = [nk](long long a, long long b) { return (int)(a * nk - a * (a - 1) / 2 + (b - a)); };
  std::vector<int2> lp(np);
  for (int a = 0, i = 0; a < nk; ++a)
    for (int b = P.coupling ? 0 : a; b < nk; ++b) lp[i++] = make_int2(a, b);
  // units: a transformed pair and, with time reversal, the image gathered from it.
  // Coupling block with spheres closed under G -> t - G: the unit is (k, k') with
  // k <= k' and its reverse (k', k); only their (v, c') rows are transformed, and
  // n_{ck, v'k'}(G) = conj(n_{v'k', ck}(t - G)) (-q = qbar + t) gives the (c, v')
  // rows of each from the other's (of itself when k = k').
  struct Unit {
    int rep, img, mode;
  };
  std::vector<Unit> units;
  units.reserve(np);
  P.cswap = P.coupling && P.tr_closed;
  for (int p = 0; p < np; ++p) {
    if (P.cswap) {
      const int ka = lp[p].x, kb = lp[p].y;
      if (ka > kb) continue;  // the reverse of a unit
      units.push_back(Unit{p, ka < kb ? kb * nk + ka : -1, 0});
      continue;
    }
    if (!opt.tr) {
      units.push_back(Unit{p, -1, 0});
      continue;
    }
    const int ka = lp[p].x, kb = lp[p].y;
    const int x = P.ktr[ka] & 0xffffff, y = P.ktr[kb] & 0xffffff;
    if (x == ka || y == kb) {  // touches a point that is its own partner: transformed
      units.push_back(Unit{p, -1, 0});
      continue;
    }
    const int img = lex(std::min(x, y), std::max(x, y));
    if (img < p) continue;  // gathered from its image
    units.push_back(Unit{p, img == p ? -1 : img, x <= y ? 0 : 1});
  }
  // chunks: consecutive units, cut between block rows once a chunk holds its share
  nchunk = std::max(1, std::min(nchunk, np));
  const long long target = (npl + nchunk - 1) / nchunk;
  std::vector<std::vector<const Unit*>> cu(1);
  long long acc = 0;
  for (size_t i = 0; i < units.size(); ++i) {
    cu.back().push_back(&units[i]);
    acc += units[i].img >= 0 ? 2 : 1;
    const bool row_end = i + 1 == units.size() || lp[units[i + 1].rep].x != lp[units[i].rep].x;
    if (row_end && acc >= target * (long long)cu.size() && (int)cu.size() < nchunk && i + 1 < units.size())
      cu.emplace_back();
  }
  const int C = (int)cu.size();
  P.pairs.assign(np, make_int4(0, 0, 0, 0));
  P.plex.assign(np, 0);
  P.qs.assign((size_t)C * (nk + 1), 0);
  P.ch.assign(C, Chunk{});
  std::vector<int> g_of_lex(np, -1);
  int next = 0;
  P.maxcp = 0;
  const int T2 = (P.ng_max + 63) / 64;
  for (int c = 0; c < C; ++c) {
    Chunk& K = P.ch[c];
    std::vector<int> members;
    for (const Unit* u : cu[c]) {
      members.push_back(u->rep);
      if (u->img >= 0) members.push_back(u->img);
    }
    std::vector<int4> pr(members.size());
    for (size_t i = 0; i < members.size(); ++i) {
      const int ka = lp[members[i]].x, kb = lp[members[i]].y;
      int iq, m0[3];
      fold(s->kmesh, ka, kb, iq, m0);
      pr[i] = make_int4(ka, kb, iq, members[i]);  // .w: lexicographic index for now
    }
    // coupling with gathered rows: B is symmetric (B^T = B for Hermitian,
    // time-reversal-consistent W and even v, as the lower half of H2 assumes),
    // so only the pairs k <= k' are contracted; the reversed pairs, whose
    // densities are gather sources only, come after them
    const bool csym = P.cswap;
    std::sort(pr.begin(), pr.end(), [csym](const int4& x, const int4& y) {
      if (csym && (x.x > x.y) != (y.x > y.y)) return y.x > y.y;
      if (x.z != y.z) return x.z < y.z;
      if (x.x != y.x) return x.x < y.x;
      return x.y < y.y;
    });
    K.p0 = next;
    K.np = (int)pr.size();
    int ncontract = 0;  // pairs of the chunk whose blocks are contracted (the first ones)
    P.maxcp = std::max(P.maxcp, K.np);
    if ((long long)K.np * std::max(P.rv_rows, P.rc_rows) >= (1LL << 31) / std::max(P.ng_max, 1))
      return fail(BSE_ERR_SHAPE, "a chunk of %d k pairs is too large", K.np);
    std::vector<int> cnt(nk, 0);
    for (size_t i = 0; i < pr.size(); ++i) {
      const int g = next + (int)i, l = pr[i].w;
      int iq, m0[3];
      fold(s->kmesh, pr[i].x, pr[i].y, iq, m0);
      P.pairs[g] = make_int4(pr[i].x, pr[i].y, iq, pack_m(m0[P.ax[0]], m0[P.ax[1]], m0[P.ax[2]]));
      P.plex[g] = l;
      g_of_lex[l] = g;
      if (!(csym && pr[i].x > pr[i].y)) {
        cnt[iq]++;
        ++ncontract;
      }
    }
    int* qs = P.qs.data() + (size_t)c * (nk + 1);
    qs[0] = next;
    for (int q = 0; q < nk; ++q) qs[q + 1] = qs[q] + cnt[q];
    K.has_q0 = cnt[0] > 0;
    // jobs of the transformed pairs and the fill items of their images
    for (const Unit* u : cu[c]) {
      const int g = g_of_lex[u->rep], loc = g - next;
      const int4 q4 = P.pairs[g];
      if (P.cswap) {  // n_{vk, c'k'} of the pair and of its reverse; the (c, v') rows of each from the other
        K.jv.push_back(PdJob{q4.x, q4.y, q4.w, q4.z, 0, nv, nv | (nc << 8), loc * nv * nc});
        const int gi = u->img >= 0 ? g_of_lex[u->img] : g, li = gi - next;
        if (u->img >= 0) {
          const int4 r4 = P.pairs[gi];
          K.jv.push_back(PdJob{r4.x, r4.y, r4.w, r4.z, 0, nv, nv | (nc << 8), li * nv * nc});
        }
        K.fill.push_back(make_int4(loc, li, q4.z << 1, sys));  // (the reversed pair's block is mirrored)
        continue;
      }
      if (P.coupling) {  // n_{vk, c'k'} and n_{ck, v'k'}
        K.jv.push_back(PdJob{q4.x, q4.y, q4.w, q4.z, 0, nv, nv | (nc << 8), loc * nv * nc});
        K.jc.push_back(PdJob{q4.x, q4.y, q4.w, q4.z, nv, 0, nc | (nv << 8), loc * nc * nv});
        continue;
      }
      K.jv.push_back(PdJob{q4.x, q4.y, q4.w, q4.z, 0, 0, nv | (nv << 8), loc * nv * nv});
      if (P.qexc == 0) {
        K.jc.push_back(PdJob{q4.x, q4.y, q4.w, q4.z, nv, nv, nc | (nc << 8), loc * nc * nc});
      } else {  // conduction pair (k + Q, k' + Q), folded on its own (same q, its own G0)
        int iq, m0[3];
        fold(s->kmesh, P.kq[q4.x], P.kq[q4.y], iq, m0);
        if (iq != q4.z) return fail(BSE_ERR_INVALID_ARG, "internal: shifted pair changes q");
        K.jc.push_back(PdJob{P.kq[q4.x], P.kq[q4.y], pack_m(m0[P.ax[0]], m0[P.ax[1]], m0[P.ax[2]]), iq, nv, nv,
                             nc | (nc << 8), loc * nc * nc});
      }
      if (u->img >= 0) {
        const int gi = g_of_lex[u->img];
        K.fill.push_back(make_int4(gi - next, loc, (P.pairs[gi].z << 1) | u->mode, sys));
      }
    }
    // stage-1 tiles per q group: rows = pairs(q) * nv^2, columns = ng(q)
    for (int q = 0; q < nk; ++q) {
      if (!cnt[q]) continue;
      const int rows = cnt[q] * P.rv_rows;
      const int mt = (rows + s1_rows - 1) / s1_rows, ntl = (P.ng[q] + 63) / 64;
      for (int i = 0; i < mt; ++i)
        for (int j = 0; j < ntl; ++j) K.s1.push_back(S1Tile{q, i, j, sys});
      if (opt.backward) {
        const int mt = (rows + 63) / 64;  // the backward's own tiles are 64 rows
        for (int i = 0; i < T2; ++i)
          for (int j = 0; j < T2; ++j) K.dwt.push_back(make_int4(q, i, j, 0));
        for (int i = 0; i < mt; ++i)
          for (int j = 0; j < T2; ++j) K.rvt.push_back(make_int4(q, i, j, 0));
      }
    }
    K.d2items = ncontract * ((P.rv_rows + 15) / 16) * ((P.rc_rows + 15) / 16);
    next += K.np;
  }
  // exchange tiles: every 64 x 64 tile that holds an entry of a block k <= k'
  // (its first row's k block is at most its last column's).  A k block of
  // nv*nc rows may span several tiles, so a diagonal block can reach tiles
  // well below the tile diagonal.
  P.xt.clear();
  const int T = (P.ns + 63) / 64;
  for (int i = 0; i < T; ++i)
    for (int j = 0; j < T; ++j) {
      const int last_col = std::min(P.ns, 64 * (j + 1)) - 1;
      if ((P.coupling && !P.cswap) || (64 * i) / P.nt <= last_col / P.nt) P.xt.push_back(HTile{i, j, sys, 0});
    }
  // mirror tiles: 32 x 32 destination tiles on or below the diagonal (the
  // coupling block: a plain transpose, when only its upper blocks are contracted)
  P.mt.clear();
  const int T32 = (P.ns + 31) / 32;
  for (int i = 0; i < T32 && (!P.coupling || P.cswap); ++i)
    for (int j = 0; j <= i; ++j) P.mt.push_back(HTile{i, j, sys, 0});
  // coupling: -G of every G of the q = 0 sphere (the h-e exchange densities)
  P.inv0.clear();
  if (P.coupling) {
    const int n0 = P.ng[0];
    P.inv0.assign(n0, -1);
    for (int g = 0; g < n0; ++g) {
      int a1, a2, a3;
      unpack_m(P.gpack[g], a1, a2, a3);
      for (int h = 0; h < n0; ++h) {
        int b1, b2, b3;
        unpack_m(P.gpack[h], b1, b2, b3);
        if (a1 == -b1 && a2 == -b2 && a3 == -b3) {
          P.inv0[g] = h;
          break;
        }
      }
      if (P.inv0[g] < 0) return fail(BSE_ERR_SHAPE, "the q = 0 sphere is not closed under G -> -G");
    }
  }

  // workspace layout
  size_t o = 0;
  auto put = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  P.o_gpack = put(P.gpack.size() * sizeof(int));
  P.o_ng = put(P.ng.size() * sizeof(int));
  P.o_pairs = put(P.pairs.size() * sizeof(int4));
  P.o_qs = put(P.qs.size() * sizeof(int));
  P.o_plex = put(P.plex.size() * sizeof(int));
  P.o_qbar = put(P.qbar.size() * sizeof(int));
  P.o_trmap = put(P.trmap.size() * sizeof(int));
  P.o_ktr = put(P.ktr.size() * sizeof(int));
  P.o_kq = put(P.kq.size() * sizeof(int));
  P.o_inv0 = put(P.inv0.size() * sizeof(int));
  P.o_wsrc = put(P.wsrc.size() * sizeof(int));
  P.o_wmap = put(P.wmap.size() * sizeof(int));
  P.o_ngirr = put(P.ngirr.size() * sizeof(int));
  P.tables = o;
  const size_t mc = (size_t)P.maxcp;
  P.o_vs = put((size_t)P.ng_max * sizeof(double));
  P.o_X = put((size_t)P.ns * P.ng_max * sizeof(double2));
  P.o_RV = put(mc * P.rv_rows * P.ng_max * sizeof(double2));
  P.o_RC = put(mc * P.rc_rows * P.ng_max * sizeof(double2));
  P.o_Z = put(mc * P.rv_rows * P.ng_max * sizeof(double2));
  if (P.coupling) P.o_Xb = put((size_t)P.ns * P.ng_max * sizeof(double2));
  if (P.rot) P.o_ut = put((size_t)P.nk * P.nb * P.N1 * P.N2 * P.N3 * sizeof(double2));
  P.kpad = (P.ng_max + 31) / 32 * 32;
  P.mixed = opt.mixed;
  if (P.mixed) {
    P.o_Ws = put((size_t)P.nk * P.ng_max * 4 * P.kpad * sizeof(float));
    P.o_RVs = put(mc * nv * nv * 4 * P.kpad * sizeof(float));
  }
  P.pd32 = opt.pd32 && pd_line_grid(P.N2, P.N3);
  if (P.pd32) P.o_u32 = put((size_t)P.nk * P.nb * P.N1 * P.N2 * P.N3 * sizeof(float2));
  if (opt.backward && opt.project) P.o_dWraw = put((size_t)P.nk * P.ng_max * P.ng_max * sizeof(double2));
  P.total = o;
  return BSE_OK;
}

// Host tables of one system at `base` inside the workspace (the region the
// system's plan laid out).
void put_tables(const Plan& P, std::vector<char>& buf, size_t base) {
  auto cp = [&](size_t off, const void* src, size_t bytes) {
    if (bytes) std::memcpy(buf.data() + base + off, src, bytes);
  };
  cp(P.o_gpack, P.gpack.data(), P.gpack.size() * sizeof(int));
  cp(P.o_ng, P.ng.data(), P.ng.size() * sizeof(int));
  cp(P.o_pairs, P.pairs.data(), P.pairs.size() * sizeof(int4));
  cp(P.o_qs, P.qs.data(), P.qs.size() * sizeof(int));
  cp(P.o_plex, P.plex.data(), P.plex.size() * sizeof(int));
  cp(P.o_qbar, P.qbar.data(), P.qbar.size() * sizeof(int));
  cp(P.o_trmap, P.trmap.data(), P.trmap.size() * sizeof(int));
  cp(P.o_ktr, P.ktr.data(), P.ktr.size() * sizeof(int));
  cp(P.o_kq, P.kq.data(), P.kq.size() * sizeof(int));
  cp(P.o_inv0, P.inv0.data(), P.inv0.size() * sizeof(int));
  cp(P.o_wsrc, P.wsrc.data(), P.wsrc.size() * sizeof(int));
  cp(P.o_wmap, P.wmap.data(), P.wmap.size() * sizeof(int));
  cp(P.o_ngirr, P.ngirr.data(), P.ngirr.size() * sizeof(int));
}

PdArgs pd_args(const Plan& P, const bse_system* s, char* region) {
  PdArgs a{};
  a.u = P.rot ? reinterpret_cast<const double2*>(region + P.o_ut) : reinterpret_cast<const double2*>(s->u);
  a.nb = P.nb;
  a.N1 = P.N1;
  a.gpack = reinterpret_cast<const int*>(region + P.o_gpack);
  a.ng = reinterpret_cast<const int*>(region + P.o_ng);
  a.ng_max = P.ng_max;
  a.lo2 = P.lo[1];
  a.lo3 = P.lo[2];
  a.F2 = P.F[1];
  a.F3 = P.F[2];
  a.vscale = nullptr;
  a.out = nullptr;
  a.u32 = P.pd32 ? reinterpret_cast<const float2*>(region + P.o_u32) : nullptr;
  return a;
}

// Contraction arguments of chunk c of a system (chunk 0 for the exchange and
// the mirror, which do not depend on it).
GemmArgs gemm_args(const Plan& P, const bse_system* s, char* region, int c) {
  GemmArgs g{};
  g.X = reinterpret_cast<const double2*>(region + P.o_X);
  g.ns = P.ns;
  g.ng_max = P.ng_max;
  g.ngx = P.ng[P.qexc];
  g.kq = P.qexc ? reinterpret_cast<const int*>(region + P.o_kq) : nullptr;
  g.H = reinterpret_cast<double2*>(s->H);
  g.cpref = 27.211386245988 / ((double)P.nk * s->omega_cell);
  g.RV = reinterpret_cast<const double2*>(region + P.o_RV);
  g.RC = reinterpret_cast<const double2*>(region + P.o_RC);
  g.Z = reinterpret_cast<double2*>(region + P.o_Z);
  g.W = reinterpret_cast<const double2*>(s->W);
  g.wsrc = P.nirr ? reinterpret_cast<const int*>(region + P.o_wsrc) : nullptr;
  g.wmap = P.nirr ? reinterpret_cast<const int*>(region + P.o_wmap) : nullptr;
  g.W0 = g.W + (P.nirr ? (size_t)P.wsrc[0] * P.ng_max * P.ng_max : 0);
  g.ng = reinterpret_cast<const int*>(region + P.o_ng);
  const int cc = c < (int)P.ch.size() ? c : 0;
  g.qstart = reinterpret_cast<const int*>(region + P.o_qs) + (size_t)cc * (P.nk + 1);
  g.pairs = reinterpret_cast<const int4*>(region + P.o_pairs);
  g.p0 = P.ch[cc].p0;
  g.eps = s->eps;
  g.nv = P.nv;
  g.nc = P.nc;
  g.nb = P.nb;
  g.npairs = P.ch[cc].np;
  g.nt = P.nt;
  g.Ws = P.mixed ? region + P.o_Ws : nullptr;
  g.kpad = P.kpad;
  g.RVs = P.mixed ? region + P.o_RVs : nullptr;
  g.ldh = P.ldh;
  g.rv_rows = P.rv_rows;
  g.rc_rows = P.rc_rows;
  g.coupling = P.coupling;
  g.mirror_plain = P.coupling ? 1 : 0;
  g.Xb = P.coupling ? reinterpret_cast<const double2*>(region + P.o_Xb) : nullptr;
  return g;
}

// ------------------------------------------------------------ batches

// Launch choices that the autotuner may change (per batch signature).
struct Tune {
  int persist = 0;    // persistent work-queue dispatch of the pair-density jobs
  int ktile = 8;      // k tile of the pair-density dispatch order
  int wg_per_cu = 2;  // persistent grid: workgroups per CU
  float pd_ms = 0.f;  // measured time of the tuned pair-density launch (0: not measured)
  int s1_rows = 64;   // rows per tile of the direct term's first contraction (64 or 128)
  float s1_ms = 0.f;  // measured time of that launch (0: not measured)
  int order = 0;      // pair-density job order: 0 per-XCD segments, 1 interleaved, 2 kind-major segments
};
std::mutex g_tune_mu;
std::vector<std::pair<std::string, Tune>> g_tune;

// Signature of a batch: everything that shapes its launches.
std::string batch_key(const std::vector<Plan>& Ps, int precision, bool pd32) {
  std::string k = "p" + std::to_string(precision) + (pd32 ? "f32" : "");
  for (const Plan& P : Ps) {
    char b[160];
    snprintf(b, sizeof b, "|%dx%dx%d:k%d:b%d+%d:g%d:w%dx%d", P.N1, P.N2, P.N3, P.nk, P.nv, P.nc, P.ng_max, P.F[1],
             P.F[2]);
    k += b;
  }
  return k;
}

Tune tune_for(const std::string& key) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& e : g_tune)
    if (e.first == key) return e.second;
  return Tune{};
}

void set_tune(const std::string& key, const Tune& t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& e : g_tune)
    if (e.first == key) {
      e.second = t;
      return;
    }
  g_tune.emplace_back(key, t);
}

// One chunk of a batch: the merged launch lists of every system's share.  The
// valence and conduction pair densities of a chunk are one launch: the jobs of
// system i name argument set 2 i (valence rows) or 2 i + 1 (conduction rows).
struct BatchChunk {
  std::vector<PdJob> jd;
  std::vector<int4> fill;
  std::vector<S1Tile> s1;
  std::vector<int> d2off;  // [nsys + 1]
  int d2n = 0;
  std::vector<int4> dwt, rvt;  // single system (backward)
  bool has_q0 = false;         // single system (backward)
  size_t o_jd = 0, o_fill = 0, o_s1 = 0, o_d2off = 0, o_gargs = 0, o_dwt = 0, o_rvt = 0;
};

// A batch of systems that share (N2, N3): per-system plans and workspace
// regions, and the merged job and tile lists of the one-launch-per-stage build.
struct Batch {
  std::vector<Plan> P;
  std::vector<size_t> base;  // workspace offset of each system's region
  int N2 = 0, N3 = 0, ng_max = 0;
  size_t lds = 0;
  std::vector<PdJob> jx;
  std::vector<HTile> xt, mt;
  std::vector<BatchChunk> C;
  bool tr = false;             // pair densities of time-reversal images derived
  bool pd32 = false;           // FP32 valence / conduction pair densities
  bool mapped = false;         // some system gives W at the irreducible q points only
  bool cswap = false;          // coupling rows gathered from the reversed pairs (fill kind 3)
  int s1_rows = 64;            // rows per tile of the first direct-term contraction
  int np32 = 2;                // their planes per step: 4 when every window has F2 <= 16
  size_t lds32 = 0;            // their LDS bytes
  size_t o_pdx = 0, o_pdd = 0, o_jx = 0, o_xt = 0, o_mt = 0, o_tra = 0;
  size_t o_cnt = 0, tables = 0, total = 0;
};

int make_batch(const bse_system* sys, int nsys, const Tune& tn, const BatchOpts& opt, Batch& B) {
  if (!sys || nsys < 1) return fail(BSE_ERR_INVALID_ARG, "no systems");
  B.tr = opt.tr;
  B.pd32 = opt.pd32;
  if (tn.s1_rows != 64 && tn.s1_rows != 128) return fail(BSE_ERR_INVALID_ARG, "stage-1 tile rows must be 64 or 128");
  B.s1_rows = tn.s1_rows;
  if (nsys > 16383) return fail(BSE_ERR_INVALID_ARG, "too many systems");
  B.P.resize(nsys);
  // chunk count: the per-pair arrays of all systems over the budget
  double bytes = 0.0;
  for (int i = 0; i < nsys; ++i) {
    int rc = check_system(&sys[i]);
    if (rc) return rc;
    const double nk = (double)sys[i].kmesh[0] * sys[i].kmesh[1] * sys[i].kmesh[2];
    bytes += (opt.coupling ? nk * nk : nk * (nk + 1) / 2) * (double)pair_bytes(&sys[i], opt.mixed, opt.coupling);
  }
  const int nchunk = (int)std::min(1e6, std::max(1.0, std::ceil(bytes / (double)g_chunk_budget.load())));
  for (int i = 0; i < nsys; ++i) {
    int rc = make_geometry(&sys[i], B.P[i]);
    if (rc) return rc;
    if (B.P[i].qexc && opt.tr)
      return fail(BSE_ERR_INVALID_ARG, "system %d: BSE_TIME_REVERSAL needs exciton momentum Q = 0", i);
    if (B.P[i].nirr && opt.backward)
      return fail(BSE_ERR_UNSUPPORTED, "system %d: the backward needs W at every q (nirr = 0)", i);
    if ((rc = plan_pairs(&sys[i], B.P[i], opt, nchunk, i, B.s1_rows))) return rc;
    const Plan& P = B.P[i];
    if (i == 0) {
      B.N2 = P.N2;
      B.N3 = P.N3;
    } else if (P.N2 != B.N2 || P.N3 != B.N3) {
      return fail(BSE_ERR_SHAPE, "systems of one batch must share N2, N3 (system %d has %d x %d, not %d x %d)", i, P.N2,
                  P.N3, B.N2, B.N3);
    }
    B.ng_max = std::max(B.ng_max, P.ng_max);
    B.mapped = B.mapped || P.nirr > 0;
    B.cswap = B.cswap || P.cswap;
    const size_t l = pd_lds_bytes(P.N1, P.N2, P.N3, P.F[1], P.F[2], P.ng_max, 0);
    B.pd32 = B.pd32 && P.pd32;
    if (l > 160 * 1024) return fail(BSE_ERR_SHAPE, "FFT window of system %d needs more than 160 KiB of LDS", i);
    B.lds = std::max(B.lds, l);
    if (opt.tr && !P.tr_closed)
      return fail(BSE_ERR_SHAPE, "system %d: time reversal needs G spheres closed under G -> t - G (qbar = -q - t)", i);
  }
  if (B.pd32) {
    B.np32 = 4;
    for (const Plan& P : B.P) B.np32 = P.F[1] <= 16 ? B.np32 : 2;
    for (int tries = 0; tries < 2; ++tries) {
      B.lds32 = 0;
      for (const Plan& P : B.P)
        B.lds32 = std::max(B.lds32, pd_lds_bytes(P.N1, P.N2, P.N3, P.F[1], P.F[2], P.ng_max, B.np32));
      if (B.lds32 <= 160 * 1024 || B.np32 == 2) break;
      B.np32 = 2;  // four planes' windows do not fit the LDS
    }
  }
  // merged lists
  int nc = 0;
  for (const Plan& P : B.P) nc = std::max(nc, (int)P.ch.size());
  B.C.assign(nc, BatchChunk{});
  std::vector<PdJob> jx;
  for (int i = 0; i < nsys; ++i) {
    const Plan& P = B.P[i];
    for (PdJob j : P.jx) jx.push_back((j.nab |= i << 16, j));
    B.xt.insert(B.xt.end(), P.xt.begin(), P.xt.end());
    B.mt.insert(B.mt.end(), P.mt.begin(), P.mt.end());
  }
  B.jx = dispatch_order(std::move(jx), tn.ktile, tn.order);
  for (int c = 0; c < nc; ++c) {
    BatchChunk& K = B.C[c];
    std::vector<PdJob> jd;
    K.d2off.assign(nsys + 1, 0);
    for (int i = 0; i < nsys; ++i) {
      const Plan& P = B.P[i];
      K.d2off[i + 1] = K.d2off[i];
      if (c >= (int)P.ch.size()) continue;
      const Chunk& S = P.ch[c];
      for (PdJob j : S.jv) jd.push_back((j.nab |= (2 * i) << 16, j));
      for (PdJob j : S.jc) jd.push_back((j.nab |= (2 * i + 1) << 16, j));
      K.fill.insert(K.fill.end(), S.fill.begin(), S.fill.end());
      K.s1.insert(K.s1.end(), S.s1.begin(), S.s1.end());
      K.d2off[i + 1] += S.d2items;
      if (nsys == 1) {
        K.dwt = S.dwt;
        K.rvt = S.rvt;
        K.has_q0 = S.has_q0;
      }
    }
    K.d2n = K.d2off[nsys];
    K.jd = dispatch_order(std::move(jd), tn.ktile, tn.order);
    K.s1 = xcd_segments(K.s1);
  }
  // workspace: batch tables, then one region per system
  size_t o = 0;
  auto put = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  B.o_pdx = put(nsys * sizeof(PdArgs));
  B.o_pdd = put(2 * nsys * sizeof(PdArgs));
  B.o_jx = put(B.jx.size() * sizeof(PdJob));
  B.o_xt = put(B.xt.size() * sizeof(HTile));
  B.o_mt = put(B.mt.size() * sizeof(HTile));
  B.o_tra = put(opt.tr || B.cswap ? nsys * sizeof(TrArgs) : 0);
  for (BatchChunk& K : B.C) {
    K.o_gargs = put(nsys * sizeof(GemmArgs));
    K.o_jd = put(K.jd.size() * sizeof(PdJob));
    K.o_fill = put(K.fill.size() * sizeof(int4));
    K.o_s1 = put(K.s1.size() * sizeof(S1Tile));
    K.o_d2off = put(K.d2off.size() * sizeof(int));
    K.o_dwt = put(K.dwt.size() * sizeof(int4));
    K.o_rvt = put(K.rvt.size() * sizeof(int4));
  }
  // the tables above are uploaded as one image [0, o_cnt); the counters are not
  B.o_cnt = put(kCntBytes + 32 + 8 * sizeof(unsigned long long));  // queues, validation
  B.base.resize(nsys);
  for (int i = 0; i < nsys; ++i) {
    B.base[i] = o;
    o = align256(o + B.P[i].total);
  }
  B.total = o;
  return BSE_OK;
}

// Key of everything the host plan of a batch depends on: shapes, sphere
// tables (hashed by content), the options and the k tile.
std::string plan_key(const bse_system* sys, int nsys, const Tune& tn, const BatchOpts& o) {
  std::string k = std::to_string(nsys) + (o.backward ? "b" : "f") + (o.project ? "p" : "") + (o.tr ? "t" : "") +
                  (o.pd32 ? "s" : "") + (o.mixed ? "m" : "") + (o.coupling ? "x" : "") + "l" + std::to_string(o.ldh) +
                  "k" + std::to_string(tn.ktile) + "r" + std::to_string(tn.s1_rows) + "o" +
                  std::to_string(tn.order) + "c" +
                  std::to_string(g_chunk_budget.load());
  for (int i = 0; i < nsys; ++i) {
    const bse_system& s = sys[i];
    const int nk = s.kmesh[0] * s.kmesh[1] * s.kmesh[2];
    unsigned long long h = 1469598103934665603ull;  // FNV-1a over the host tables
    auto mix = [&](const void* p, size_t n) {
      const unsigned char* b = static_cast<const unsigned char*>(p);
      for (size_t j = 0; j < n; ++j) h = (h ^ b[j]) * 1099511628211ull;
    };
    if (s.ng) mix(s.ng, sizeof(int) * (size_t)std::max(nk, 0));
    if (s.gvec && s.ng_max > 0) mix(s.gvec, sizeof(int) * 3 * (size_t)std::max(nk, 0) * s.ng_max);
    if (s.nirr > 0 && s.wsrc && s.wmap && s.ng_max > 0) {
      mix(&s.nirr, sizeof(int));
      mix(s.wsrc, sizeof(int) * 2 * (size_t)std::max(nk, 0));
      mix(s.wmap, sizeof(int) * (size_t)std::max(nk, 0) * s.ng_max);
    }
    char b[200];
    snprintf(b, sizeof b, "|%d,%d,%d:%d,%d,%d:%d,%d:%d:%llx:Q%d", s.grid[0], s.grid[1], s.grid[2], s.kmesh[0],
             s.kmesh[1], s.kmesh[2], s.nv, s.nc, s.ng_max, h, s.qexc);
    k += b;
  }
  return k;
}

// The last few host plans built on this thread (least recently used one
// replaced): a repeated build of the same batch shape skips planning, also
// when a tuned k tile asks for a second plan of the same batch.
struct PlanCache {
  std::string key;
  Batch B;
  unsigned long long used = 0;
};
constexpr int kPlanSlots = 4;
thread_local PlanCache g_plan[kPlanSlots];
thread_local unsigned long long g_plan_clock = 0;

// make_batch through the cache.
int cached_batch(const bse_system* sys, int nsys, const Tune& tn, const BatchOpts& opt, const Batch** out) {
  if (nsys < 1 || !sys) return fail(BSE_ERR_INVALID_ARG, "no systems");
  for (int i = 0; i < nsys; ++i) {
    int rc = check_system(&sys[i]);
    if (rc) return rc;
  }
  const std::string key = plan_key(sys, nsys, tn, opt);
  PlanCache* slot = nullptr;
  for (PlanCache& c : g_plan)
    if (!c.key.empty() && c.key == key) slot = &c;
  if (!slot) {
    slot = &g_plan[0];
    for (PlanCache& c : g_plan)
      if (c.used < slot->used) slot = &c;
    Batch B;
    int rc = make_batch(sys, nsys, tn, opt, B);
    if (rc) {
      slot->key.clear();
      slot->used = 0;
      return rc;
    }
    slot->B = std::move(B);
    slot->key = key;
  }
  slot->used = ++g_plan_clock;
  *out = &slot->B;
  return BSE_OK;
}

// Uploads every table of the batch (asynchronous copies from pinned staging).
int upload_batch(const Batch& B, const bse_system* sys, int precision, char* ws, hipStream_t st) {
  const int nsys = (int)B.P.size();
  // staging image: the batch tables, then each system's own tables
  size_t n = B.o_cnt;
  std::vector<size_t> at(nsys);
  for (int i = 0; i < nsys; ++i) {
    at[i] = n;
    n += B.P[i].tables;
  }
  char* buf = nullptr;
  int rc = staging_acquire(n, &buf);
  if (rc) return rc;
  std::memset(buf, 0, n);
  auto cp = [&](size_t off, const void* src, size_t bytes) {
    if (bytes) std::memcpy(buf + off, src, bytes);
  };
  std::vector<PdArgs> ax(nsys), ad(2 * nsys);
  std::vector<TrArgs> ta(B.tr || B.cswap ? nsys : 0);
  for (int i = 0; i < nsys; ++i) {
    const Plan& P = B.P[i];
    char* region = ws + B.base[i];
    PdArgs a = pd_args(P, &sys[i], region);
    ax[i] = a;
    ax[i].vscale = reinterpret_cast<const double*>(region + P.o_vs);
    ax[i].out = reinterpret_cast<double2*>(region + P.o_X);
    ad[2 * i] = a;
    ad[2 * i].out = reinterpret_cast<double2*>(region + P.o_RV);
    ad[2 * i + 1] = a;
    ad[2 * i + 1].out = reinterpret_cast<double2*>(region + P.o_RC);
    if (B.tr || B.cswap) {
      TrArgs& r = ta[i];
      r.rv = reinterpret_cast<double2*>(region + P.o_RV);
      r.rc = reinterpret_cast<double2*>(region + P.o_RC);
      r.ng = reinterpret_cast<const int*>(region + P.o_ng);
      r.trmap = reinterpret_cast<const int*>(region + P.o_trmap);
      r.ng_max = P.ng_max;
      r.nv = P.nv;
      r.nc = P.nc;
    }
  }
  cp(B.o_pdx, ax.data(), nsys * sizeof(PdArgs));
  cp(B.o_pdd, ad.data(), 2 * nsys * sizeof(PdArgs));
  cp(B.o_jx, B.jx.data(), B.jx.size() * sizeof(PdJob));
  cp(B.o_xt, B.xt.data(), B.xt.size() * sizeof(HTile));
  cp(B.o_mt, B.mt.data(), B.mt.size() * sizeof(HTile));
  cp(B.o_tra, ta.data(), ta.size() * sizeof(TrArgs));
  std::vector<GemmArgs> ga(nsys);
  for (size_t c = 0; c < B.C.size(); ++c) {
    const BatchChunk& K = B.C[c];
    for (int i = 0; i < nsys; ++i) {
      ga[i] = gemm_args(B.P[i], &sys[i], ws + B.base[i], (int)c);
      ga[i].w_head_fp64 = precision != BSE_FP64;  // mixed: the q = 0 head of W is added in FP64
    }
    cp(K.o_gargs, ga.data(), nsys * sizeof(GemmArgs));
    cp(K.o_jd, K.jd.data(), K.jd.size() * sizeof(PdJob));
    cp(K.o_fill, K.fill.data(), K.fill.size() * sizeof(int4));
    cp(K.o_s1, K.s1.data(), K.s1.size() * sizeof(S1Tile));
    cp(K.o_d2off, K.d2off.data(), K.d2off.size() * sizeof(int));
    cp(K.o_dwt, K.dwt.data(), K.dwt.size() * sizeof(int4));
    cp(K.o_rvt, K.rvt.data(), K.rvt.size() * sizeof(int4));
  }
  std::vector<char> tb;
  for (int i = 0; i < nsys; ++i) {
    tb.assign(B.P[i].tables, 0);
    put_tables(B.P[i], tb, 0);
    cp(at[i], tb.data(), tb.size());
  }
  HIP_TRY(hipMemcpyAsync(ws, buf, B.o_cnt, hipMemcpyHostToDevice, st));
  for (int i = 0; i < nsys; ++i)
    HIP_TRY(hipMemcpyAsync(ws + B.base[i], buf + at[i], B.P[i].tables, hipMemcpyHostToDevice, st));
  return staging_release(st);
}

// Workgroups of a persistent pair-density launch: wg_per_cu per CU, fewer if
// the LDS footprint allows fewer, a multiple of 8.
int persistent_grid(size_t lds, int njobs, int wg_per_cu) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  const int per_cu = std::max(1, std::min(wg_per_cu, (int)((160 * 1024) / std::max<size_t>(lds, 1))));
  int g = std::max(kXcds, (cus * per_cu) / kXcds * kXcds);
  return std::min(g, std::max(njobs, kXcds));
}

// One pair-density launch over the batch: kind 0 the exchange densities (every
// k), kind 1 the valence and conduction densities of the pairs of chunk c.
int run_pd(const Batch& B, char* ws, int kind, int c, const Tune& tn, hipStream_t st) {
  const std::vector<PdJob>& jobs = kind == 0 ? B.jx : B.C[c].jd;
  const size_t o_args = kind == 0 ? B.o_pdx : B.o_pdd;
  const size_t o_jobs = kind == 0 ? B.o_jx : B.C[c].o_jd;
  if (jobs.empty()) return BSE_OK;
  PdBatch b{};
  b.sys = reinterpret_cast<const PdArgs*>(ws + o_args);
  b.jobs = reinterpret_cast<const PdJob*>(ws + o_jobs);
  b.njobs = (int)jobs.size();
  b.persist = tn.persist;
  b.cnt = reinterpret_cast<unsigned*>(ws + B.o_cnt) + (size_t)kind * kXcds * kQueueStride;
  const int stage_id = kind == 0 ? BSE_STAGE_PD_EXCH : BSE_STAGE_PD_VV;
  const bool f32 = B.pd32 && kind != 0;
  const size_t lds = f32 ? B.lds32 : B.lds;
  const int f32_planes = f32 ? B.np32 : 0;
  const int grid = tn.persist ? persistent_grid(lds, b.njobs, tn.wg_per_cu) : b.njobs;
  if (tn.persist) HIP_TRY(launch_zero_u32(b.cnt, kXcds * kQueueStride, st));
  HIP_TRY(stage(stage_id, st, [&] {
    return launch_pair_density(b, B.N2, B.N3, B.ng_max, lds, grid, kind == 0, f32_planes, st);
  }));
  return BSE_OK;
}

// Pair densities of the time-reversal images of chunk c (kind 1 vv, 2 cc),
// after the pair-density launch of the same kind.
// kind 1, 2: time-reversal images (valence, conduction rows); kind 3: the
// coupling block's (c, v') rows from the reversed pairs' (v, c') rows.
int run_tr_fill(const Batch& B, char* ws, int kind, int c, hipStream_t st) {
  if (!(kind == 3 ? B.cswap : B.tr) || kind == 0 || B.C[c].fill.empty()) return BSE_OK;
  HIP_TRY(stage(BSE_STAGE_TR_FILL, st, [&] {
    return launch_tr_fill(reinterpret_cast<const TrArgs*>(ws + B.o_tra),
                          reinterpret_cast<const int4*>(ws + B.C[c].o_fill), (int)B.C[c].fill.size(), kind, st);
  }));
  return BSE_OK;
}

// Wave functions in the pair-density frame, for systems whose axes are rotated.
int rotate_if_needed(const Plan& P, const bse_system& s, char* region, hipStream_t st) {
  if (!P.rot) return BSE_OK;
  HIP_TRY(stage(BSE_STAGE_ROTATE, st, [&] {
    return launch_rotate_axes(reinterpret_cast<const double2*>(s.u), reinterpret_cast<double2*>(region + P.o_ut),
                              (long long)P.nk * P.nb, s.grid[0], s.grid[1], s.grid[2], st);
  }));
  return BSE_OK;
}

// Wave functions in the form the pair-density launches read: rotated into the
// frame where needed, and the FP32 copy for FP32 pair densities.
int prepare_u(const Batch& B, const bse_system* sys, char* ws, hipStream_t st) {
  for (size_t i = 0; i < B.P.size(); ++i) {
    const Plan& P = B.P[i];
    char* region = ws + B.base[i];
    int rc = rotate_if_needed(P, sys[i], region, st);
    if (rc) return rc;
    if (!B.pd32) continue;
    const double2* src =
        P.rot ? reinterpret_cast<const double2*>(region + P.o_ut) : reinterpret_cast<const double2*>(sys[i].u);
    HIP_TRY(stage(BSE_STAGE_TO_F32, st, [&] {
      return launch_to_f32(src, reinterpret_cast<float2*>(region + P.o_u32), (size_t)P.nk * P.nb * P.N1 * P.N2 * P.N3,
                           st);
    }));
  }
  return BSE_OK;
}

// The forward build of every system of the batch, all on `st`: the exchange
// densities and the exchange term once, then per chunk the valence and
// conduction densities and the two stages of the direct term (one launch per
// stage over all systems), then the mirror.
// Mixed precisions: W of every system split (and unfolded through its maps)
// once per build, the B operand of the first direct-term contraction.
int split_w_all(const Batch& B, const bse_system* sys, int precision, char* ws, hipStream_t st) {
  if (precision == BSE_FP64) return BSE_OK;
  for (size_t i = 0; i < B.P.size(); ++i) {
    const Plan& P = B.P[i];
    char* region = ws + B.base[i];
    HIP_TRY(stage(BSE_STAGE_SPLIT_W, st, [&] {
      return launch_split_w(reinterpret_cast<const double2*>(sys[i].W), reinterpret_cast<const int*>(region + P.o_ng),
                            P.nirr ? reinterpret_cast<const int*>(region + P.o_wsrc) : nullptr,
                            P.nirr ? reinterpret_cast<const int*>(region + P.o_wmap) : nullptr, P.nk, P.ng_max,
                            P.kpad, 1, precision, region + P.o_Ws, st);
    }));
  }
  return BSE_OK;
}

// Mixed precisions: the valence pair-density rows of chunk c split once, the A
// operand of the first direct-term contraction.
int split_rv_chunk(const Batch& B, int precision, char* ws, int c, hipStream_t st) {
  if (precision == BSE_FP64) return BSE_OK;
  for (size_t i = 0; i < B.P.size(); ++i) {
    const Plan& P = B.P[i];
    if (c >= (int)P.ch.size()) continue;
    char* region = ws + B.base[i];
    HIP_TRY(stage(BSE_STAGE_SPLIT_W, st, [&] {
      return launch_split_rv(reinterpret_cast<const double2*>(region + P.o_RV),
                             reinterpret_cast<const int4*>(region + P.o_pairs) + P.ch[c].p0,
                             reinterpret_cast<const int*>(region + P.o_ng), (size_t)P.ch[c].np * P.rv_rows,
                             P.rv_rows, P.ng_max, P.kpad, precision, region + P.o_RVs, st);
    }));
  }
  return BSE_OK;
}

int run_build(const Batch& B, const bse_system* sys, int precision, const Tune& tn, char* ws, hipStream_t st) {
  const int nsys = (int)B.P.size();
  int rc = upload_batch(B, sys, precision, ws, st);
  if (rc) return rc;
  for (int i = 0; i < nsys; ++i) {
    const Plan& P = B.P[i];
    double* vs = reinterpret_cast<double*>(ws + B.base[i] + P.o_vs);
    HIP_TRY(stage(BSE_STAGE_VSCALE, st,
                  [&] { return launch_vscale(sys[i].vx, P.ng[P.qexc], P.ng_max, P.g0x, vs, st); }));
  }
  if ((rc = prepare_u(B, sys, ws, st))) return rc;
  if ((rc = split_w_all(B, sys, precision, ws, st))) return rc;
  const GemmArgs* g0 = reinterpret_cast<const GemmArgs*>(ws + B.C[0].o_gargs);
  const HTile* xt = reinterpret_cast<const HTile*>(ws + B.o_xt);
  const HTile* mt = reinterpret_cast<const HTile*>(ws + B.o_mt);
  if ((rc = run_pd(B, ws, 0, 0, tn, st))) return rc;
  for (int i = 0; i < nsys; ++i) {  // coupling block: the h-e exchange rows from the e-h ones
    const Plan& P = B.P[i];
    if (!P.coupling) continue;
    char* region = ws + B.base[i];
    HIP_TRY(launch_xbar(reinterpret_cast<const double2*>(region + P.o_X), reinterpret_cast<const int*>(region + P.o_inv0),
                        P.ns, P.ng[0], P.ng_max, reinterpret_cast<double2*>(region + P.o_Xb), st));
  }
  HIP_TRY(stage(BSE_STAGE_EXCHANGE, st, [&] { return launch_exchange(g0, xt, (int)B.xt.size(), precision, st); }));
  for (int c = 0; c < (int)B.C.size(); ++c) {
    const BatchChunk& K = B.C[c];
    const GemmArgs* gs = reinterpret_cast<const GemmArgs*>(ws + K.o_gargs);
    if ((rc = run_pd(B, ws, 1, c, tn, st)) || (rc = run_tr_fill(B, ws, 1, c, st)) ||
        (rc = run_tr_fill(B, ws, 2, c, st)) || (rc = run_tr_fill(B, ws, 3, c, st)))
      return rc;
    if ((rc = split_rv_chunk(B, precision, ws, c, st))) return rc;
    const S1Tile* s1 = reinterpret_cast<const S1Tile*>(ws + K.o_s1);
    const int* d2off = reinterpret_cast<const int*>(ws + K.o_d2off);
    HIP_TRY(stage(BSE_STAGE_DIRECT1, st,
                  [&] {
                    return launch_direct_s1(gs, s1, (int)K.s1.size(), precision, B.mapped ? 1 : 0, B.s1_rows, st);
                  }));
    HIP_TRY(stage(BSE_STAGE_DIRECT2, st, [&] { return launch_direct_s2(gs, d2off, nsys, K.d2n, st); }));
  }
  HIP_TRY(stage(BSE_STAGE_MIRROR, st, [&] { return launch_mirror(g0, mt, (int)B.mt.size(), st); }));
  return BSE_OK;
}

// ------------------------------------------------------------ screening

// Plan of bse_screening: chunks of q whose pair densities (2 nv nc rows per
// k) fit the chunk budget, their jobs, pair table and HERK tiles.  The q
// points are every q of the mesh, or (nirr > 0) the irreducible ones: output
// matrix (slot) i is W at qof[i].
struct ScrPlan {
  Plan G;                               // geometry of the system
  std::vector<int> qof;                 // q of each output slot
  std::vector<std::vector<int>> qs;     // q of each chunk
  std::vector<std::vector<PdJob>> jobs; // per chunk, dispatch order
  std::vector<std::vector<int4>> pk;    // per chunk: (k, k + q, q, -) per (q_local, k)
  std::vector<std::vector<int4>> tiles; // per chunk: (slot, row tile, column tile, q_local)
  // the empty x occupied rows gathered from the partner q's occupied x empty rows:
  // per chunk (destination row base, source row base, q, -), rows of Y
  bool gather = false;
  std::vector<std::vector<int4>> fill;
  // HERK slices per chunk (a chunk of few q splits its row sums to fill the
  // GPU) and the slot of each q_local
  std::vector<int> nsplit;
  std::vector<std::vector<int>> cslot;
  size_t o_part = 0;
  std::vector<size_t> o_cslot;
  int max_part_q = 0, max_split = 1;
  size_t o_gpack = 0, o_ng = 0, o_vq = 0, o_args = 0, o_ut = 0, o_Y = 0, o_qof = 0, o_trmap = 0, total = 0;
  std::vector<size_t> o_jobs, o_pk, o_tiles, o_fill;
  size_t tables = 0;
  int maxq = 0;                         // q per chunk, largest
};

int make_screening_plan(const bse_system* s, ScrPlan& S) {
  int rc = make_geometry(s, S.G, false);
  if (rc) return rc;
  const Plan& P = S.G;
  const int nk = P.nk, nv = P.nv, nc = P.nc;
  const size_t rows_q = (size_t)nk * 2 * nv * nc;
  const size_t bytes_q = rows_q * P.ng_max * sizeof(double2);
  if (rows_q * P.ng_max >= (size_t(1) << 31)) return fail(BSE_ERR_SHAPE, "pair densities of one q too large");
  if (P.ng_max > 1024) return fail(BSE_ERR_SHAPE, "ng_max above 1024");
  // output slots: every q, or the q that maps to source matrix i by the identity
  // (not conjugated; the lowest such q)
  S.qof.clear();
  if (P.nirr == 0) {
    for (int q = 0; q < nk; ++q) S.qof.push_back(q);
  } else {
    for (int i = 0; i < P.nirr; ++i) {
      int found = -1;
      for (int q = 0; q < nk && found < 0; ++q) {
        if (P.wsrc[2 * q] != i || P.wsrc[2 * q + 1] != 0) continue;
        bool ident = true;
        for (int g = 0; g < P.ng[q] && ident; ++g) ident = P.wmap[(size_t)q * P.ng_max + g] == g;
        if (ident) found = q;
      }
      if (found < 0)
        return fail(BSE_ERR_SHAPE, "no q maps to W matrix %d by the identity (its irreducible point is unknown)", i);
      S.qof.push_back(found);
    }
  }
  const int nq = (int)S.qof.size();
  const int per_chunk = (int)std::max<size_t>(1, std::min<size_t>(nq, g_chunk_budget.load() / std::max<size_t>(bytes_q, 1)));
  // every q of the mesh with spheres closed under G -> t - G: n_{ck, v k+q}(G) =
  // conj(n_{v k+q, c k}(t - G)) (-q = qbar + t), the occupied x empty density of
  // the pair (k + q, k), whose transfer is qbar; so q and qbar share a chunk and
  // only occupied x empty pairs are transformed
  S.gather = P.nirr == 0 && P.tr_closed;
  std::vector<std::vector<int>> chunk_slots(1);
  {
    std::vector<int> slot_of(nk, -1);
    for (int i = 0; i < nq; ++i) slot_of[S.qof[i]] = i;
    std::vector<char> placed(nq, 0);
    for (int i = 0; i < nq; ++i) {
      if (placed[i]) continue;
      std::vector<int> unit{i};
      placed[i] = 1;
      if (S.gather) {
        const int j = slot_of[P.qbar[S.qof[i]]];
        if (j != i) {
          unit.push_back(j);
          placed[j] = 1;
        }
      }
      if (!chunk_slots.back().empty() && (int)(chunk_slots.back().size() + unit.size()) > per_chunk)
        chunk_slots.emplace_back();
      chunk_slots.back().insert(chunk_slots.back().end(), unit.begin(), unit.end());
    }
  }
  const int nchunk = (int)chunk_slots.size();
  S.maxq = 0;
  for (const auto& cs : chunk_slots) S.maxq = std::max(S.maxq, (int)cs.size());
  S.qs.assign(nchunk, {});
  S.jobs.assign(nchunk, {});
  S.pk.assign(nchunk, {});
  S.tiles.assign(nchunk, {});
  S.fill.assign(nchunk, {});
  const int* n = s->kmesh;
  const int T2 = (P.ng_max + 63) / 64;
  for (int c = 0; c < nchunk; ++c) {
    std::vector<PdJob> jobs;
    std::vector<int> ql_of(nk, -1);  // position of each q in the chunk
    for (size_t i = 0; i < chunk_slots[c].size(); ++i) ql_of[S.qof[chunk_slots[c][i]]] = (int)i;
    for (int slot : chunk_slots[c]) {
      const int q = S.qof[slot];
      const int ql = (int)S.qs[c].size();
      S.qs[c].push_back(q);
      const int qv[3] = {q / (n[1] * n[2]), (q / n[2]) % n[1], q % n[2]};
      for (int k = 0; k < nk; ++k) {
        const int kv[3] = {k / (n[1] * n[2]), (k / n[2]) % n[1], k % n[2]};
        const int kq = (((kv[0] + qv[0]) % n[0]) * n[1] + (kv[1] + qv[1]) % n[1]) * n[2] + (kv[2] + qv[2]) % n[2];
        int iq, m0[3];
        fold(s->kmesh, k, kq, iq, m0);
        const int m0p = pack_m(m0[P.ax[0]], m0[P.ax[1]], m0[P.ax[2]]);
        const int row0 = (ql * nk + k) * 2 * nv * nc;
        // occupied at k x empty at k + q, then empty at k x occupied at k + q (or
        // gathered: the first rows of the pair (k + q, k) of qbar)
        jobs.push_back(PdJob{k, kq, m0p, iq, 0, nv, nv | (nc << 8), row0});
        if (S.gather)
          S.fill[c].push_back(make_int4(row0 + nv * nc, (ql_of[P.qbar[q]] * nk + kq) * 2 * nv * nc, q, 0));
        else
          jobs.push_back(PdJob{k, kq, m0p, iq, nv, 0, nc | (nv << 8), row0 + nv * nc});
        S.pk[c].push_back(make_int4(k, kq, q, 0));
      }
      for (int i = 0; i < T2; ++i)  // eps is Hermitian: the tiles on and above the diagonal
        for (int j = i; j < T2; ++j) S.tiles[c].push_back(make_int4(slot, i, j, ql));
    }
    S.jobs[c] = dispatch_order(std::move(jobs), Tune{}.ktile);
  }
  // the HERK runs three workgroups per CU; a call with fewer tiles than about
  // two rounds of that splits every row sum into slices (at most 8).  The
  // count follows the whole call, not its chunks, so that W does not depend
  // on the chunk budget.
  constexpr int kHerkSlots = 3 * 256;
  size_t nt_all = 0;
  for (int c = 0; c < nchunk; ++c) nt_all += S.tiles[c].size();
  const int ns = nt_all >= 2 * kHerkSlots / 3
                     ? 1
                     : (int)std::min<size_t>(8, (kHerkSlots + nt_all - 1) / std::max<size_t>(nt_all, 1));
  S.nsplit.assign(nchunk, 1);
  S.cslot.assign(nchunk, {});
  S.max_part_q = 0;
  S.max_split = 1;
  for (int c = 0; c < nchunk; ++c) {
    S.cslot[c] = chunk_slots[c];
    const int nt = (int)S.tiles[c].size();
    S.nsplit[c] = ns;
    if (ns > 1) {
      std::vector<int4> t;
      t.reserve((size_t)nt * ns);
      for (int sl = 0; sl < ns; ++sl)
        for (const int4& x : S.tiles[c]) t.push_back(make_int4(x.x, x.y | (sl << 8), x.z, x.w));
      S.tiles[c].swap(t);
      S.max_split = std::max(S.max_split, ns);
      S.max_part_q = std::max(S.max_part_q, (int)chunk_slots[c].size());
    }
  }
  // workspace: tables, the rotated wave functions, the pair densities of a chunk
  size_t o = 0;
  auto put = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  S.o_gpack = put(P.gpack.size() * sizeof(int));
  S.o_ng = put(P.ng.size() * sizeof(int));
  S.o_args = put(sizeof(PdArgs));
  S.o_qof = put(S.qof.size() * sizeof(int));
  S.o_trmap = put(S.gather ? P.trmap.size() * sizeof(int) : 0);
  S.o_jobs.resize(nchunk);
  S.o_pk.resize(nchunk);
  S.o_tiles.resize(nchunk);
  S.o_fill.resize(nchunk);
  S.o_cslot.resize(nchunk);
  for (int c = 0; c < nchunk; ++c) {
    S.o_jobs[c] = put(S.jobs[c].size() * sizeof(PdJob));
    S.o_pk[c] = put(S.pk[c].size() * sizeof(int4));
    S.o_tiles[c] = put(S.tiles[c].size() * sizeof(int4));
    S.o_fill[c] = put(S.fill[c].size() * sizeof(int4));
    S.o_cslot[c] = put(S.cslot[c].size() * sizeof(int));
  }
  S.tables = o;
  if (P.rot) S.o_ut = put((size_t)P.nk * P.nb * P.N1 * P.N2 * P.N3 * sizeof(double2));
  S.o_Y = put((size_t)S.maxq * bytes_q);
  S.o_part = put(S.max_split > 1 ? (size_t)S.max_split * S.max_part_q * P.ng_max * P.ng_max * sizeof(double2) : 0);
  S.total = o;
  return BSE_OK;
}

// ------------------------------------------------------------ validation

// BSE_VALIDATE: scans every system's inputs and waits for the result.
int validate(const Batch& B, const bse_system* sys, char* ws, hipStream_t st) {
  unsigned* bad = reinterpret_cast<unsigned*>(ws + B.o_cnt + kCntBytes);
  unsigned long long* wstat = reinterpret_cast<unsigned long long*>(ws + B.o_cnt + kCntBytes + 32);
  for (size_t i = 0; i < B.P.size(); ++i) {
    const Plan& P = B.P[i];
    const bse_system& s = sys[i];
    char* r = ws + B.base[i];
    HIP_TRY(launch_zero_u32(bad, 8 + 16, st));  // the 3 flags and the 64-bit maxima after them
    // W of the irreducible q points: its nirr matrices on their own sphere sizes; time
    // reversal then holds by construction of the maps
    HIP_TRY(launch_validate(s.u, (size_t)P.nk * P.nb * P.N1 * P.N2 * P.N3 * 2, s.eps, (size_t)P.nk * P.nb, s.vx,
                            (size_t)P.ng[P.qexc], reinterpret_cast<const double2*>(s.W),
                            reinterpret_cast<const int*>(r + (P.nirr ? P.o_ngirr : P.o_ng)),
                            reinterpret_cast<const int*>(r + P.o_qbar), reinterpret_cast<const int*>(r + P.o_trmap),
                            P.nirr ? P.nirr : P.nk, P.ng_max, P.tr_closed && !P.nirr ? 1 : 0, bad, wstat, st));
    unsigned hb[3];
    unsigned long long hw[3];
    HIP_TRY(hipMemcpyAsync(hb, bad, sizeof hb, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hw, wstat, sizeof hw, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double w[3];
    std::memcpy(w, hw, sizeof w);
    static const char* names[3] = {"u", "eps", "vx"};
    for (int k = 0; k < 3; ++k)
      if (hb[k]) return fail(BSE_ERR_NONFINITE, "system %zu: non-finite value in %s", i, names[k]);
    if (!std::isfinite(w[0])) return fail(BSE_ERR_NONFINITE, "system %zu: non-finite value in W", i);
    const double tol = 1e-10 * w[0];
    if (w[1] > tol)
      return fail(BSE_ERR_NOT_HERMITIAN, "system %zu: W(q) not Hermitian (deviation %.3e, max |W| %.3e)", i, w[1], w[0]);
    if (w[2] > tol)
      return fail(BSE_ERR_NOT_HERMITIAN, "system %zu: W violates time reversal (deviation %.3e, max |W| %.3e)", i, w[2],
                  w[0]);
    if (B.tr) {
      HIP_TRY(launch_validate_u_tr(reinterpret_cast<const double2*>(s.u), reinterpret_cast<const int*>(r + P.o_ktr),
                                   P.nk, P.nb, s.grid[0], s.grid[1], s.grid[2], wstat, st));
      unsigned long long hu[2];
      HIP_TRY(hipMemcpyAsync(hu, wstat + 3, sizeof hu, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      double du[2];
      std::memcpy(du, hu, sizeof du);
      if (!(du[1] <= 1e-10 * du[0]))
        return fail(BSE_ERR_NOT_SYMMETRIC, "system %zu: u violates time reversal (deviation %.3e, max |u| %.3e)", i,
                    du[1], du[0]);
    }
  }
  return BSE_OK;
}

// ------------------------------------------------------------ autotuning

// Tuning cache: one line per batch signature,
//   {"key": "<signature>", "persist": P, "ktile": T, "wg_per_cu": W, "pd_ms": M, "s1_rows": R, "s1_ms": S,
//    "order": O}
bool cache_lookup(const char* path, const std::string& key, Tune& out) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[4096];
  bool hit = false;
  const std::string want = "{\"key\": \"" + key + "\",";
  while (fgets(line, sizeof line, f)) {
    if (std::strncmp(line, want.c_str(), want.size()) != 0) continue;
    Tune t;
    float ms = 0.f, s1ms = 0.f;
    if (sscanf(line + want.size(),
               " \"persist\": %d, \"ktile\": %d, \"wg_per_cu\": %d, \"pd_ms\": %f, \"s1_rows\": %d, \"s1_ms\": %f, "
               "\"order\": %d",
               &t.persist, &t.ktile, &t.wg_per_cu, &ms, &t.s1_rows, &s1ms, &t.order) == 7 &&
        (t.persist == 0 || t.persist == 1) && t.ktile >= 1 && t.ktile <= 1024 && t.wg_per_cu >= 1 && t.wg_per_cu <= 8 &&
        (t.s1_rows == 64 || t.s1_rows == 128) && (t.order >= 0 && t.order <= 2)) {
      t.pd_ms = ms;
      t.s1_ms = s1ms;
      out = t;
      hit = true;  // the last matching line wins
    }
  }
  fclose(f);
  return hit;
}

void cache_store(const char* path, const std::string& key, const Tune& t) {
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "{\"key\": \"%s\", \"persist\": %d, \"ktile\": %d, \"wg_per_cu\": %d, \"pd_ms\": %.9g, \"s1_rows\": %d, "
          "\"s1_ms\": %.9g, \"order\": %d}\n", key.c_str(), t.persist, t.ktile, t.wg_per_cu, (double)t.pd_ms, t.s1_rows,
          (double)t.s1_ms, t.order);
  fclose(f);
}

// Candidates timed by the last autotuning on this thread (reported by
// bse_autotune_last).
thread_local std::vector<Tune> g_tried;

// Times the valence and conduction pair-density launch (the dominant stage) of the
// batch's first chunk under each candidate dispatch and keeps the fastest.
int autotune(const bse_system* sys, int nsys, int precision, bool pd32, const char* cache, Tune& best, char* ws,
             size_t ws_bytes, hipStream_t st) {
  Batch B0;
  BatchOpts opt;
  opt.pd32 = pd32;
  opt.mixed = precision != BSE_FP64;
  int rc = make_batch(sys, nsys, Tune{}, opt, B0);
  if (rc) return rc;
  const std::string key = batch_key(B0.P, precision, B0.pd32);
  if (cache_lookup(cache, key, best)) {
    set_tune(key, best);
    return BSE_OK;
  }
  if (ws_bytes < B0.total) return fail(BSE_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, B0.total);
  std::vector<Tune> cand;
  for (int od : {0, 2, 1})
    for (int kt : {4, 8, 16}) {
      Tune t;
      t.ktile = kt;
      t.order = od;
      cand.push_back(t);
    }
  for (int w : {1, 2, 3, 4}) {
    Tune t;
    t.persist = 1;
    t.wg_per_cu = w;
    cand.push_back(t);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  best = Tune{};
  best.pd_ms = -1.f;
  g_tried.clear();
  for (const Tune& c : cand) {
    Batch B;
    if ((rc = make_batch(sys, nsys, c, opt, B))) break;
    if ((rc = upload_batch(B, sys, precision, ws, st))) break;
    if ((rc = prepare_u(B, sys, ws, st))) break;
    float ms = 0.f;
    hipError_t e = hipSuccess;
    // the first run warms caches and code; the best of the other two counts
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
      float m = 0.f;
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      if (e == hipSuccess && (rc = run_pd(B, ws, 1, 0, c, st))) break;
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&m, e0, e1);
      if (rep == 1 || (rep == 2 && m < ms)) ms = m;
    }
    if (rc) break;
    if (e != hipSuccess) {
      rc = fail(BSE_ERR_HIP, "autotune timing: %s", hipGetErrorString(e));
      break;
    }
    Tune rec = c;
    rec.pd_ms = ms;
    g_tried.push_back(rec);
    if (best.pd_ms < 0.f || ms < best.pd_ms) best = rec;
  }
  // the first direct-term contraction of the first chunk (its operands made by
  // the chosen dispatch) with 64- and 128-row tiles
  if (!rc) {
    float s1_best = -1.f;
    int rows_best = 64;
    for (int rows : {64, 128}) {
      if (rows == 128 && precision != BSE_BF16X3) continue;  // FP64 and FP32 parts: 64-row tiles only
      Tune c = best;
      c.s1_rows = rows;
      Batch B;
      if ((rc = make_batch(sys, nsys, c, opt, B))) break;
      if ((rc = upload_batch(B, sys, precision, ws, st)) || (rc = prepare_u(B, sys, ws, st)) ||
          (rc = split_w_all(B, sys, precision, ws, st)) || (rc = run_pd(B, ws, 1, 0, c, st)) ||
          (rc = split_rv_chunk(B, precision, ws, 0, st)))
        break;
      const BatchChunk& K = B.C[0];
      const GemmArgs* gs = reinterpret_cast<const GemmArgs*>(ws + K.o_gargs);
      const S1Tile* s1 = reinterpret_cast<const S1Tile*>(ws + K.o_s1);
      float ms = 0.f;
      hipError_t e = hipSuccess;
      for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
        float m = 0.f;
        e = hipEventRecord(e0, st);
        if (e == hipSuccess) e = launch_direct_s1(gs, s1, (int)K.s1.size(), precision, B.mapped ? 1 : 0, rows, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&m, e0, e1);
        if (rep == 1 || (rep == 2 && m < ms)) ms = m;
      }
      if (e != hipSuccess) {
        rc = fail(BSE_ERR_HIP, "autotune timing: %s", hipGetErrorString(e));
        break;
      }
      Tune rec = c;
      rec.s1_ms = ms;
      g_tried.push_back(rec);
      if (s1_best < 0.f || ms < s1_best) {
        s1_best = ms;
        rows_best = rows;
      }
    }
    best.s1_rows = rows_best;
    best.s1_ms = s1_best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  set_tune(key, best);
  cache_store(cache, key, best);
  return BSE_OK;
}

// Reciprocal vectors b = 2 pi A^-T (rows) of the cell A (rows a1, a2, a3) and
// the checks of the full-grid FFT the k.p matrix elements need.
int grad_setup(const bse_system* sys, const Plan& P, const double* cell, GradCell& bc) {
  if (!cell) return fail(BSE_ERR_INVALID_ARG, "cell is NULL (needed for the dipoles)");
  const int G1 = sys->grid[0], G2 = sys->grid[1], G3 = sys->grid[2];  // grid order, not the pair-density frame
  if (!fft_len_supported(G1) || !fft_len_supported(G2) || !fft_len_supported(G3))
    return fail(BSE_ERR_SHAPE, "grid (%d, %d, %d) has no full-grid FFT", G1, G2, G3);
  if (P.nc > 8) return fail(BSE_ERR_SHAPE, "dipoles support at most 8 conduction bands");
  const double* A = cell;
  const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                     A[2] * (A[3] * A[7] - A[4] * A[6]);
  if (!(std::fabs(det) > 0.0)) return fail(BSE_ERR_INVALID_ARG, "singular cell");
  const double tp = 6.283185307179586476925286766559 / det;
  // rows of 2 pi (A^-1)^T = 2 pi / det * cofactor rows
  bc.b[0][0] = tp * (A[4] * A[8] - A[5] * A[7]);
  bc.b[0][1] = tp * (A[5] * A[6] - A[3] * A[8]);
  bc.b[0][2] = tp * (A[3] * A[7] - A[4] * A[6]);
  bc.b[1][0] = tp * (A[2] * A[7] - A[1] * A[8]);
  bc.b[1][1] = tp * (A[0] * A[8] - A[2] * A[6]);
  bc.b[1][2] = tp * (A[1] * A[6] - A[0] * A[7]);
  bc.b[2][0] = tp * (A[1] * A[5] - A[2] * A[4]);
  bc.b[2][1] = tp * (A[2] * A[3] - A[0] * A[5]);
  bc.b[2][2] = tp * (A[0] * A[4] - A[1] * A[3]);
  return BSE_OK;
}

// Arguments of bse_spectrum (shared with its variant without workspace).
int spectrum_args(int ns, int nlam, const double* E, const double* A, const double* d, int nq, int nk,
                  double omega_cell, int nw, double eta_eV, double* eps2) {
  if (ns < 1 || nlam < 1 || nlam > ns || nw < 1) return fail(BSE_ERR_INVALID_ARG, "bad sizes");
  if (nq < 1 || nk < 1) return fail(BSE_ERR_INVALID_ARG, "nq and nk must be positive");
  if (!E || !A || !d || !eps2) return fail(BSE_ERR_INVALID_ARG, "NULL pointer");
  if (!(eta_eV > 0.0)) return fail(BSE_ERR_INVALID_ARG, "eta must be positive");
  if (!(omega_cell > 0.0)) return fail(BSE_ERR_INVALID_ARG, "omega_cell must be positive");
  return BSE_OK;
}

// The adjoint for a system with W at every q.
int backward_impl(const bse_system* sys, const double* dH, double* dW, double* deps, double* dX, double* drho_vv,
                  double* drho_cc, int precision, int flags, void* ws, size_t ws_bytes, hipStream_t st) {
  if (!dH || !ws) return fail(BSE_ERR_INVALID_ARG, "dH / ws is NULL");
  if (precision < BSE_FP64 || precision > BSE_BF16X3) return fail(BSE_ERR_INVALID_ARG, "bad precision %d", precision);
  if (flags & ~(BSE_PROJECT_DW | BSE_TIME_REVERSAL | BSE_FP32_PAIRDENS))
    return fail(BSE_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  if ((flags & BSE_FP32_PAIRDENS) && precision == BSE_FP64)
    return fail(BSE_ERR_INVALID_ARG, "BSE_FP32_PAIRDENS needs a mixed precision (split-FP32 or BF16x3)");
  if (sys->qexc != 0 && (dX || drho_vv || drho_cc))
    return fail(BSE_ERR_UNSUPPORTED, "the gradients of the pair densities need exciton momentum Q = 0");
  const bool project = (flags & BSE_PROJECT_DW) != 0;
  Batch B;
  BatchOpts opt;
  opt.backward = true;
  opt.project = project && dW;
  opt.tr = (flags & BSE_TIME_REVERSAL) != 0;
  opt.pd32 = (flags & BSE_FP32_PAIRDENS) != 0;
  int rc = make_batch(sys, 1, Tune{}, opt, B);
  if (rc) return rc;
  const Plan& P = B.P[0];
  if (ws_bytes < B.total) return fail(BSE_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, B.total);
  if (project && !P.tr_closed)
    return fail(BSE_ERR_NOT_HERMITIAN, "G spheres are not closed under time reversal; cannot project dW");
  char* w = static_cast<char*>(ws);
  if ((rc = upload_batch(B, sys, BSE_FP64, w, st))) return rc;
  char* r = w + B.base[0];
  if ((rc = prepare_u(B, sys, w, st))) return rc;
  AdjArgs g{};
  g.dH = reinterpret_cast<const double2*>(dH);
  g.RV = reinterpret_cast<const double2*>(r + P.o_RV);
  g.RC = reinterpret_cast<const double2*>(r + P.o_RC);
  g.T = reinterpret_cast<double2*>(r + P.o_Z);
  g.dWfinal = reinterpret_cast<double2*>(dW);
  g.dWout = dW ? (project ? reinterpret_cast<double2*>(r + P.o_dWraw) : reinterpret_cast<double2*>(dW)) : nullptr;
  g.deps = deps;
  g.pairs = reinterpret_cast<const int4*>(r + P.o_pairs);
  g.ng = reinterpret_cast<const int*>(r + P.o_ng);
  g.qbar = reinterpret_cast<const int*>(r + P.o_qbar);
  g.trmap = reinterpret_cast<const int*>(r + P.o_trmap);
  g.nk = P.nk;
  g.nv = P.nv;
  g.nc = P.nc;
  g.ns = P.ns;
  g.ng_max = P.ng_max;
  g.cpref = 27.211386245988 / ((double)P.nk * sys->omega_cell);
  for (int d = 0; d < 3; ++d) g.kn[d] = sys->kmesh[d];
  g.qe[0] = P.qexc / (sys->kmesh[1] * sys->kmesh[2]);
  g.qe[1] = (P.qexc / sys->kmesh[2]) % sys->kmesh[1];
  g.qe[2] = P.qexc % sys->kmesh[2];
  g.Z = reinterpret_cast<const double2*>(r + P.o_Z);
  g.W = reinterpret_cast<const double2*>(sys->W);
  g.Xs = reinterpret_cast<const double2*>(r + P.o_X);
  g.vs = reinterpret_cast<const double*>(r + P.o_vs);
  g.plex = reinterpret_cast<const int*>(r + P.o_plex);
  g.ngx = P.ng[0];
  g.dX = reinterpret_cast<double2*>(dX);
  g.drv = reinterpret_cast<double2*>(drho_vv);
  g.drc = reinterpret_cast<double2*>(drho_cc);
  // the exchange densities (only for dX) and their gradient
  if (dX) {
    double* vs = reinterpret_cast<double*>(r + P.o_vs);
    HIP_TRY(launch_vscale(sys->vx, P.ng[P.qexc], P.ng_max, P.g0x, vs, st));
    if ((rc = run_pd(B, w, 0, 0, Tune{}, st))) return rc;
    HIP_TRY(launch_adj_dx(g, st));
  }
  if (g.dWout) HIP_TRY(launch_zero_f64(reinterpret_cast<double*>(g.dWout), (size_t)P.nk * P.ng_max * P.ng_max * 2, st));
  // per chunk: recompute the pair densities, then the chunk's share of every gradient
  for (int c = 0; c < (int)B.C.size(); ++c) {
    const BatchChunk& K = B.C[c];
    if ((rc = run_pd(B, w, 1, c, Tune{}, st)) || (rc = run_tr_fill(B, w, 1, c, st)) ||
        (rc = run_tr_fill(B, w, 2, c, st)))
      return rc;
    g.qstart = reinterpret_cast<const int*>(r + P.o_qs) + (size_t)c * (P.nk + 1);
    g.p0 = P.ch[c].p0;
    g.npairs = P.ch[c].np;
    g.dwtiles = reinterpret_cast<const int4*>(w + K.o_dwt);
    g.rvtiles = reinterpret_cast<const int4*>(w + K.o_rvt);
    if (drho_cc) {
      // Z = conj(rho_vv')^T W (the forward stage 1, FP64) into the Z area
      const GemmArgs* gs = reinterpret_cast<const GemmArgs*>(w + K.o_gargs);
      const S1Tile* s1 = reinterpret_cast<const S1Tile*>(w + K.o_s1);
      HIP_TRY(launch_direct_s1(gs, s1, (int)K.s1.size(), BSE_FP64, 0, B.s1_rows, st));
      HIP_TRY(launch_adj_drc(g, st));
    }
    // T (over the Z area), the chunk's share of dW
    HIP_TRY(launch_adjoint(g, precision, (int)K.dwt.size(), K.has_q0, st));
    if (drho_vv) HIP_TRY(launch_adj_drv(g, (int)K.rvt.size(), st));
  }
  HIP_TRY(launch_adjoint_finish(g, project, st));
  return BSE_OK;
}

// The backward with W at the irreducible q points runs the adjoint above on W
// unfolded into the workspace and folds dW back onto the nirr matrices.
// Workspace: [fold tables | unfolded W | dW at every q | the adjoint's own].
struct IrrBackward {
  Plan G;                       // geometry, with the validated maps
  std::vector<int> tab;         // wsrc [2 Nk], wmap, winv [Nk][ng_max], csr [nirr + 1], qlist [Nk], ngirr, ng
  size_t t_wsrc = 0, t_wmap = 0, t_winv = 0, t_csr = 0, t_qlist = 0, t_ngirr = 0, t_ng = 0;  // int offsets
  size_t o_Wf = 0, o_dWf = 0, extra = 0;
};

int plan_irr_backward(const bse_system* sys, bool want_dw, IrrBackward& R) {
  int rc = make_geometry(sys, R.G);
  if (rc) return rc;
  const Plan& P = R.G;
  const int nk = P.nk, ngm = P.ng_max, nirr = P.nirr;
  R.tab.clear();
  auto take = [&](size_t n) {
    const size_t at = R.tab.size();
    R.tab.resize(at + n, 0);
    return at;
  };
  R.t_wsrc = take(2 * (size_t)nk);
  R.t_wmap = take((size_t)nk * ngm);
  R.t_winv = take((size_t)nk * ngm);
  R.t_csr = take((size_t)nirr + 1);
  R.t_qlist = take(nk);
  R.t_ngirr = take(nirr);
  R.t_ng = take(nk);
  std::copy(P.wsrc.begin(), P.wsrc.end(), R.tab.begin() + R.t_wsrc);
  std::copy(P.wmap.begin(), P.wmap.end(), R.tab.begin() + R.t_wmap);
  for (int q = 0; q < nk; ++q)
    for (int g = 0; g < P.ng[q]; ++g) R.tab[R.t_winv + (size_t)q * ngm + P.wmap[(size_t)q * ngm + g]] = g;
  std::vector<int> cnt(nirr, 0);
  for (int q = 0; q < nk; ++q) cnt[P.wsrc[2 * q]]++;
  for (int i = 0; i < nirr; ++i) R.tab[R.t_csr + i + 1] = R.tab[R.t_csr + i] + cnt[i];
  std::vector<int> fillp(R.tab.begin() + R.t_csr, R.tab.begin() + R.t_csr + nirr);
  for (int q = 0; q < nk; ++q) R.tab[R.t_qlist + fillp[P.wsrc[2 * q]]++] = q;  // increasing q per source
  std::copy(P.ngirr.begin(), P.ngirr.end(), R.tab.begin() + R.t_ngirr);
  std::copy(P.ng.begin(), P.ng.end(), R.tab.begin() + R.t_ng);
  const size_t mat = (size_t)nk * ngm * ngm * sizeof(double2);
  R.o_Wf = align256(R.tab.size() * sizeof(int));
  R.o_dWf = align256(R.o_Wf + mat);
  R.extra = align256(R.o_dWf + (want_dw ? mat : 0));
  return BSE_OK;
}

// sys with W at every q in the unfolded area (the plan's view of the system).
bse_system unfolded_view(const bse_system* sys, const double* Wf) {
  bse_system s = *sys;
  s.nirr = 0;
  s.wsrc = nullptr;
  s.wmap = nullptr;
  s.W = Wf;
  return s;
}

}  // namespace

// Used by the variant of bse_spectrum without workspace (noalloc.hip).
namespace bse {
int api_fail(int code, const char* msg) { return fail(code, "%s", msg); }
int api_spectrum_args(int ns, int nlam, const double* E, const double* A, const double* d, int nq, int nk,
                      double omega_cell, int nw, double eta_eV, double* eps2) {
  return spectrum_args(ns, nlam, E, A, d, nq, nk, omega_cell, nw, eta_eV, eps2);
}
}  // namespace bse

// The beyond-TDA matrix: the resonant block by the Tamm-Dancoff build and
// the coupling block by the same stages over every ordered k pair, both
// written into H2 (row stride 2 NS), then the lower half.
int full_batches(const bse_system* sys, int precision, int flags, const Batch** BA, const Batch** BB) {
  if (!sys) return fail(BSE_ERR_INVALID_ARG, "system pointer is NULL");
  if (precision != BSE_FP64) return fail(BSE_ERR_UNSUPPORTED, "the beyond-TDA build is FP64 only");
  if (flags & ~(BSE_VALIDATE | BSE_PERSISTENT)) return fail(BSE_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  if (sys->qexc != 0) return fail(BSE_ERR_UNSUPPORTED, "the beyond-TDA build needs exciton momentum Q = 0");
  const long long ns = (long long)sys->kmesh[0] * sys->kmesh[1] * sys->kmesh[2] * sys->nv * sys->nc;
  if (ns < 1 || 2 * ns > (1LL << 20)) return fail(BSE_ERR_SHAPE, "2 NS = %lld out of range", 2 * ns);
  BatchOpts a;
  a.ldh = (int)(2 * ns);
  BatchOpts b = a;
  b.coupling = true;
  int rc = cached_batch(sys, 1, Tune{}, a, BA);
  if (!rc) rc = cached_batch(sys, 1, Tune{}, b, BB);
  return rc;
}

extern "C" {

size_t bse_workspace_size(const bse_system* sys, int nsys, int precision, int flags) {
  if (!sys || nsys < 1) return 0;
  // the forward build, with room for the time-reversal tables where the
  // spheres allow them; one system: the backward as well
  BatchOpts o;
  o.pd32 = (flags & BSE_FP32_PAIRDENS) != 0;
  o.mixed = precision != BSE_FP64;
  Batch B;
  if (make_batch(sys, nsys, Tune{}, o, B)) return 0;
  size_t total = B.total;
  const std::string keep = g_err;  // spheres without time reversal are no error here
  for (int pass = 0; pass < 3; ++pass) {
    BatchOpts x = o;
    x.tr = pass != 1;
    if (pass > 0) {
      if (nsys != 1) continue;
      x.backward = true;
      x.project = (flags & BSE_PROJECT_DW) != 0;
      x.mixed = false;  // the backward contracts unsplit operands
    }
    Batch Bx;
    if (pass > 0 && sys->nirr > 0) {  // the backward runs on W unfolded into the workspace
      IrrBackward R;
      if (plan_irr_backward(sys, true, R) != BSE_OK) continue;
      const bse_system s2 = unfolded_view(sys, sys->W);
      if (make_batch(&s2, 1, Tune{}, x, Bx) == BSE_OK) total = std::max(total, R.extra + Bx.total);
      continue;
    }
    if (make_batch(sys, nsys, Tune{}, x, Bx) == BSE_OK) total = std::max(total, Bx.total);
  }
  g_err = keep;
  return total;
}

int bse_pair_density(const bse_system* sys, int kind, const int* kpairs, int npairs, const double* cell,
                     double* out, void* ws, size_t ws_bytes, void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Plan P;
  int rc = make_geometry(sys, P);
  if (rc) return rc;
  if (!out || !ws) return fail(BSE_ERR_INVALID_ARG, "out / ws is NULL");
  std::vector<PdJob> jobs;
  if (kind == BSE_PD_EXCH) {
    jobs = P.jx;
  } else if (kind == BSE_PD_VV || kind == BSE_PD_CC) {
    if (!kpairs || npairs < 0) return fail(BSE_ERR_INVALID_ARG, "kpairs is NULL");
    const int nA = kind == BSE_PD_VV ? P.nv : P.nc, b0 = kind == BSE_PD_VV ? 0 : P.nv;
    for (int i = 0; i < npairs; ++i) {
      const int ka = kpairs[2 * i], kb = kpairs[2 * i + 1];
      if (ka < 0 || kb < 0 || ka >= P.nk || kb >= P.nk) return fail(BSE_ERR_INVALID_ARG, "k pair %d out of range", i);
      int iq, m0[3];
      fold(sys->kmesh, ka, kb, iq, m0);
      jobs.push_back(PdJob{ka, kb, pack_m(m0[P.ax[0]], m0[P.ax[1]], m0[P.ax[2]]), iq, b0, b0, nA | (nA << 8),
                           i * nA * nA});
    }
  } else if (kind == BSE_PD_DIPOLE) {
    GradCell bc;
    if ((rc = grad_setup(sys, P, cell, bc))) return rc;
    const size_t need = (size_t)P.nk * P.nb * P.N1 * P.N2 * P.N3 * sizeof(double2);
    if (ws_bytes < need) return fail(BSE_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    HIP_TRY(launch_grad(reinterpret_cast<const double2*>(sys->u), static_cast<double2*>(ws), P.nk, P.nb, P.nv, P.nc,
                        sys->grid[0], sys->grid[1], sys->grid[2], bc, reinterpret_cast<double2*>(out), st));
    return BSE_OK;
  } else {
    return fail(BSE_ERR_INVALID_ARG, "unknown kind %d", kind);
  }
  const size_t lds = pd_lds_bytes(P.N1, P.N2, P.N3, P.F[1], P.F[2], P.ng_max, 0);
  if (lds > 160 * 1024) return fail(BSE_ERR_SHAPE, "FFT window needs more than 160 KiB of LDS");
  jobs = dispatch_order(std::move(jobs), Tune{}.ktile);
  // tables: gpack, ng, the one system's arguments, jobs
  const size_t o_g = 0, o_n = align256(P.gpack.size() * sizeof(int));
  const size_t o_a = align256(o_n + P.ng.size() * sizeof(int));
  const size_t o_j = align256(o_a + sizeof(PdArgs));
  const size_t tab = align256(o_j + jobs.size() * sizeof(PdJob));
  const size_t ut_bytes = P.rot ? (size_t)P.nk * P.nb * P.N1 * P.N2 * P.N3 * sizeof(double2) : 0;
  const size_t need = tab + ut_bytes;  // tables, then the rotated wave functions
  if (ws_bytes < need) return fail(BSE_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  char* w = static_cast<char*>(ws);
  if (P.rot)
    HIP_TRY(launch_rotate_axes(reinterpret_cast<const double2*>(sys->u), reinterpret_cast<double2*>(w + tab),
                               (long long)P.nk * P.nb, sys->grid[0], sys->grid[1], sys->grid[2], st));
  PdArgs a{};
  a.u = P.rot ? reinterpret_cast<const double2*>(w + tab) : reinterpret_cast<const double2*>(sys->u);
  a.nb = P.nb;
  a.N1 = P.N1;
  a.gpack = reinterpret_cast<const int*>(w + o_g);
  a.ng = reinterpret_cast<const int*>(w + o_n);
  a.ng_max = P.ng_max;
  a.lo2 = P.lo[1];
  a.lo3 = P.lo[2];
  a.F2 = P.F[1];
  a.F3 = P.F[2];
  a.vscale = nullptr;
  a.out = reinterpret_cast<double2*>(out);
  char* buf = nullptr;
  if ((rc = staging_acquire(tab, &buf))) return rc;
  std::memset(buf, 0, tab);
  std::memcpy(buf + o_g, P.gpack.data(), P.gpack.size() * sizeof(int));
  std::memcpy(buf + o_n, P.ng.data(), P.ng.size() * sizeof(int));
  std::memcpy(buf + o_a, &a, sizeof(PdArgs));
  if (!jobs.empty()) std::memcpy(buf + o_j, jobs.data(), jobs.size() * sizeof(PdJob));
  HIP_TRY(hipMemcpyAsync(w, buf, tab, hipMemcpyHostToDevice, st));
  if ((rc = staging_release(st))) return rc;
  PdBatch b{};
  b.sys = reinterpret_cast<const PdArgs*>(w + o_a);
  b.jobs = reinterpret_cast<const PdJob*>(w + o_j);
  b.njobs = (int)jobs.size();
  b.persist = 0;
  b.cnt = nullptr;
  HIP_TRY(launch_pair_density(b, P.N2, P.N3, P.ng_max, lds, b.njobs, false, 0, st));
  return BSE_OK;
}

int bse_build_H(const bse_system* sys, int nsys, int precision, int flags, void* ws, size_t ws_bytes, void* stream) {
  if (!sys || nsys < 1) return fail(BSE_ERR_INVALID_ARG, "no systems");
  if (!ws) return fail(BSE_ERR_INVALID_ARG, "workspace is NULL");
  if (precision < BSE_FP64 || precision > BSE_BF16X3) return fail(BSE_ERR_INVALID_ARG, "bad precision %d", precision);
  if (flags & ~(BSE_VALIDATE | BSE_PERSISTENT | BSE_TIME_REVERSAL | BSE_FP32_PAIRDENS))
    return fail(BSE_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  if ((flags & BSE_FP32_PAIRDENS) && precision == BSE_FP64)
    return fail(BSE_ERR_INVALID_ARG, "BSE_FP32_PAIRDENS needs a mixed precision (split-FP32 or BF16x3)");
  for (int i = 0; i < nsys; ++i)
    if (!sys[i].H) return fail(BSE_ERR_INVALID_ARG, "H of system %d is NULL", i);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const Batch* Bp = nullptr;
  BatchOpts opt;
  opt.tr = (flags & BSE_TIME_REVERSAL) != 0;
  opt.pd32 = (flags & BSE_FP32_PAIRDENS) != 0;
  opt.mixed = precision != BSE_FP64;
  int rc = cached_batch(sys, nsys, Tune{}, opt, &Bp);
  if (rc) return rc;
  Tune tn = tune_for(batch_key(Bp->P, precision, Bp->pd32));
  if (flags & BSE_PERSISTENT) tn.persist = 1;
  if (precision != BSE_BF16X3) tn.s1_rows = 64;  // FP64 and FP32 parts: 64-row tiles only
  if ((tn.ktile != Tune{}.ktile || tn.s1_rows != Tune{}.s1_rows || tn.order != Tune{}.order) &&
      (rc = cached_batch(sys, nsys, tn, opt, &Bp)))
    return rc;
  const Batch& B = *Bp;
  if (ws_bytes < B.total) return fail(BSE_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, B.total);
  if (flags & BSE_VALIDATE) {
    if ((rc = upload_batch(B, sys, precision, static_cast<char*>(ws), st))) return rc;
    if ((rc = validate(B, sys, static_cast<char*>(ws), st))) return rc;
  }
  return run_build(B, sys, precision, tn, static_cast<char*>(ws), st);
}

size_t bse_build_H_full_workspace(const bse_system* sys) {
  const Batch *BA = nullptr, *BB = nullptr;
  if (full_batches(sys, BSE_FP64, 0, &BA, &BB)) return 0;
  return std::max(BA->total, BB->total);
}

int bse_build_H_full(const bse_system* sys, double* H2, int precision, int flags, void* ws, size_t ws_bytes,
                     void* stream) {
  if (!H2 || !ws) return fail(BSE_ERR_INVALID_ARG, "H2 / ws is NULL");
  const Batch *BA = nullptr, *BB = nullptr;
  int rc = full_batches(sys, precision, flags, &BA, &BB);
  if (rc) return rc;
  // (the plan cache keeps its four most recent plans, so the second lookup
  // cannot evict the first)
  const Batch& A = *BA;
  const Batch& Bc = *BB;
  const size_t need = std::max(A.total, Bc.total);
  if (ws_bytes < need) return fail(BSE_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  const int ns = A.P[0].ns;
  bse_system s = *sys;
  s.H = H2;
  Tune tn;
  if (flags & BSE_PERSISTENT) tn.persist = 1;
  if (flags & BSE_VALIDATE) {
    if ((rc = upload_batch(A, &s, BSE_FP64, w, st)) || (rc = validate(A, &s, w, st))) return rc;
  }
  if ((rc = run_build(A, &s, BSE_FP64, tn, w, st))) return rc;
  s.H = H2 + 2 * (size_t)ns;  // the coupling block starts at column NS
  if ((rc = run_build(Bc, &s, BSE_FP64, tn, w, st))) return rc;
  HIP_TRY(launch_full_lower(reinterpret_cast<double2*>(H2), ns, st));
  return BSE_OK;
}

int bse_build_H_backward(const bse_system* sys, const double* dH, double* dW, double* deps, double* dX,
                         double* drho_vv, double* drho_cc, int precision, int flags, void* ws, size_t ws_bytes,
                         void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (!sys) return fail(BSE_ERR_INVALID_ARG, "system pointer is NULL");
  if (sys->nirr <= 0)
    return backward_impl(sys, dH, dW, deps, dX, drho_vv, drho_cc, precision, flags, ws, ws_bytes, st);
  if (!dH || !ws) return fail(BSE_ERR_INVALID_ARG, "dH / ws is NULL");
  IrrBackward R;
  int rc = plan_irr_backward(sys, dW != nullptr, R);
  if (rc) return rc;
  if (ws_bytes < R.extra) return fail(BSE_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, R.extra);
  char* w = static_cast<char*>(ws);
  const int* dt = reinterpret_cast<const int*>(w);
  char* buf = nullptr;
  if ((rc = staging_acquire(R.tab.size() * sizeof(int), &buf))) return rc;
  std::memcpy(buf, R.tab.data(), R.tab.size() * sizeof(int));
  HIP_TRY(hipMemcpyAsync(w, buf, R.tab.size() * sizeof(int), hipMemcpyHostToDevice, st));
  if ((rc = staging_release(st))) return rc;
  const Plan& P = R.G;
  double2* Wf = reinterpret_cast<double2*>(w + R.o_Wf);
  HIP_TRY(launch_unfold_w(reinterpret_cast<const double2*>(sys->W), dt + R.t_wsrc, dt + R.t_wmap, dt + R.t_ng, P.nk,
                          P.ng_max, Wf, st));
  const bse_system s2 = unfolded_view(sys, reinterpret_cast<const double*>(Wf));
  double* dWf = dW ? reinterpret_cast<double*>(w + R.o_dWf) : nullptr;
  if ((rc = backward_impl(&s2, dH, dWf, deps, dX, drho_vv, drho_cc, precision, flags, w + R.extra,
                          ws_bytes - R.extra, st)))
    return rc;
  if (dW)
    HIP_TRY(launch_fold_dw(reinterpret_cast<const double2*>(dWf), dt + R.t_csr, dt + R.t_qlist, dt + R.t_wsrc,
                           dt + R.t_winv, dt + R.t_ngirr, P.nirr, P.ng_max, reinterpret_cast<double2*>(dW), st));
  return BSE_OK;
}

int bse_autotune(const bse_system* sys, int nsys, int precision, int flags, const char* cache_path,
                 bse_tuning* chosen, void* ws, size_t ws_bytes, void* stream) {
  if (!sys || nsys < 1) return fail(BSE_ERR_INVALID_ARG, "no systems");
  if (!ws) return fail(BSE_ERR_INVALID_ARG, "workspace is NULL");
  if (precision < BSE_FP64 || precision > BSE_BF16X3) return fail(BSE_ERR_INVALID_ARG, "bad precision %d", precision);
  if (flags & ~BSE_FP32_PAIRDENS) return fail(BSE_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  if ((flags & BSE_FP32_PAIRDENS) && precision == BSE_FP64)
    return fail(BSE_ERR_INVALID_ARG, "BSE_FP32_PAIRDENS needs a mixed precision (split-FP32 or BF16x3)");
  Tune t;
  int rc = autotune(sys, nsys, precision, (flags & BSE_FP32_PAIRDENS) != 0, cache_path, t, static_cast<char*>(ws),
                    ws_bytes, reinterpret_cast<hipStream_t>(stream));
  if (rc) return rc;
  if (chosen) {
    chosen->persistent = t.persist;
    chosen->ktile = t.ktile;
    chosen->wg_per_cu = t.wg_per_cu;
    chosen->pd_ms = t.pd_ms;
    chosen->s1_rows = t.s1_rows;
    chosen->s1_ms = t.s1_ms;
    chosen->order = t.order;
  }
  return BSE_OK;
}

int bse_autotune_last(bse_tuning* tried, int max_tried) {
  if (max_tried < 0 || (max_tried > 0 && !tried)) return fail(BSE_ERR_INVALID_ARG, "bad output array");
  const int n = std::min<int>(max_tried, (int)g_tried.size());
  for (int i = 0; i < n; ++i) {
    tried[i].persistent = g_tried[i].persist;
    tried[i].ktile = g_tried[i].ktile;
    tried[i].wg_per_cu = g_tried[i].wg_per_cu;
    tried[i].pd_ms = g_tried[i].pd_ms;
    tried[i].s1_rows = g_tried[i].s1_rows;
    tried[i].s1_ms = g_tried[i].s1_ms;
    tried[i].order = g_tried[i].order;
  }
  return (int)g_tried.size();
}

int bse_transition_dipoles(const bse_system* sys, const double* cell, const double* qhat, int nq, double* d,
                           void* ws, size_t ws_bytes, void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Plan P;
  int rc = make_geometry(sys, P);
  if (rc) return rc;
  if (!d || !ws || !qhat) return fail(BSE_ERR_INVALID_ARG, "d / ws / qhat is NULL");
  if (nq < 1 || nq > kMaxQhat) return fail(BSE_ERR_INVALID_ARG, "nq = %d not in 1..%d", nq, kMaxQhat);
  GradCell bc;
  if ((rc = grad_setup(sys, P, cell, bc))) return rc;
  Qhats qh{};
  for (int q = 0; q < nq; ++q)
    for (int x = 0; x < 3; ++x) {
      qh.v[q][x] = qhat[3 * q + x];
      if (!std::isfinite(qh.v[q][x])) return fail(BSE_ERR_INVALID_ARG, "qhat is not finite");
    }
  const size_t fft = align256((size_t)P.nk * P.nb * P.N1 * P.N2 * P.N3 * sizeof(double2));
  const size_t need = fft + (size_t)P.ns * 3 * sizeof(double2);
  if (ws_bytes < need) return fail(BSE_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  char* w = static_cast<char*>(ws);
  double2* D = reinterpret_cast<double2*>(w + fft);
  HIP_TRY(launch_grad(reinterpret_cast<const double2*>(sys->u), reinterpret_cast<double2*>(w), P.nk, P.nb, P.nv, P.nc,
                      sys->grid[0], sys->grid[1], sys->grid[2], bc, D, st));
  HIP_TRY(launch_dipole_project(D, sys->eps, qh, nq, P.nk, P.nv, P.nc, reinterpret_cast<double2*>(d), st));
  return BSE_OK;
}

size_t bse_transition_dipoles_workspace(const bse_system* sys) {
  Plan P;
  if (make_geometry(sys, P)) return 0;
  return align256((size_t)P.nk * P.nb * P.N1 * P.N2 * P.N3 * sizeof(double2)) + (size_t)P.ns * 3 * sizeof(double2);
}

int bse_spectrum(int ns, int nlam, const double* E, const double* A, const double* d, int nq, int nk,
                 double omega_cell, int nw, double w0_eV, double w1_eV, double eta_eV, double* eps2, void* ws,
                 size_t ws_bytes, void* stream) {
  int rc = spectrum_args(ns, nlam, E, A, d, nq, nk, omega_cell, nw, eta_eV, eps2);
  if (rc) return rc;
  if (!ws) return fail(BSE_ERR_INVALID_ARG, "workspace is NULL");
  if (ws_bytes < (size_t)nlam * sizeof(double)) return fail(BSE_ERR_WORKSPACE, "workspace below nlam doubles");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(launch_spectrum(ns, nlam, nq, E, reinterpret_cast<const double2*>(A), reinterpret_cast<const double2*>(d),
                          (double)nk * omega_cell, nw, w0_eV, w1_eV, eta_eV, static_cast<double*>(ws), eps2, st));
  return BSE_OK;
}

size_t bse_screening_workspace(const bse_system* sys) {
  ScrPlan S;
  if (make_screening_plan(sys, S)) return 0;
  return S.total;
}

int bse_screening(const bse_system* sys, const double* vq, double head, double* W, void* ws, size_t ws_bytes,
                  void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (!vq || !W || !ws) return fail(BSE_ERR_INVALID_ARG, "vq / W / ws is NULL");
  if (!std::isfinite(head)) return fail(BSE_ERR_INVALID_ARG, "head is not finite");
  ScrPlan S;
  int rc = make_screening_plan(sys, S);
  if (rc) return rc;
  if (ws_bytes < S.total) return fail(BSE_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, S.total);
  const Plan& P = S.G;
  const size_t lds = pd_lds_bytes(P.N1, P.N2, P.N3, P.F[1], P.F[2], P.ng_max, 0);
  if (lds > 160 * 1024) return fail(BSE_ERR_SHAPE, "FFT window needs more than 160 KiB of LDS");
  char* w = static_cast<char*>(ws);
  PdArgs a{};
  a.u = P.rot ? reinterpret_cast<const double2*>(w + S.o_ut) : reinterpret_cast<const double2*>(sys->u);
  a.nb = P.nb;
  a.N1 = P.N1;
  a.gpack = reinterpret_cast<const int*>(w + S.o_gpack);
  a.ng = reinterpret_cast<const int*>(w + S.o_ng);
  a.ng_max = P.ng_max;
  a.lo2 = P.lo[1];
  a.lo3 = P.lo[2];
  a.F2 = P.F[1];
  a.F3 = P.F[2];
  a.vscale = nullptr;
  a.out = reinterpret_cast<double2*>(w + S.o_Y);
  a.u32 = nullptr;
  char* buf = nullptr;
  if ((rc = staging_acquire(S.tables, &buf))) return rc;
  std::memset(buf, 0, S.tables);
  std::memcpy(buf + S.o_gpack, P.gpack.data(), P.gpack.size() * sizeof(int));
  std::memcpy(buf + S.o_ng, P.ng.data(), P.ng.size() * sizeof(int));
  std::memcpy(buf + S.o_args, &a, sizeof(PdArgs));
  std::memcpy(buf + S.o_qof, S.qof.data(), S.qof.size() * sizeof(int));
  if (S.gather) std::memcpy(buf + S.o_trmap, P.trmap.data(), P.trmap.size() * sizeof(int));
  for (size_t c = 0; c < S.qs.size(); ++c) {
    std::memcpy(buf + S.o_jobs[c], S.jobs[c].data(), S.jobs[c].size() * sizeof(PdJob));
    std::memcpy(buf + S.o_pk[c], S.pk[c].data(), S.pk[c].size() * sizeof(int4));
    std::memcpy(buf + S.o_tiles[c], S.tiles[c].data(), S.tiles[c].size() * sizeof(int4));
    if (!S.fill[c].empty()) std::memcpy(buf + S.o_fill[c], S.fill[c].data(), S.fill[c].size() * sizeof(int4));
    std::memcpy(buf + S.o_cslot[c], S.cslot[c].data(), S.cslot[c].size() * sizeof(int));
  }
  HIP_TRY(hipMemcpyAsync(w, buf, S.tables, hipMemcpyHostToDevice, st));
  if ((rc = staging_release(st))) return rc;
  if (P.rot)
    HIP_TRY(launch_rotate_axes(reinterpret_cast<const double2*>(sys->u), reinterpret_cast<double2*>(w + S.o_ut),
                               (long long)P.nk * P.nb, sys->grid[0], sys->grid[1], sys->grid[2], st));
  RpaArgs r{};
  r.Y = reinterpret_cast<double2*>(w + S.o_Y);
  r.M = reinterpret_cast<double2*>(W);
  r.ng = reinterpret_cast<const int*>(w + S.o_ng);
  r.eps = sys->eps;
  r.vq = vq;
  r.nv = P.nv;
  r.nc = P.nc;
  r.nk = P.nk;
  r.ng_max = P.ng_max;
  r.omega = (double)P.nk * sys->omega_cell;
  r.qof = reinterpret_cast<const int*>(w + S.o_qof);
  const int nslot = (int)S.qof.size();
  HIP_TRY(launch_rpa_init(r.M, r.ng, r.qof, nslot, P.ng_max, st));
  for (size_t c = 0; c < S.qs.size(); ++c) {
    PdBatch b{};
    b.sys = reinterpret_cast<const PdArgs*>(w + S.o_args);
    b.jobs = reinterpret_cast<const PdJob*>(w + S.o_jobs[c]);
    b.njobs = (int)S.jobs[c].size();
    b.persist = 0;
    b.cnt = nullptr;
    HIP_TRY(launch_pair_density(b, P.N2, P.N3, P.ng_max, lds, b.njobs, false, 0, st));
    if (S.gather)
      HIP_TRY(launch_rpa_fill(r.Y, reinterpret_cast<const int4*>(w + S.o_fill[c]), (int)S.fill[c].size(),
                              reinterpret_cast<const int*>(w + S.o_trmap), r.ng, P.nv, P.nc, P.ng_max, st));
    r.pk = reinterpret_cast<const int4*>(w + S.o_pk[c]);
    HIP_TRY(launch_rpa_scale(r, (int)S.pk[c].size(), st));
    r.nsplit = S.nsplit[c];
    r.part = reinterpret_cast<double2*>(w + S.o_part);
    r.part_q = S.max_part_q;
    HIP_TRY(launch_rpa_herk(r, reinterpret_cast<const int4*>(w + S.o_tiles[c]), (int)S.tiles[c].size(), st));
    HIP_TRY(launch_rpa_reduce(r, reinterpret_cast<const int*>(w + S.o_cslot[c]), (int)S.cslot[c].size(), st));
  }
  HIP_TRY(launch_rpa_mirror(r.M, r.ng, r.qof, nslot, P.ng_max, st));
  HIP_TRY(launch_rpa_invert(r.M, r.ng, r.qof, nslot, P.ng_max, st));
  HIP_TRY(launch_rpa_w(r.M, r.ng, r.qof, vq, nslot, P.ng_max, head, st));
  return BSE_OK;
}

size_t bse_haydock_workspace(int ns, int nq, int niter) {
  if (ns < 1 || nq < 1 || nq > kMaxQhat || niter < 1) return 0;
  return 3 * align256((size_t)nq * ns * sizeof(double2)) + align256((size_t)nq * niter * 2 * sizeof(double)) +
         align256((size_t)nq * sizeof(double));
}

int bse_haydock_spectrum(int ns, const double* H, const double* d, int nq, int niter, int nk, double omega_cell,
                         int nw, double w0_eV, double w1_eV, double eta_eV, double* eps2, double* coef, void* ws,
                         size_t ws_bytes, void* stream) {
  if (ns < 1 || nw < 1 || nk < 1 || niter < 1) return fail(BSE_ERR_INVALID_ARG, "bad sizes");
  if (nq < 1 || nq > kMaxQhat) return fail(BSE_ERR_INVALID_ARG, "nq = %d not in 1..%d", nq, kMaxQhat);
  if (!H || !d || !eps2 || !ws) return fail(BSE_ERR_INVALID_ARG, "NULL pointer");
  if (!(eta_eV > 0.0)) return fail(BSE_ERR_INVALID_ARG, "eta must be positive");
  if (!(omega_cell > 0.0)) return fail(BSE_ERR_INVALID_ARG, "omega_cell must be positive");
  const size_t need = bse_haydock_workspace(ns, nq, niter);
  if (ws_bytes < need) return fail(BSE_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  char* w = static_cast<char*>(ws);
  const size_t vec = align256((size_t)nq * ns * sizeof(double2));
  double2* V0 = reinterpret_cast<double2*>(w);
  double2* V1 = reinterpret_cast<double2*>(w + vec);
  double2* Y = reinterpret_cast<double2*>(w + 2 * vec);
  double* cf = reinterpret_cast<double*>(w + 3 * vec);
  double* n2 = reinterpret_cast<double*>(w + 3 * vec + align256((size_t)nq * niter * 2 * sizeof(double)));
  HIP_TRY(launch_haydock(ns, reinterpret_cast<const double2*>(H), reinterpret_cast<const double2*>(d), nq, niter,
                         (double)nk * omega_cell, nw, w0_eV, w1_eV, eta_eV, eps2, coef ? coef : cf, V0, V1, Y, n2,
                         reinterpret_cast<hipStream_t>(stream)));
  return BSE_OK;
}

int bse_profile(int enable) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = enable != 0;
  return BSE_OK;
}

int bse_profile_read(double* total_ms, long long* launches, int nstages, int reset) {
  if (nstages < 0 || (nstages > 0 && (!total_ms || !launches))) return fail(BSE_ERR_INVALID_ARG, "bad output arrays");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (const ProfRec& r : g_prof_pending) {
    float ms = 0.f;
    HIP_TRY(hipEventSynchronize(r.b));
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    g_prof_ms[r.stage] += ms;
    g_prof_n[r.stage] += 1;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof_pending.clear();
  for (int i = 0; i < nstages && i < BSE_NSTAGES; ++i) {
    total_ms[i] = g_prof_ms[i];
    launches[i] = g_prof_n[i];
  }
  if (reset)
    for (int i = 0; i < BSE_NSTAGES; ++i) {
      g_prof_ms[i] = 0;
      g_prof_n[i] = 0;
    }
  return BSE_OK;
}

int bse_set_chunk_budget(size_t bytes) {
  g_chunk_budget.store(bytes ? bytes : kChunkBudget);
  return BSE_OK;
}

int bse_release_host_state(void) {
  Staging& S = g_staging;
  if (S.pending) {
    HIP_TRY(hipEventSynchronize(S.done));
    S.pending = false;
  }
  if (S.buf) HIP_TRY(hipHostFree(S.buf));
  S.buf = nullptr;
  S.cap = 0;
  if (S.done) HIP_TRY(hipEventDestroy(S.done));
  S.done = nullptr;
  for (PlanCache& c : g_plan) {
    c.key.clear();
    c.B = Batch{};
    c.used = 0;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  return BSE_OK;
}

const char* bse_last_error(void) { return g_err.c_str(); }

}  // extern "C"
