/*
 * Plain FP64 CPU oracle for the Tamm-Dancoff Bethe-Salpeter Hamiltonian.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it exists so that the GPU path can be checked against a
 * slow, obviously correct evaluation of the same definitions.  It shares no
 * code, header, table or constant with the GPU library.
 *
 * Conventions (paper: Yan, Jacobsen, Thygesen, PRB 86, 045208 (2012)):
 *   grid N = (N1,N2,N3), real-space index j = (j1*N2 + j2)*N3 + j3;
 *   k-mesh n = (n1,n2,n3), k index (i1*n2 + i2)*n3 + i3;
 *   u[k][b][j] periodic parts with sum_j |u|^2 = 1, bands 0..nv-1 valence;
 *   gvec[q][g][3] Miller indices of the plane-wave sphere of momentum q;
 *   W[q][g][g'] screened interaction (4 pi inside), vx[g] Coulomb on S(0);
 *   transition S = (k, v, c) with index (k*nv + v)*nc + c; H in eV.
 * All arithmetic is IEEE double, round-to-nearest, no fast-math.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double TWO_PI = 6.283185307179586476925286766559;
static const double HARTREE_EV = 27.211386245988;

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static void triplet(const int *n, int k, int *t)
{
    t[2] = k % n[2];
    t[1] = (k / n[2]) % n[1];
    t[0] = k / (n[1] * n[2]);
}

/*
 * Momentum transfer between two mesh points (Sec. III.A: the q mesh has the
 * form of the k mesh and contains Gamma).  k' - k = q + G0 with q on the mesh
 * (iq, componentwise in [0, n)) and G0 = sum_d m0_d b_d, m0_d in {-1, 0}.
 */
void oracle_fold(const int *kmesh, int ka, int kb, int *iq, int *m0)
{
    int ta[3], tb[3], r[3];
    triplet(kmesh, ka, ta);
    triplet(kmesh, kb, tb);
    for (int d = 0; d < 3; ++d) {
        int dd = tb[d] - ta[d];
        r[d] = ((dd % kmesh[d]) + kmesh[d]) % kmesh[d];
        m0[d] = (dd - r[d]) / kmesh[d];
    }
    *iq = (r[0] * kmesh[1] + r[1]) * kmesh[2] + r[2];
}

static long long posmod(long long a, long long n)
{
    long long r = a % n;
    return r < 0 ? r + n : r;
}

/*
 * Pair density (charge density matrix), Sec. II.B:
 *   n_{a k, b k'}(G) = < psi_ak | exp(-i (q + G).r) | psi_bk' >
 * With psi = exp(i k.r) u and k' = k + q + G0 the Bloch phases cancel except
 * exp(i G0.r), so on the grid
 *   n(m) = sum_j conj(u_a(j)) u_b(j) exp(-2 pi i sum_d (m_d - m0_d) j_d / N_d)
 * for every Miller index m of the sphere of q.
 *
 * This is the full three-dimensional sum, term by term.  The exponent is
 * reduced to an integer modulo N1*N2*N3 before the cosine and sine are taken.
 */
void oracle_pair_density_full(const int *grid, const cplx *ua, const cplx *ub,
                              const int *m0, const int *gvec, int ng, cplx *out)
{
    const long long N1 = grid[0], N2 = grid[1], N3 = grid[2];
    const long long Nr = N1 * N2 * N3;
    cplx *tab = (cplx *)malloc(sizeof(cplx) * Nr);
    cplx *p = (cplx *)malloc(sizeof(cplx) * Nr);
    for (long long t = 0; t < Nr; ++t)
        tab[t] = cos(TWO_PI * (double)t / (double)Nr) - I * sin(TWO_PI * (double)t / (double)Nr);
    for (long long j = 0; j < Nr; ++j)
        p[j] = conj(ua[j]) * ub[j];
    for (int g = 0; g < ng; ++g) {
        long long f1 = gvec[3 * g + 0] - m0[0];
        long long f2 = gvec[3 * g + 1] - m0[1];
        long long f3 = gvec[3 * g + 2] - m0[2];
        cplx s = 0.0;
        for (long long j1 = 0; j1 < N1; ++j1)
            for (long long j2 = 0; j2 < N2; ++j2)
                for (long long j3 = 0; j3 < N3; ++j3) {
                    long long t = posmod(f1 * j1 * N2 * N3 + f2 * j2 * N1 * N3 + f3 * j3 * N1 * N2, Nr);
                    s += p[(j1 * N2 + j2) * N3 + j3] * tab[t];
                }
        out[g] = s;
    }
    free(tab);
    free(p);
}

/*
 * The same sum with the exponential factored into one factor per axis,
 *   n(m) = sum_j1 w1^{f1 j1} sum_j2 w2^{f2 j2} sum_j3 w3^{f3 j3} p(j),
 * w_d = exp(-2 pi i / N_d), f = m - m0.  Inner sums are taken only for the
 * f3 (then f2) values that occur in the sphere.  No fast transform is used.
 */
void oracle_pair_density_sep(const int *grid, const cplx *ua, const cplx *ub,
                             const int *m0, const int *gvec, int ng, cplx *out)
{
    const int N1 = grid[0], N2 = grid[1], N3 = grid[2];
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
    for (int g = 0; g < ng; ++g)
        for (int d = 0; d < 3; ++d) {
            int f = gvec[3 * g + d] - m0[d];
            if (f < lo[d]) lo[d] = f;
            if (f > hi[d]) hi[d] = f;
        }
    const int F2 = hi[1] - lo[1] + 1, F3 = hi[2] - lo[2] + 1;
    cplx *w1 = (cplx *)malloc(sizeof(cplx) * N1);
    cplx *w2 = (cplx *)malloc(sizeof(cplx) * N2);
    cplx *w3 = (cplx *)malloc(sizeof(cplx) * N3);
    for (int t = 0; t < N1; ++t) w1[t] = cos(TWO_PI * t / N1) - I * sin(TWO_PI * t / N1);
    for (int t = 0; t < N2; ++t) w2[t] = cos(TWO_PI * t / N2) - I * sin(TWO_PI * t / N2);
    for (int t = 0; t < N3; ++t) w3[t] = cos(TWO_PI * t / N3) - I * sin(TWO_PI * t / N3);
    cplx *T1 = (cplx *)malloc(sizeof(cplx) * (size_t)N1 * N2 * F3);
    cplx *T2 = (cplx *)malloc(sizeof(cplx) * (size_t)N1 * F2 * F3);
    for (int j1 = 0; j1 < N1; ++j1)
        for (int j2 = 0; j2 < N2; ++j2) {
            const size_t row = ((size_t)j1 * N2 + j2) * N3;
            for (int a3 = 0; a3 < F3; ++a3) {
                long long f3 = lo[2] + a3;
                cplx s = 0.0;
                for (int j3 = 0; j3 < N3; ++j3)
                    s += conj(ua[row + j3]) * ub[row + j3] * w3[posmod(f3 * j3, N3)];
                T1[((size_t)j1 * N2 + j2) * F3 + a3] = s;
            }
        }
    for (int j1 = 0; j1 < N1; ++j1)
        for (int a2 = 0; a2 < F2; ++a2) {
            long long f2 = lo[1] + a2;
            for (int a3 = 0; a3 < F3; ++a3) {
                cplx s = 0.0;
                for (int j2 = 0; j2 < N2; ++j2)
                    s += T1[((size_t)j1 * N2 + j2) * F3 + a3] * w2[posmod(f2 * j2, N2)];
                T2[((size_t)j1 * F2 + a2) * F3 + a3] = s;
            }
        }
    for (int g = 0; g < ng; ++g) {
        long long f1 = gvec[3 * g + 0] - m0[0];
        int a2 = gvec[3 * g + 1] - m0[1] - lo[1];
        int a3 = gvec[3 * g + 2] - m0[2] - lo[2];
        cplx s = 0.0;
        for (int j1 = 0; j1 < N1; ++j1)
            s += T2[((size_t)j1 * F2 + a2) * F3 + a3] * w1[posmod(f1 * j1, N1)];
        out[g] = s;
    }
    free(w1); free(w2); free(w3); free(T1); free(T2);
}

static void pair_density(int separable, const int *grid, const cplx *ua, const cplx *ub,
                         const int *m0, const int *gvec, int ng, cplx *out)
{
    if (separable)
        oracle_pair_density_sep(grid, ua, ub, m0, gvec, ng, out);
    else
        oracle_pair_density_full(grid, ua, ub, m0, gvec, ng, out);
}

/* A batch of independent pair densities (for tests): item i uses bands
 * (ka, a) and (kb, b) from u, shift m0 and the sphere of iq. */
void oracle_pair_density_batch(const int *grid, int nb, const cplx *u, int ng_max, const int *ng,
                               const int *gvec, const int *items /*[n][6]: ka a kb b iq +pad*/, const int *m0s,
                               int n, int separable, cplx *out /*[n][ng_max]*/)
{
    const size_t Nr = (size_t)grid[0] * grid[1] * grid[2];
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < n; ++i) {
        const int *it = items + 6 * i;
        const int iq = it[4];
        pair_density(separable, grid, u + ((size_t)it[0] * nb + it[1]) * Nr,
                     u + ((size_t)it[2] * nb + it[3]) * Nr, m0s + 3 * i,
                     gvec + (size_t)iq * ng_max * 3, ng[iq], out + (size_t)i * ng_max);
    }
}

/*
 * Blocks (k, k') of the Hamiltonian, computed independently of each other:
 *   H_SS' = (e_ck - e_vk) d_SS' + c (2 Vbar_SS' - D_SS'),  c = E_h / (Nk Omega_cell)
 * with S = (k v c), S' = (k' v' c') and
 *   Vbar_SS' = sum_{G != 0} conj(n_{vk,ck}(G)) v(G) n_{v'k',c'k'}(G)      (e-h exchange, Sec. II.C)
 *   D_SS'    = sum_{G,G'} conj(n_{vk,v'k'}(G)) W_GG'(k'-k) n_{ck,c'k'}(G')  (direct term, Sec. II.C)
 * The singlet kernel is 2 Vbar - W (K = V - W/2 with the spin factor 2), the
 * transition energy is e_c - e_v > 0, and Omega = Nk Omega_cell is the crystal
 * volume; the 4 pi lives inside v and W.
 */
int oracle_build_blocks(const int *grid, const int *kmesh, int nv, int nc, double omega_cell,
                        int ng_max, const int *ng, const int *gvec, const double *vx,
                        const cplx *u, const double *eps, const cplx *W,
                        const int *blocks, int nblk, int separable, cplx *out)
{
    const int nk = kmesh[0] * kmesh[1] * kmesh[2];
    const int nb = nv + nc;
    const int nt = nv * nc;
    const size_t Nr = (size_t)grid[0] * grid[1] * grid[2];
    const double c = HARTREE_EV / ((double)nk * omega_cell);
    const int zero[3] = {0, 0, 0};

    /* exchange pair densities n_{vk,ck}(G) on the q = 0 sphere, for the k that are needed */
    char *need = (char *)calloc(nk, 1);
    for (int b = 0; b < nblk; ++b) {
        need[blocks[2 * b]] = 1;
        need[blocks[2 * b + 1]] = 1;
    }
    cplx *X = (cplx *)calloc((size_t)nk * nt * ng_max, sizeof(cplx));
#pragma omp parallel for schedule(dynamic) collapse(2)
    for (int k = 0; k < nk; ++k)
        for (int vc = 0; vc < nt; ++vc) {
            if (!need[k]) continue;
            int v = vc / nc, cc = vc % nc;
            pair_density(separable, grid, u + ((size_t)k * nb + v) * Nr, u + ((size_t)k * nb + nv + cc) * Nr,
                         zero, gvec, ng[0], X + ((size_t)k * nt + vc) * ng_max);
        }

#pragma omp parallel for schedule(dynamic)
    for (int b = 0; b < nblk; ++b) {
        const int ka = blocks[2 * b], kb = blocks[2 * b + 1];
        int iq, m0[3];
        oracle_fold(kmesh, ka, kb, &iq, m0);
        const int n = ng[iq];
        const int *gq = gvec + (size_t)iq * ng_max * 3;
        const cplx *Wq = W + (size_t)iq * ng_max * ng_max;
        cplx *rv = (cplx *)malloc(sizeof(cplx) * nv * nv * n);
        cplx *rc = (cplx *)malloc(sizeof(cplx) * nc * nc * n);
        cplx *y = (cplx *)malloc(sizeof(cplx) * nc * nc * n);
        for (int v = 0; v < nv; ++v)
            for (int v2 = 0; v2 < nv; ++v2)
                pair_density(separable, grid, u + ((size_t)ka * nb + v) * Nr, u + ((size_t)kb * nb + v2) * Nr,
                             m0, gq, n, rv + (size_t)(v * nv + v2) * n);
        for (int c1 = 0; c1 < nc; ++c1)
            for (int c2 = 0; c2 < nc; ++c2)
                pair_density(separable, grid, u + ((size_t)ka * nb + nv + c1) * Nr,
                             u + ((size_t)kb * nb + nv + c2) * Nr, m0, gq, n, rc + (size_t)(c1 * nc + c2) * n);
        /* y_cc'(G) = sum_G' W_GG' n_{ck,c'k'}(G') */
        for (int cc = 0; cc < nc * nc; ++cc)
            for (int g = 0; g < n; ++g) {
                cplx s = 0.0;
                for (int g2 = 0; g2 < n; ++g2)
                    s += Wq[(size_t)g * ng_max + g2] * rc[(size_t)cc * n + g2];
                y[(size_t)cc * n + g] = s;
            }
        cplx *blk = out + (size_t)b * nt * nt;
        for (int v = 0; v < nv; ++v)
            for (int c1 = 0; c1 < nc; ++c1)
                for (int v2 = 0; v2 < nv; ++v2)
                    for (int c2 = 0; c2 < nc; ++c2) {
                        const cplx *xa = X + ((size_t)ka * nt + v * nc + c1) * ng_max;
                        const cplx *xb = X + ((size_t)kb * nt + v2 * nc + c2) * ng_max;
                        cplx vx_sum = 0.0;
                        for (int g = 0; g < ng[0]; ++g) {
                            const int *m = gvec + 3 * g;
                            if (m[0] == 0 && m[1] == 0 && m[2] == 0) continue; /* Vbar: G = 0 left out */
                            vx_sum += conj(xa[g]) * vx[g] * xb[g];
                        }
                        const cplx *a = rv + (size_t)(v * nv + v2) * n;
                        const cplx *yy = y + (size_t)(c1 * nc + c2) * n;
                        cplx d_sum = 0.0;
                        for (int g = 0; g < n; ++g)
                            d_sum += conj(a[g]) * yy[g];
                        cplx h = c * (2.0 * vx_sum - d_sum);
                        if (ka == kb && v == v2 && c1 == c2)
                            h += eps[(size_t)ka * nb + nv + c1] - eps[(size_t)ka * nb + v];
                        blk[(size_t)(v * nc + c1) * nt + (v2 * nc + c2)] = h;
                    }
        free(rv); free(rc); free(y);
    }
    free(X);
    free(need);
    return 0;
}
