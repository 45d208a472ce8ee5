/*
 * bse.h -- C ABI of the MI355X (gfx950) Tamm-Dancoff Bethe-Salpeter
 * Hamiltonian builder.
 *
 * Paper: J. Yan, K. W. Jacobsen, K. S. Thygesen, "Optical properties of bulk
 * semiconductors and graphene/boron-nitride: the Bethe-Salpeter equation with
 * derivative discontinuity-corrected DFT energies", PRB 86, 045208 (2012).
 *
 * What is computed (Sec. II.C, with the Tamm-Dancoff approximation of Sec. IV.C
 * and the appendix):
 *
 *   H_SS' = (e_ck - e_vk) delta_SS' + c * (2 Vbar_SS' - D_SS'),
 *   c     = E_h / (Nk * Omega_cell)             (E_h = 27.211386245988 eV),
 *   S = (k, v, c) with row index (k*nv + v)*nc + c,
 *   Vbar_SS' = sum_{G != 0} conj(n_{vk,ck}(G)) v(G) n_{v'k',c'k'}(G)    (e-h exchange, G = 0 left out)
 *   D_SS'    = sum_{G,G'} conj(n_{vk,v'k'}(G)) W_GG'(k'-k) n_{ck,c'k'}(G')  (screened direct term)
 *   n_{ak,bk'}(G) = sum_r conj(u_ak(r)) u_bk'(r) exp(-2 pi i (m - m0).j / N)  (pair density, Sec. II.B)
 *
 * where k' - k = q + G0 is folded onto the k-shaped q mesh (Sec. III.A),
 * m are the Miller indices of the plane-wave sphere of q and m0 those of G0.
 *
 * Conventions shared by every entry point:
 *   - Complex numbers are interleaved (re, im) doubles.
 *   - Arrays marked DEVICE live in GPU memory of the current HIP device;
 *     arrays marked HOST live in host memory and are read during the call.
 *   - The caller owns every buffer, including the workspace.  The library
 *     allocates no device memory.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *     on it and the call returns; the caller synchronises.  Host-side plan
 *     tables go to the workspace by asynchronous copies from a pinned host
 *     staging buffer that the library keeps per calling thread; the next
 *     call on that thread waits for those copies before reusing it.
 *   - A non-zero return means nothing was enqueued (argument errors) or that
 *     a HIP call failed; bse_last_error() gives text for the calling thread.
 *   - Calls on one device that share a workspace must not overlap.
 *
 * State kept between calls (host side only; no device memory):
 *   - a pinned host staging buffer per calling thread (hipHostMalloc, grown
 *     on demand) from which the plan tables are copied;
 *   - a cache of the last four host plans per calling thread, keyed by the
 *     shapes and the contents of the host sphere tables, so that a repeated
 *     build of one shape skips planning;
 *   - the launch choices bse_autotune measured, per batch signature, for the
 *     life of the process (shared by all threads);
 *   - the per-stage timing records while bse_profile is enabled;
 *   - the text of the last error per thread.
 * bse_release_host_state() frees the first three.  The only file the library
 * touches is the tuning cache that the caller names in bse_autotune: read on
 * every call and appended to when a new signature is timed; bse_build_H
 * reads no file.
 */
#ifndef BSE_H
#define BSE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum bse_status {
    BSE_OK = 0,
    BSE_ERR_INVALID_ARG = -1,  /* null pointer, bad size or unsupported value  */
    BSE_ERR_SHAPE = -2,        /* grid / sphere / band counts not supported      */
    BSE_ERR_WORKSPACE = -3,    /* ws_bytes below bse_workspace_size()            */
    BSE_ERR_HIP = -4,          /* a HIP runtime call failed                      */
    BSE_ERR_NOT_HERMITIAN = -5,/* BSE_VALIDATE: W(q) violates Hermiticity / TR   */
    BSE_ERR_NONFINITE = -6,    /* BSE_VALIDATE: NaN or Inf in an input           */
    BSE_ERR_UNSUPPORTED = -7,  /* mode not implemented                           */
    BSE_ERR_NOT_SYMMETRIC = -8 /* BSE_VALIDATE with BSE_TIME_REVERSAL: u is not
                                  time-reversal symmetric                        */
};

/* Arithmetic of the two dense contractions: the exchange and the first stage
 * of the direct term (conj(rho_vv')^T W(q) per q).  The second stage of the
 * direct term (one pass over its operands, bound by memory bandwidth), the
 * pair densities (unless BSE_FP32_PAIRDENS), the transition-energy diagonal
 * and the q = 0 head of W are FP64 in every mode. */
enum bse_precision {
    BSE_FP64 = 0,       /* FP64 MFMA                                           */
    BSE_SPLIT_FP32 = 1, /* operands split into FP32 hi + lo, 3 products, FP32 acc */
    BSE_BF16X3 = 2      /* operands split into BF16 hi + lo, 3 products, FP32 acc */
};

enum bse_flags {
    BSE_VALIDATE = 1,    /* scan the inputs first and wait for the result:
                            NaN/Inf in u, eps, vx or W -> BSE_ERR_NONFINITE;
                            W(q) not Hermitian, or not obeying time reversal
                            where the spheres allow the check, by more than
                            1e-10 max|W| (|re| + |im| of the difference)
                            -> BSE_ERR_NOT_HERMITIAN                             */
    BSE_PERSISTENT = 2,  /* build a batch of systems with one persistent launch   */
    BSE_PROJECT_DW = 4,  /* backward: project dW onto Hermitian, time-reversal
                            symmetric W (group average of Sec. III.A, T = 1)     */
    BSE_TIME_REVERSAL = 8, /* bse_build_H (and the backward): the inputs obey
                            time reversal without spin-orbit coupling.  For kbar
                            the mesh point of -k, with -k = kbar - K (K a lattice
                            vector, entries 0 or 1 in units of the mesh),
                            u_{n,kbar}(r_j) = exp(-i K.r_j) conj(u_{n,k}(r_j)),
                            r_j = j/N per axis, for every k with kbar != k (as
                            when the wave functions at -k are made from those at
                            k; nothing is assumed at points that are their own
                            partner).  Then the pair densities of a k pair follow
                            from those of its image (kbar, kbar') (Sec. III.A,
                            the pair-density transformation with time reversal):
                            of each pair and its image only one is transformed,
                            the other is gathered from it (conjugate on the
                            sphere map of W, or the two bands exchanged).  Pairs
                            that touch a point with kbar = k are transformed
                            directly.  The G spheres must be closed under that
                            map (else BSE_ERR_SHAPE).  With BSE_VALIDATE the
                            relation of u is checked to 1e-10 max|u| (else
                            BSE_ERR_NOT_SYMMETRIC); without it, inputs that
                            break it give a wrong H                            */
    BSE_FP32_PAIRDENS = 16 /* bse_build_H, bse_autotune and the backward, with
                            BSE_SPLIT_FP32 or BSE_BF16X3 only
                            (else BSE_ERR_INVALID_ARG): the valence-valence and
                            conduction-conduction pair densities are transformed
                            in FP32 from an FP32 copy of u (rounded to nearest,
                            made once per call in the workspace) and stored as
                            FP64; the exchange pair densities stay FP64.  Applies
                            to grids whose pair-density planes (after the axis
                            rotation) are at most 32 x 32 with even sides; other
                            grids keep FP64.  Relative error of a density about
                            1e-6; the workspace grows by Nk*nb*Nr*8 bytes      */
};

enum bse_pd_kind {
    BSE_PD_EXCH = 0,   /* n_{vk,ck}(G) on S(0):   out [Nk][nv][nc][ng_max]             */
    BSE_PD_VV = 1,     /* n_{vk,v'k'}(G) on S(q): out [npairs][nv][nv][ng_max]          */
    BSE_PD_CC = 2,     /* n_{ck,c'k'}(G) on S(q): out [npairs][nc][nc][ng_max]          */
    BSE_PD_DIPOLE = 3  /* <u_vk| grad |u_ck>:     out [Nk][nv][nc][3]                   */
};

/*
 * One crystal.  Shapes: Nk = n1*n2*n3, nb = nv + nc, Nr = N1*N2*N3,
 * NS = Nk*nv*nc.  Supported grids: N2, N3 in {8, 12, 16, 24, 32, 48, 64, 96},
 * any N1 >= 1.
 */
typedef struct bse_system {
    int grid[3];          /* N1, N2, N3; real-space index (j1*N2 + j2)*N3 + j3            */
    int kmesh[3];         /* n1, n2, n3; k index (i1*n2 + i2)*n3 + i3                       */
    int nv, nc;           /* valence and conduction bands in H (bands 0..nv-1 are valence)  */
    double omega_cell;    /* unit-cell volume in bohr^3                                     */
    int ng_max;           /* row stride of gvec, W and every pair-density row               */
    const int *ng;        /* HOST  [Nk]               sphere size N_G(q), q indexed like k     */
    const int *gvec;      /* HOST  [Nk][ng_max][3]    Miller indices; gvec[0][0] = (0,0,0)     */
    const double *vx;     /* DEVICE [ng_max]          Coulomb v(Q+G) on S(Q), the sphere of the
                                                      exciton momentum (4 pi inside), units of W;
                                                      the entry of G = 0 is not read            */
    const double *u;      /* DEVICE [Nk][nb][Nr] complex  periodic parts, sum_r |u|^2 = 1      */
    const double *eps;    /* DEVICE [Nk][nb]           band energies in eV                       */
    const double *W;      /* DEVICE [Nk][ng_max][ng_max] complex, W[q][G][G'] (4 pi inside);
                                                      Hermitian and obeying time reversal;
                                                      entries past ng(q) are not read           */
    double *H;            /* DEVICE [NS][NS] complex, out, eV; every element is written        */
    int qexc;             /* exciton momentum Q as a q-mesh index (0: the optical limit).  The
                             e-h basis of the BSE eigenproblem (Sec. II.C) pairs the hole at k
                             with the electron at k + Q: S = (k, v, c) stands for (v k, c k+Q),
                             the transition energy is e_{c,k+Q} - e_{v,k}, the exchange runs
                             over S(Q) without G = 0 with the densities n_{vk,c k+Q}, and the
                             direct term pairs n_{vk,v'k'} with n_{c k+Q, c' k'+Q} (Eqs. V_eh,
                             W_SS).  Q != 0: BSE_TIME_REVERSAL -> BSE_ERR_INVALID_ARG; the
                             backward gives dW and deps (the gradients of the pair
                             densities -> BSE_ERR_UNSUPPORTED); BSE_PD_EXCH then gives
                             n_{vk, c k+Q}.  Out of range -> BSE_ERR_INVALID_ARG.          */
    /* W from the irreducible q points only (Sec. III.A).  nirr = 0: W holds W(q) for every q
     * as above.  nirr > 0: W holds nirr matrices [nirr][ng_max][ng_max], the screened
     * interaction at the irreducible q points, and every W(q) is unfolded from them by the
     * point-group and time-reversal relations of Sec. III.A:
     *   q =  T q_IBZ + G0:  W_GG'(q) = W_{T^-1(G+G0), T^-1(G'+G0)}(q_IBZ),
     *   q = -T q_IBZ + G0:  W_GG'(q) = conj(W_{-T^-1(G+G0), -T^-1(G'+G0)}(q_IBZ)),
     * given as index maps: W_GG'(q) = W[wsrc[q][0]][wmap[q][G]][wmap[q][G']], conjugated
     * when wsrc[q][1] != 0.  The FP64 contraction reads W through the maps (no unfolded copy);
     * the mixed modes unfold while they split W.  Every q mapped to one matrix has the same
     * ng(q), row q of wmap is a permutation of 0..ng(q)-1 (else BSE_ERR_SHAPE), and
     * wmap[0][0] = 0 (G = 0 of q = 0 stays in place).  BSE_VALIDATE then checks the nirr
     * matrices for finiteness and Hermiticity; the time-reversal relation holds by
     * construction of the maps and is not checked.  bse_build_H_backward then returns dW as
     * [nirr][ng_max][ng_max], the gradient with respect to those matrices: the adjoint of the
     * unfolding, dW_s[a][b] = sum over the q and G, G' that read entry (a, b) of matrix s of
     * dW(q)[G][G'], conjugated for the time-reversed images (it unfolds W into its workspace,
     * which grows by 2 Nk ng_max^2 complex values).  nirr < 0 or > Nk, a NULL map, or a map
     * entry out of range -> BSE_ERR_INVALID_ARG.  The maps are HOST memory, read while the
     * call plans.                                                                        */
    int nirr;
    const int *wsrc;      /* HOST [Nk][2]       (source matrix, conjugate flag) per q            */
    const int *wmap;      /* HOST [Nk][ng_max]  position of +-T^-1(G + G0) in the source sphere;
                                                entries past ng(q) are not read              */
} bse_system;

/* Bytes of device workspace that bse_build_H / bse_pair_density /
 * bse_build_H_backward need for these systems, with or without
 * BSE_TIME_REVERSAL; with BSE_FP32_PAIRDENS in flags, also room for the FP32
 * copy of u (precision and the other flags are not used). */
size_t bse_workspace_size(const bse_system *sys, int nsys, int precision, int flags);

/*
 * Pair densities n_{ak,bk'}(G) (Sec. II.B, eq. for the charge density matrix)
 * for the ordered k pairs `kpairs` (HOST [npairs][2] = (k, k')), or for every
 * k (BSE_PD_EXCH, BSE_PD_DIPOLE; kpairs ignored).  Entries g >= ng(q) of each
 * row are written as zero.  BSE_PD_EXCH rows are NOT scaled by v(G).
 * BSE_PD_DIPOLE gives the k.p matrix element <u_vk|grad|u_ck> of Sec. II.B
 * (Cartesian, bohr^-1) from the spectral derivative of u with the Nyquist
 * planes removed, using the cell given in `cell` (HOST [9], rows a1 a2 a3 in
 * bohr; ignored for other kinds); it needs every grid length in the supported
 * set (N1 included), nc <= 8 and a workspace of Nk*nb*Nr complex.
 * `out` is DEVICE complex; sys->H is not read.
 */
int bse_pair_density(const bse_system *sys, int kind, const int *kpairs, int npairs,
                     const double *cell, double *out, void *ws, size_t ws_bytes, void *stream);

/*
 * Builds H for `nsys` independent systems (each writes its own sys[i].H).
 * precision: enum bse_precision.  flags: enum bse_flags.
 */
int bse_build_H(const bse_system *sys, int nsys, int precision, int flags,
                void *ws, size_t ws_bytes, void *stream);

/*
 * Adjoint of bse_build_H for one system: given dL/dH (DEVICE [NS][NS] complex,
 * the PyTorch convention dL/dRe H + i dL/dIm H), returns (every output
 * DEVICE complex or real as shown, nullable, fully written when given):
 *   dW      [Nk][ng_max][ng_max]     dL/dW_GG'(q), zero past ng(q) ([nirr][ng_max][ng_max] with W given
 *                                    at the irreducible q points: see bse_system.nirr)
 *   deps    [Nk][nb] (real)          dL/de (eV/eV); at exciton momentum Q the conduction
 *                                    energy of S = (k, v, c) is e_{c,k+Q}, so its gradient lands at k+Q
 *   dX      [Nk][nv][nc][ng_max]     dL/dn_{vk,ck}(G) on S(0) (the pair density
 *                                    itself, not scaled by v), zero at G = 0
 *                                    and past ng(0)
 *   drho_vv [npairs][nv][nv][ng_max] dL/dn_{vk,v'k'}(G) on S(q(k,k'))
 *   drho_cc [npairs][nc][nc][ng_max] dL/dn_{ck,c'k'}(G), zero past ng(q)
 * for the pairs k <= k' in lexicographic order (0,0), (0,1), ..., (Nk-1,Nk-1)
 * (Sec. II.C: the lower k blocks of H are the conjugate transpose of the
 * upper ones, so the densities of the upper pairs are the independent ones).
 * Pair densities are recomputed, not read from a previous build.  Without
 * BSE_PROJECT_DW, dW is the partial derivative of the map the build computes
 * (upper k blocks, lower ones mirrored); with it, dW is projected onto the
 * Hermitian, time-reversal symmetric W on which that map and the all-blocks
 * definition agree.  With BSE_TIME_REVERSAL the recomputed pair densities
 * use the time-reversal images as in bse_build_H (same contract on u, not
 * checked here); with BSE_FP32_PAIRDENS (mixed precisions only) the valence
 * and conduction densities are recomputed in FP32 as in bse_build_H.  precision selects the arithmetic of the dW contraction
 * (its q = 0 head entry is FP64 in every mode); the density gradients are
 * FP64.  At exciton momentum Q != 0 the recomputed conduction densities are
 * those of the pairs (k+Q, k'+Q), as in bse_build_H; dX, drho_vv and drho_cc
 * must then be NULL (else BSE_ERR_UNSUPPORTED), and BSE_TIME_REVERSAL is
 * refused as in the build.  sys->H is not read.
 */
int bse_build_H_backward(const bse_system *sys, const double *dH, double *dW, double *deps, double *dX,
                         double *drho_vv, double *drho_cc, int precision, int flags, void *ws, size_t ws_bytes,
                         void *stream);

/*
 * Launch choices of bse_build_H for one batch signature (grids, k meshes,
 * bands, sphere sizes and windows of every system, precision).
 */
typedef struct bse_tuning {
    int persistent;  /* 1: persistent work-queue dispatch of the pair densities   */
    int ktile;       /* k tile of the pair-density dispatch order                 */
    int wg_per_cu;   /* persistent dispatch: workgroups per compute unit          */
    float pd_ms;     /* measured pair-density launch (first chunk), ms            */
    int s1_rows;     /* rows per workgroup tile (64, or 128 with the BF16
                        parts) of the first direct-term contraction
                        conj(rho_vv')^T W(q)                                     */
    float s1_ms;     /* measured launch of that contraction (first chunk), ms;
                        0 in the entries that time the pair densities          */
    int order;       /* static pair-density job order: 0 one contiguous segment
                        of k tiles per XCD; 1 the tiles dealt in order across
                        the XCDs; 2 as 0 with the valence-pair jobs of a
                        system before its conduction-pair jobs                 */
} bse_tuning;

/*
 * Autotuner (for callers that build the same batch shape many times).  Times
 * the dominant launch (the valence and conduction pair densities of the first
 * chunk of k pairs) of this batch under
 * static dispatch with k tiles 4, 8, 16 in each job order (field order of
 * bse_tuning), and persistent dispatch with 1..4 workgroups per CU; then, with the fastest of those, the first direct-term
 * contraction of that chunk (in the given precision) with workgroup tiles of
 * 64 x 64 and (BF16x3 only) 128 x 64 complex outputs.  It keeps both choices for every
 * later bse_build_H of the same signature in this process (BSE_PERSISTENT
 * still forces persistent dispatch).  flags: 0, or BSE_FP32_PAIRDENS (with a mixed precision) to tune
 * the FP32 pair-density kernel, whose builds then use that choice.  cache_path (HOST, nullable): a text file of one JSON object per
 * line; a matching line is used without timing, a new result is appended.
 * Blocks until the timing runs finish; needs the forward workspace of
 * bse_build_H and overwrites its pair-density area.  `chosen` (HOST,
 * nullable) receives the choice.  Results of bse_build_H do not depend on the
 * choice (every pair density is computed the same way in any order).
 */
int bse_autotune(const bse_system *sys, int nsys, int precision, int flags, const char *cache_path,
                 bse_tuning *chosen, void *ws, size_t ws_bytes, void *stream);

/* The candidates (with their times) that the last bse_autotune on this thread
 * measured: writes up to max_tried entries to `tried` (HOST) and returns how
 * many there were (0 after a cache hit), or a negative status. */
int bse_autotune_last(bse_tuning *tried, int max_tried);

/*
 * The Bethe-Salpeter Hamiltonian beyond the Tamm-Dancoff approximation in the
 * optical limit (Sec. II.C and the appendix: e-h states (v k, c k) and h-e
 * states (c k, v k), whose kernel rows carry the opposite occupation factor):
 *   H2 = [[A, B], [-B^H, -conj(A)]],  A = the H of bse_build_H,
 *   B[(k v c)][(k' v' c')] = c (2 Vbar - D) between (v k, c k) and (c' k', v' k'):
 *     Vbar = sum_{G != 0} conj(n_{vk,ck}(G)) v(G) n_{c'k',v'k'}(G),
 *     D    = sum_{G,G'} conj(n_{vk,c'k'}(G)) W_GG'(k'-k) n_{ck,v'k'}(G').
 * The lower blocks follow from the upper ones for Hermitian,
 * time-reversal-consistent W, a q = 0 sphere closed under G -> -G (else
 * BSE_ERR_SHAPE) and v(-G) = v(G).  H2: DEVICE [2 NS][2 NS] complex, eV,
 * every element written; sys->H is not used.  FP64 only (else
 * BSE_ERR_UNSUPPORTED), sys->qexc = 0 (else BSE_ERR_UNSUPPORTED); flags 0,
 * BSE_VALIDATE, BSE_PERSISTENT.  ws: bse_build_H_full_workspace(sys) bytes.
 */
int bse_build_H_full(const bse_system *sys, double *H2, int precision, int flags, void *ws, size_t ws_bytes,
                     void *stream);
size_t bse_build_H_full_workspace(const bse_system *sys);

/*
 * Transition dipoles of the optical limit (Sec. II.B: for q -> 0 the pair
 * density n_{vk,ck}(0) tends to -i q.<u_vk|grad|u_ck>/(e_ck - e_vk); the
 * spectrum of Sec. II.C pairs each exciton with that factor per unit |q|):
 *   d[p][S] = qhat_p . <u_vk|grad|u_ck> / ((e_ck - e_vk) / E_h)
 * in Hartree atomic units (bohr), S = (k*nv + v)*nc + c, for nq polarisations
 * qhat (HOST [nq][3], Cartesian, used as given; 1 <= nq <= 8).  The matrix
 * element is the spectral derivative of u with the Nyquist planes removed
 * (cell: HOST [9], rows a1 a2 a3 in bohr).  d is DEVICE [nq][NS] complex.
 * Every grid length must be in the supported set and nc <= 8.  ws needs
 * bse_transition_dipoles_workspace(sys) bytes.
 */
int bse_transition_dipoles(const bse_system *sys, const double *cell, const double *qhat, int nq, double *d,
                           void *ws, size_t ws_bytes, void *stream);
size_t bse_transition_dipoles_workspace(const bse_system *sys);

/*
 * Absorption spectrum from the spectral representation of the irreducible
 * response (Sec. II.C, macroscopic dielectric function with Vbar; Tamm-Dancoff
 * so the overlap matrix is the identity), averaged over nq polarisations:
 *   t_pl    = sum_S A[S][l] d[p][S]
 *   eps2(w) = 8 pi / (nk * omega_cell) * (1/nq) sum_p sum_l |t_pl|^2 * eta / ((w - E_l)^2 + eta^2)
 * (spin 2, eta the half width).  E (DEVICE [nlam], eV), A (DEVICE [ns][nlam]
 * complex, eigenvectors as columns), d (DEVICE [nq][ns] complex, from
 * bse_transition_dipoles), eps2 (DEVICE [nw]) on w_i = w0 + i*(w1-w0)/(nw-1).
 * Energies and eta are in eV and converted to Hartree inside.  ws (DEVICE)
 * needs nlam doubles.
 */
int bse_spectrum(int ns, int nlam, const double *E, const double *A, const double *d, int nq, int nk,
                 double omega_cell, int nw, double w0_eV, double w1_eV, double eta_eV, double *eps2, void *ws,
                 size_t ws_bytes, void *stream);

/*
 * Static RPA screened interaction W(q) of bse_build_H from the wave
 * functions (Sec. II.B: Eq. chi0_GG at omega = 0 and Eq. epsilon_-1 with the
 * RPA kernel; Sec. III.A: W_GG' = 4 pi eps^-1_GG' / (|q+G||q+G'|)):
 *   chi0_GG'(q) = (2/Omega) sum_k sum_{n,n'} (f_nk - f_n'k+q) n(G) conj(n(G')) / (e_nk - e_n'k+q),
 *   n = n_{nk,n'k+q} (pair density), Omega = Nk * Omega_cell, f = 1 for the
 *   nv occupied and 0 for the nc empty bands of sys (both orders of an
 *   occupied-empty pair enter),
 *   eps = 1 - v^1/2 chi0 v^1/2 (Hermitian positive definite),
 *   W(q) = v^1/2 eps^-1 v^1/2, with v^1/2 = sqrt(vq[q][G]).
 * At q = 0 the G = 0 row and column are left out of eps; W[0][0][0] = head
 * and the wings W[0][0][G], W[0][G][0] are zero (the divergent head is
 * integrated out in the paper; here it is a given value).
 * sys: grid, kmesh, nv, nc, omega_cell, ng_max, ng, gvec, u and eps as for
 * bse_build_H (empty bands at least 1 meV above every occupied one); W, vx
 * and H are not read.  vq: DEVICE [Nk][ng_max], v(q+G) on each sphere (4 pi
 * inside; bulk or truncated; the entry of G = 0 at q = 0 is not read).
 * W: DEVICE [Nk][ng_max][ng_max] complex out, zero past ng(q); it is the
 * input W of bse_build_H for the same spheres.  With sys->nirr > 0 only the
 * irreducible q points are computed (Sec. III.A: the q sum is reduced by the
 * symmetry, every other W(q) is its image): W is then [nirr][ng_max][ng_max],
 * matrix i at the q that sys->wsrc / sys->wmap map to matrix i without
 * conjugation by the identity map (the lowest such q; none ->
 * BSE_ERR_SHAPE), which is the input W of bse_build_H with the same maps.
 * ws: bse_screening_workspace(sys) bytes (pair densities of a chunk of q,
 * sized by bse_set_chunk_budget).  FP64 throughout.
 */
int bse_screening(const bse_system *sys, const double *vq, double head, double *W, void *ws, size_t ws_bytes,
                  void *stream);
size_t bse_screening_workspace(const bse_system *sys);

/*
 * The spectrum of bse_spectrum without the eigenpairs of H, for Hamiltonians
 * too large to diagonalise: the resolvent of the appendix (Eq. resolvent,
 * Tamm-Dancoff) in the state v = conj(d_p) satisfies
 *   sum_l |t_pl|^2 eta / ((w - E_l)^2 + eta^2) = -Im v^H (w + i eta - H)^-1 v,
 * evaluated by the Haydock recursion: niter steps of the Lanczos three-term
 * recurrence from v/|v| (no reorthogonalisation; one pass over H per step for
 * all polarisations together), then the continued fraction
 *   g(z) = 1 / (z - a_0 - b_0^2 / (z - a_1 - ... / (z - a_{niter-1}))).
 * The broadened spectrum converges with niter (bandwidth / niter well below
 * eta; at most a few hundred steps for eta = 0.1 eV at the sizes here).
 * H: DEVICE [ns][ns] complex, Hermitian, eV (e.g. from bse_build_H);
 * d: DEVICE [nq][ns] complex (bse_transition_dipoles), 1 <= nq <= 8;
 * eps2: DEVICE [nw] as in bse_spectrum (8 pi / (nk omega_cell), average over
 * the polarisations); coef: DEVICE [nq][niter][2] (a_j, b_j in eV), nullable.
 * ws: bse_haydock_workspace(ns, nq, niter) bytes.
 */
int bse_haydock_spectrum(int ns, const double *H, const double *d, int nq, int niter, int nk, double omega_cell,
                         int nw, double w0_eV, double w1_eV, double eta_eV, double *eps2, double *coef, void *ws,
                         size_t ws_bytes, void *stream);
size_t bse_haydock_workspace(int ns, int nq, int niter);

/*
 * bse_spectrum without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments and result as bse_spectrum; the nlam
 * partial results (one double per exciton) live in a static device array of
 * BSE_NOALLOC_MAX_NLAM doubles (8 MiB) that each GPU the library runs on holds
 * until the process ends.  nlam > BSE_NOALLOC_MAX_NLAM -> BSE_ERR_WORKSPACE
 * (nothing enqueued).  Calls no allocating routine.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads) race and must be ordered by the caller.
 */
#define BSE_NOALLOC_MAX_NLAM 1048576
int bse_spectrum_noalloc(int ns, int nlam, const double *E, const double *A, const double *d, int nq, int nk,
                         double omega_cell, int nw, double w0_eV, double w1_eV, double eta_eV, double *eps2,
                         void *stream);

/*
 * Per-stage GPU timing of bse_build_H.  While enabled, every kernel launch of
 * bse_build_H is bracketed by two hipEvents recorded on the call's stream.
 * bse_profile_read waits for the recorded events, adds their elapsed times
 * (ms) and launch counts per stage into total_ms / launches (HOST, nstages
 * entries, stage order of enum bse_stage) and, if reset, forgets them.
 */
enum bse_stage {
    BSE_STAGE_VSCALE = 0,   /* sqrt v(G) table                         */
    BSE_STAGE_PD_EXCH = 1,  /* pair densities n_{vk,ck}                 */
    BSE_STAGE_PD_VV = 2,    /* pair densities n_{vk,v'k'} and n_{ck,c'k'}
                               (one launch per chunk of k pairs)       */
    BSE_STAGE_PD_CC = 3,    /* (no longer used: counted with PD_VV)    */
    BSE_STAGE_EXCHANGE = 4, /* exchange GEMM                            */
    BSE_STAGE_DIRECT1 = 5,  /* direct term, conj(rho_vv') W(q)          */
    BSE_STAGE_DIRECT2 = 6,  /* direct term contraction + diagonal       */
    BSE_STAGE_MIRROR = 7,   /* lower blocks from the upper ones         */
    BSE_STAGE_ROTATE = 8,   /* wave functions transposed for grids whose
                               long axis is last (pair-density frame)    */
    BSE_STAGE_TR_FILL = 9,  /* BSE_TIME_REVERSAL: pair densities of the
                               image pairs                               */
    BSE_STAGE_TO_F32 = 10,  /* BSE_FP32_PAIRDENS: FP32 copy of u          */
    BSE_STAGE_SPLIT_W = 11, /* mixed precisions: W(q) and the valence
                               pair densities split into parts once per
                               call for the first stage of the direct term */
    BSE_NSTAGES = 12
};
int bse_profile(int enable);
int bse_profile_read(double *total_ms, long long *launches, int nstages, int reset);

/* Budget of the per-pair arrays of a build: the k pairs k <= k' of a batch
 * are processed in chunks (ranges of block rows of H) whose valence and
 * conduction pair densities, first-stage products and, in the mixed
 * precisions, split operands take about `bytes` together (0 = the default,
 * 6 GiB).  Smaller budgets need less workspace and launch more, smaller
 * kernels; H does not depend on it.  Applies to the plans made after the call
 * (bse_workspace_size included), for every thread. */
int bse_set_chunk_budget(size_t bytes);

/* Frees the calling thread's pinned staging buffer and plan cache (after
 * waiting for the copies that read the buffer) and forgets every tuned launch
 * choice; the next call rebuilds what it needs. */
int bse_release_host_state(void);

/* Text describing the last non-zero status returned on this thread. */
const char *bse_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BSE_H */
