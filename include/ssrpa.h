/*
 * ssrpa.h -- C ABI of the static-subspace RPA hot path on AMD MI355X (gfx950).
 *
 * The library computes the random-phase-approximation correlation energy of a
 * plane-wave system at one q-point (q = 0) and the Gamma point, following the
 * Method section of Weinberg et al., "Static Subspace Approximation for Random
 * Phase Approximation Correlation Energies: Implementation and Performance"
 * (arXiv:2405.20258):
 *
 *   orbitals psi_n(G), energies e_n, cell, chi0 cutoff       (problem statement)
 *   -> pair matrix elements M_vc(G) by batched 3-D FFTs      (Eq. 3)
 *   -> static chi0(G,G'; 0) = M^H Delta M / Omega, streamed over valence
 *      blocks                                               (Eqs. 6, 15)
 *   -> the N_eig eigenvectors of v^1/2 chi0 v^1/2 with the largest |eigenvalue|
 *      (static subspace)
 *   -> chi0_s(i w_j) = M_s^H Delta(i w_j) M_s in that subspace (Eqs. 7, 8)
 *   -> F_j = ln det(1 - chi0_s v) + Tr chi0_s v, from a triangular factor
 *   -> E_c = (1/2 pi) sum_j w_j F_j                          (Eq. 1)
 *
 * Conventions (Hartree atomic units throughout):
 *  - Valence bands 0..n_v-1 have occupation 1, conduction bands n_v..n_b-1
 *    occupation 0, unless occupation factors are given (partial occupations,
 *    Eqs. 4-6; see ssrpa_system_desc); spin degeneracy 2; one k-point of
 *    weight 1.
 *  - Delta_vc(i w) = -4 (e_c - e_v) / ((e_c - e_v)^2 + w^2): the resonant and
 *    anti-resonant terms of Eq. (2) together, so chi0 is Hermitian and
 *    negative semidefinite at every imaginary frequency.
 *  - M_vc(G) = <psi_v| e^{+iG.r} |psi_c>; chi0_GG' = (1/Omega) sum_vc
 *    conj(M_vc(G)) Delta_vc M_vc(G') (Eq. 6), with 1/Omega exactly once.
 *  - v(G) = 4 pi / |G|^2 (or its slab-truncated form, see
 *    ssrpa_system_desc); the symmetrized matrix is v^1/2 chi0 v^1/2.
 *  - The chi0 basis is {G != 0 : |G|^2 / 2 <= ecut_chi}, in the order reported
 *    by ssrpa_chi_gvectors (lexicographic in the Miller indices).
 *
 * Memory and ownership:
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *    memory on the context's device (e.g. torch tensor data_ptr()).
 *  - The caller owns every buffer it passes in; the library never frees or
 *    keeps caller pointers beyond the call.  The library owns a device copy of
 *    the orbitals and all workspace (within the context's HBM budget) until
 *    the matching *_destroy.
 *  - Complex arrays are interleaved (re, im) doubles, row-major.
 *  - Calls are ordered on the HIP stream passed in (NULL = the default
 *    stream).  Host outputs are valid when a call returns; device outputs are
 *    valid once the stream has reached the call's end.
 *
 * Errors: every entry point returns an ssrpa_status; none throws or aborts.
 * A failed call leaves the system usable, except after SSRPA_ERR_HIP (a HIP
 * runtime error), after which the context should be destroyed.  The text of
 * the last error of a context is available from ssrpa_last_error.
 * A context may be shared by threads that work on different systems (the
 * memory accounting is locked); one system must not be used by two threads
 * at once.
 */
#ifndef SSRPA_H
#define SSRPA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSRPA_API __attribute__((visibility("default")))

typedef enum ssrpa_status {
  SSRPA_OK = 0,
  SSRPA_ERR_ARG = 1,      /* invalid argument (null, size, range)            */
  SSRPA_ERR_ALIAS = 2,    /* FFT grid below the alias-free bound             */
  SSRPA_ERR_NOMEM = 3,    /* HBM budget or device allocation exhausted       */
  SSRPA_ERR_HIP = 4,      /* HIP runtime error                               */
  SSRPA_ERR_NUMERIC = 5,  /* factorization failed (matrix not positive etc.) */
  SSRPA_ERR_STATE = 6     /* call order (e.g. no subspace yet)               */
} ssrpa_status;

/* Arithmetic of the chi0 / projection / subspace contractions.  The static
 * eigendecomposition and the per-frequency log-determinant are always FP64. */
typedef enum ssrpa_precision {
  SSRPA_FP64 = 0,    /* FP64 MFMA, FP64 accumulation                          */
  SSRPA_FP32 = 1,    /* FP32 MFMA, FP32 accumulation per K chunk, FP64 across  */
  SSRPA_BF16X3 = 2   /* x = hi + lo in bfloat16; hi*hi + hi*lo + lo*hi on BF16
                        MFMA, FP32 accumulation per K chunk, FP64 across       */
} ssrpa_precision;

typedef struct ssrpa_context ssrpa_context;
typedef struct ssrpa_system ssrpa_system;
typedef struct ssrpa_ticket ssrpa_ticket;

/* The problem statement: orbitals in a plane-wave basis with their energies,
 * the cell, the FFT grid and the chi0 cutoff (Method section, Eqs. 2-3). */
typedef struct ssrpa_system_desc {
  double lattice[9];      /* bohr; rows are a1, a2, a3                        */
  int32_t fft[3];         /* N1, N2, N3, each 2^i 3^j <= 128; must satisfy
                             N_i >= 2 max|n_psi,i| + max|n_chi,i| + 1, else
                             SSRPA_ERR_ALIAS                                  */
  int32_t n_pw;           /* wavefunction plane waves                         */
  const int32_t *miller;  /* host, n_pw x 3 Miller indices of the plane waves */
  int32_t n_v;            /* valence bands: occupied (and, with occupation,
                             partially occupied) bands 0..n_v-1              */
  int32_t n_c;            /* the remaining bands n_v..n_v+n_c-1               */
  const double *coeff;    /* (n_v + n_c) x n_pw complex, one band per row;
                             orthonormal rows; host or device (see below)     */
  int32_t coeff_on_device;/* 0: coeff is host memory, 1: device memory        */
  const double *energy;   /* host, n_v + n_c band energies (Ha); without
                             occupation each energy of bands >= n_v lies above
                             every energy of bands < n_v                      */
  double ecut_chi;        /* Ha; chi0 basis {G != 0 : |G|^2/2 <= ecut_chi}     */
  const double *occupation; /* host, n_v + n_c occupation factors f_n, or
                             NULL for an insulator (f = 1 below n_v, 0 from
                             n_v on).  Partial occupations (Method, Eqs. 4-6):
                             f_n in [0, 1], non-increasing along the bands,
                             energies non-decreasing and bands of equal energy
                             with equal f; n_v = the number of bands with
                             f > 0.  The valence set is {f > 0}, the
                             conduction set {f < 1}; a pair of two partially
                             occupied bands counts once (lower band as v),
                             and Delta_vc(i w) = -4 (f_v - f_c) de /
                             (de^2 + w^2).  SSRPA_ERR_ARG otherwise.          */
  int32_t coulomb_truncation; /* 0: bare v(G) = 4 pi / |G|^2.  1: slab
                             truncation along a3 (Computational Details: for
                             surfaces the interaction is cut along the axis
                             normal to the slab): v(G) = 4 pi / |G|^2
                             [1 - exp(-G_par z_c) cos(G_z z_c)], z_c = |a3|/2,
                             G_z = G . a3/|a3|, G_par the rest; a3 must be
                             normal to a1 and a2 (else SSRPA_ERR_ARG).  G
                             with v(G) = 0 drop out of v^1/2 chi0 v^1/2.      */
  int32_t real_orbitals;  /* 1: the orbitals are real (c(-G) = conj c(G) for
                             every plane wave, within 1e-10; time-reversal
                             symmetric orbitals at the Gamma point).  The
                             pair densities are then real: two conduction
                             orbitals share one complex pair transform, and
                             chi0, the subspace and the frequency
                             contractions work in the real cos/sin basis of
                             the chi0 set (a quarter of the complex flops).
                             FP64 contractions only.  The plane-wave set must
                             hold -G with every G.  Outputs are reported in
                             the plane-wave basis except chi_sub (cos/sin
                             basis for n_eig >= N_G).  0: general complex.   */
} ssrpa_system_desc;

/* Human-readable name of a status code (static string). */
SSRPA_API const char *ssrpa_status_string(ssrpa_status s);

/* Text of the most recent error of a call on this context made by the
 * calling thread ("" if that call succeeded). */
SSRPA_API const char *ssrpa_last_error(const ssrpa_context *ctx);

/* Library version string, e.g. "0.1.0 gfx950". */
SSRPA_API const char *ssrpa_version(void);

/* Create a context on HIP device `hip_device`.  `hbm_budget_bytes` caps the
 * device memory the library allocates for this context (0 = 90% of the
 * device's free memory at creation).  *out receives the handle. */
SSRPA_API ssrpa_status ssrpa_context_create(int hip_device,
                                            size_t hbm_budget_bytes,
                                            ssrpa_context **out);
/* Destroy a context; SSRPA_ERR_STATE (and nothing freed) while systems
 * created on it are still alive. */
SSRPA_API ssrpa_status ssrpa_context_destroy(ssrpa_context *ctx);

/* Device bytes held by this context (live plus cached blocks) and the
 * high-water mark of live allocations. */
SSRPA_API ssrpa_status ssrpa_context_memory(const ssrpa_context *ctx,
                                            size_t *in_use, size_t *high_water);

/* Device footprint (bytes) of a whole E_c solve for `desc` with `n_eig`
 * subspace vectors (n_eig >= N_G: full basis), `n_freq` frequencies, the
 * given precision and `valence_block` valence bands per block (0: all).
 * Host-only; touches no device.  The valence-block algorithm (Eqs. 14-15)
 * bounds the pair-matrix part of this number by the block size. */
SSRPA_API ssrpa_status ssrpa_footprint(const ssrpa_system_desc *desc,
                                       int n_eig, int n_freq,
                                       ssrpa_precision precision,
                                       int valence_block, size_t *bytes);

/* Largest valence block (<= n_v) whose footprint fits `budget_bytes`;
 * 0 in *valence_block (and SSRPA_ERR_NOMEM) if even one band does not fit. */
SSRPA_API ssrpa_status ssrpa_plan_valence_block(const ssrpa_system_desc *desc,
                                                int n_eig, int n_freq,
                                                ssrpa_precision precision,
                                                size_t budget_bytes,
                                                int *valence_block);

/* Validate `desc`, build the chi0 G set, copy the orbitals to the device and
 * transform them to the real-space grid (orbital staging; the wavefunctions
 * stay resident, as in the valence-block algorithm where they are the
 * memory floor).  Enqueued on `hip_stream` and synchronized before return. */
SSRPA_API ssrpa_status ssrpa_system_create(ssrpa_context *ctx,
                                           const ssrpa_system_desc *desc,
                                           void *hip_stream,
                                           ssrpa_system **out);
SSRPA_API ssrpa_status ssrpa_system_destroy(ssrpa_system *sys);

/* The band sets of a system (Method, Eqs. 4-6): *n_val valence bands
 * 0..n_val-1 (f > 0) and *n_cond conduction bands c_first..c_first+n_cond-1
 * (f < 1).  Pair rows of a valence block are p = (v - v0) n_cond + c with
 * band c_first + c.  Insulator: c_first = n_val.  Nullable outputs. */
SSRPA_API ssrpa_status ssrpa_system_bands(const ssrpa_system *sys, int *n_val,
                                          int *c_first, int *n_cond);

/* Number of chi0 basis vectors N_G and (if `miller` is not NULL) their host
 * n_g x 3 Miller indices in the library's order. */
SSRPA_API ssrpa_status ssrpa_chi_gvectors(const ssrpa_system *sys, int *n_g,
                                          int32_t *miller);

/* Real-space orbitals psi_n(r_j) = Omega^-1/2 sum_G c_n(G) e^{iG.r_j} on the
 * grid r_j = j1/N1 a1 + j2/N2 a2 + j3/N3 a3, written to device memory `psi`
 * as (n_v + n_c) x N3 x N2 x N1 complex (j1 fastest). */
SSRPA_API ssrpa_status ssrpa_orbitals_realspace(ssrpa_system *sys, double *psi,
                                                void *hip_stream);

/* Pair matrix elements of Eq. (3) for valence bands v0..v0+n_vb-1 and every
 * conduction band: device output `m`, (n_vb * n_c) x N_G complex with row
 * p = (v - v0) * n_c + c.  scaled = 1 multiplies by v(G)^1/2 (the W used by
 * the contractions), scaled = 0 gives M itself. */
SSRPA_API ssrpa_status ssrpa_pair_matrix(ssrpa_system *sys, int v0, int n_vb,
                                         int scaled, double *m,
                                         void *hip_stream);

/* Static polarizability chi0(G, G'; i0) of Eq. (6), accumulated over valence
 * blocks of `valence_block` bands (0: automatic from the HBM budget), Eq. (15).
 * The symmetrized matrix stays resident for ssrpa_subspace.  If `chi0` is not
 * NULL it receives the N_G x N_G complex device matrix: the paper's chi0
 * (with 1/Omega) if symmetrized = 0, v^1/2 chi0 v^1/2 if symmetrized = 1. */
SSRPA_API ssrpa_status ssrpa_chi0_static(ssrpa_system *sys,
                                         ssrpa_precision precision,
                                         int valence_block, double *chi0,
                                         int symmetrized, void *hip_stream);

/* Static subspace: the n_eig eigenpairs of the resident v^1/2 chi0 v^1/2 with
 * the largest |eigenvalue| (the most negative), computed in FP64 on the GPU.
 * `eigval` (host, n_eig) receives them in ascending order; `basis` (device,
 * nullable) the N_G x n_eig complex eigenvector columns C_s.  Requires
 * ssrpa_chi0_static first (SSRPA_ERR_STATE otherwise). 1 <= n_eig <= N_G. */
SSRPA_API ssrpa_status ssrpa_subspace(ssrpa_system *sys, int n_eig,
                                      double *eigval, double *basis,
                                      void *hip_stream);

/* Which static matrix defines the subspace basis (Method, static subspace
 * paragraph).  SYMMETRIZED: eigenvectors of v^1/2 chi0 v^1/2 (then
 * Tr ln(1 - chi0 v) = ln det(I - X) with X the projected symmetrized
 * matrix).  CHI0: eigenvectors of chi0 itself, as the paper states; the
 * Coulomb kernel is then projected too, v_s = C_s^H v C_s = Z Z^H, and
 * det(1 - chi0_s v_s) = det(I - Z^H chi0_s Z), so X = Z^H chi0_s Z. */
typedef enum ssrpa_basis {
  SSRPA_BASIS_SYMMETRIZED = 0,
  SSRPA_BASIS_CHI0 = 1
} ssrpa_basis;

/* ssrpa_subspace with a choice of basis.  For SSRPA_BASIS_CHI0 `eigval`
 * receives the n_eig most negative eigenvalues of the paper's chi0 (with
 * 1/Omega) and `basis` its eigenvectors; the later ssrpa_correlation_energy
 * and ssrpa_epsilon_inverse use the projected kernel v_s.
 * SSRPA_ERR_ARG for an unknown kind. */
SSRPA_API ssrpa_status ssrpa_subspace_basis(ssrpa_system *sys, ssrpa_basis kind,
                                            int n_eig, double *eigval,
                                            double *basis, void *hip_stream);

/* Correlation energy by quadrature of Eq. (1) over `n_freq` imaginary
 * frequencies `omega` (host, Ha) with weights `weight` (host).
 *  n_eig < N_G: static-subspace form; requires ssrpa_subspace(sys, n_eig, ..)
 *               first (SSRPA_ERR_STATE otherwise).
 *  n_eig >= N_G: full G basis (no subspace needed).
 * `coupling` scales the interaction (1.0 for RPA; F_j = ln det(1 - l X) +
 * l Tr X).  Outputs: *ec (host); integrand (host, nullable) the n_freq values
 * F_j; chi_sub (device, nullable) the n_freq x n x n complex matrices
 * v^1/2 chi0_s(i w_j) v^1/2 (n = min(n_eig, N_G)).  Precision applies to the
 * projection and per-frequency contractions; the pair matrix is recomputed
 * per valence block when there is more than one block. */
SSRPA_API ssrpa_status ssrpa_correlation_energy(ssrpa_system *sys, int n_eig,
                                                int n_freq, const double *omega,
                                                const double *weight,
                                                ssrpa_precision precision,
                                                int valence_block,
                                                double coupling, double *ec,
                                                double *integrand,
                                                double *chi_sub,
                                                void *hip_stream);

/* Inverse dielectric matrices eps^-1(i w_j) = (I - X_j)^-1 (Implementation
 * section, last paragraph: the factorization of 1 - chi0 v also gives
 * eps^-1 for later GW steps).  X_j is the matrix that
 * ssrpa_correlation_energy returns in chi_sub: v^1/2 chi0 v^1/2 in the full
 * basis (n_eig >= N_G) or projected onto the current subspace (n_eig < N_G,
 * after ssrpa_subspace / ssrpa_subspace_basis).  eps_inv: device,
 * n_freq x n x n complex, n = min(n_eig, N_G); by Gauss-Jordan elimination
 * in FP64 on the GPU.  In the G basis the subspace form reads
 * eps^-1 = I + C_s (eps_s^-1 - I) C_s^H.  SSRPA_ERR_NUMERIC if some
 * I - X_j is not positive definite. */
SSRPA_API ssrpa_status ssrpa_epsilon_inverse(ssrpa_system *sys, int n_eig,
                                             int n_freq, const double *omega,
                                             ssrpa_precision precision,
                                             int valence_block, double *eps_inv,
                                             void *hip_stream);

/* F_j = ln det(I - l X_j) + l Tr X_j for a batch of Hermitian matrices X_j
 * (device, n_mat x n x n complex), by Cholesky factors in FP64 on the GPU.
 * `f` is host memory (n_mat).  SSRPA_ERR_NUMERIC if some I - l X_j is not
 * positive definite.  The per-frequency step of the correlation energy,
 * exposed for direct use. */
SSRPA_API ssrpa_status ssrpa_trace_log(ssrpa_context *ctx, const double *x,
                                       int n, int n_mat, double coupling,
                                       double *f, void *hip_stream);

/* Allocation-free form of ssrpa_trace_log, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same kernels and the same F_j; the work memory
 * (the n_mat factor copies, pivots and failure marks:
 * 16 n^2 n_mat + 8 n n_mat + 4 n_mat bytes, each part rounded up to 256)
 * lives in a fixed 64 MiB device array per GPU, set up when a context is
 * created on that GPU and held until the process ends.
 *  x:    device, n_mat x n x n complex (Hermitian), not modified.
 *  f:    device, n_mat doubles; F_j, or NaN where I - l X_j is not positive
 *        definite.
 *  flag: device int (nullable): 0, or nonzero if some factorization failed.
 * Nothing is allocated or synchronized: the results are valid once the
 * stream reaches the call's end.  SSRPA_ERR_ARG for a batch whose work
 * memory exceeds 64 MiB (nothing is launched).  All calls on one GPU share
 * the array, so calls that overlap on one GPU (different streams or
 * threads) race; serialize them on one stream. */
SSRPA_API ssrpa_status ssrpa_trace_log_noalloc(ssrpa_context *ctx,
                                               const double *x, int n,
                                               int n_mat, double coupling,
                                               double *f, int *flag,
                                               void *hip_stream);

/* Measurement aid, no step of the method: a plain device-to-device copy of
 * `bytes` (a multiple of 16; both pointers 16-byte aligned, device memory)
 * with 16-byte loads and stores, the access width of the contraction
 * kernels.  Its dispatch is the reference for scaling the beyond-L2 byte
 * counters (FETCH_SIZE, WRITE_SIZE) of the other kernels.  Returns after
 * the copy finished. */
SSRPA_API ssrpa_status ssrpa_device_copy(ssrpa_context *ctx, const void *src,
                                         void *dst, size_t bytes,
                                         void *hip_stream);

/* Gauss-Legendre rule with n points mapped to [0, inf) by
 * w = omega0 (1 + x)/(1 - x), weight 2 omega0 w_x / (1 - x)^2 (host). */
SSRPA_API ssrpa_status ssrpa_frequency_grid(int n, double omega0,
                                            double *omega, double *weight);

/* ---- stage timing ------------------------------------------------------- */

/* Stages of the path after system creation, timed with HIP events recorded
 * on the caller's stream around the kernels of each stage. */
typedef enum ssrpa_stage {
  SSRPA_STAGE_PAIR_FFT = 0,     /* pair densities -> M (Eq. 3), per block     */
  SSRPA_STAGE_CHI0_HERK = 1,    /* static chi0 contraction kernel (Eq. 6)     */
  SSRPA_STAGE_EIGEN = 2,        /* static subspace eigensolver                */
  SSRPA_STAGE_PROJECTION = 3,   /* M_s = M C_s (Eq. 7), per block             */
  SSRPA_STAGE_FREQ_HERK = 4,    /* per-frequency subspace contraction (Eq. 8) */
  SSRPA_STAGE_TRACE_LOG = 5,    /* log-determinants and quadrature            */
  SSRPA_N_STAGES = 6
} ssrpa_stage;

/* enable = 1 starts (and resets) event timing on this system, 0 stops it.
 * ms and launches (host, SSRPA_N_STAGES each, nullable) receive the time and
 * number of timed launches per stage accumulated since the last reset; the
 * call waits for the recorded events.  Timing adds one event pair per
 * launch and is off by default. */
SSRPA_API ssrpa_status ssrpa_stage_times(ssrpa_system *sys, int enable,
                                         double *ms, int *launches);

/* ---- k-point sampling and q != 0 (Eqs. 1-3 with the sums over k, q) ---- */

typedef struct ssrpa_kmesh ssrpa_kmesh;

/* A k mesh of n_k k-points for an insulator.  descs[i] holds the orbitals of
 * k-point i as plane-wave coefficients: psi_nk(r) = Omega^-1/2 sum_G
 * c_nk(G) e^{i(k+G).r}, `miller` the G (the sphere |k + G|^2/2 <= E_psi of
 * that k), bands 0..n_v-1 occupied.  All descriptions share lattice, FFT
 * grid, ecut_chi, n_v and n_c; occupation NULL, real_orbitals 0 and no
 * Coulomb truncation.  kfrac (host, n_k x 3): k in fractions of b1, b2, b3;
 * kweight (host, n_k): g_k of Eq. (2), >= 0 with at least one > 0; a
 * k-point of weight 0 adds no pairs of its own and serves only as a k + q
 * partner (for example the shifted points k + q0 of a small-q0 evaluation
 * of the q -> 0 term, whose basis then holds G = 0).  The orbitals are
 * staged once (their periodic parts u_nk on the grid) and stay resident. */
SSRPA_API ssrpa_status ssrpa_kmesh_create(ssrpa_context *ctx, int n_k,
                                          const ssrpa_system_desc *descs,
                                          const double *kfrac,
                                          const double *kweight,
                                          void *hip_stream, ssrpa_kmesh **out);
SSRPA_API ssrpa_status ssrpa_kmesh_destroy(ssrpa_kmesh *km);

/* The chi0 basis at q (fractions of b1, b2, b3): the G with
 * |G - q|^2 / 2 <= ecut_chi, G != q, lexicographic (see below for the sign
 * convention).  miller (host, nullable) n_g x 3.  A q on the reciprocal
 * lattice must be passed as q = 0 (SSRPA_ERR_ARG otherwise). */
SSRPA_API ssrpa_status ssrpa_kmesh_chi_gvectors(const ssrpa_kmesh *km,
                                                const double *q, int *n_g,
                                                int32_t *miller);

/* E_c(q), the q term of Eq. (1): kq[i] (n_k) and g0[i] (n_k x 3 ints) with
 * k_i + q = k_kq[i] + g0[i] for every k-point of nonzero weight (entries of
 * weight-0 points are not read).  Pair matrix with the bra
 * on the valence side, P_vc,k(q; G) = int u*_vk u_c,k+q e^{iG.r} (u_{k+q}
 * = e^{-iG0.r} u_kq[i]); Eq. (3)'s element is conj P(-G), so with
 * v(G - q) = 4 pi / |G - q|^2 the matrices are those of the paper at -G,
 * complex conjugated: the same eigenvalues, F_j and E_c(q).  chi0(q) =
 * (1/Omega) sum_k g_k sum_vc conj(P) Delta P with Delta the resonant plus
 * anti-resonant factor of reading Delta (exact for a time-reversal
 * symmetric k mesh).  n_eig < N_G(q): static subspace, else the full basis.
 * Outputs: *ec, integrand (host, nullable, n_freq), chi0 (device, nullable:
 * the static chi0(q), N_G x N_G interleaved complex, rows and columns in
 * ssrpa_kmesh_chi_gvectors order).  FP64.  Device work runs on hip_stream;
 * the call returns after it finished.  E_c = sum_q w_q E_c(q) is left to the caller.
 * SSRPA_ERR_ALIAS when N_i < 2 max|n_psi,i| + max|n_chi,i| + max|g0_i| + 1. */
SSRPA_API ssrpa_status ssrpa_kmesh_correlation_energy(
    ssrpa_kmesh *km, const double *q, const int32_t *kq, const int32_t *g0,
    int n_eig, int n_freq, const double *omega, const double *weight,
    double *ec, double *integrand, double *chi0, void *hip_stream);

/* Stage times of the mesh's ssrpa_kmesh_correlation_energy calls, as
 * ssrpa_stage_times for a system. */
SSRPA_API ssrpa_status ssrpa_kmesh_stage_times(ssrpa_kmesh *km, int enable,
                                               double *ms, int *launches);

/* ---- serving: the same solve, enqueued without blocking the caller ------ */

/* Start a whole E_c solve (system creation from `desc` is done by the
 * caller beforehand) on `hip_stream`, running the chi0 -> subspace -> E_c
 * stages on the device in stream order; returns at once with a ticket.
 * Different systems on different streams overlap on the device. */
SSRPA_API ssrpa_status ssrpa_correlation_energy_enqueue(
    ssrpa_system *sys, int n_eig, int n_freq, const double *omega,
    const double *weight, ssrpa_precision precision, int valence_block,
    void *hip_stream, ssrpa_ticket **ticket);

/* *done = 1 once the ticket's solve has finished (non-blocking). */
SSRPA_API ssrpa_status ssrpa_ticket_query(ssrpa_ticket *t, int *done);

/* Block until the solve finishes; write E_c and (nullable) the n_freq
 * integrand values; free the ticket.  Returns the solve's status. */
SSRPA_API ssrpa_status ssrpa_ticket_wait(ssrpa_ticket *t, double *ec,
                                         double *integrand);

/* ---- serving: a request loop with admission by HBM footprint ---------- */

typedef struct ssrpa_server ssrpa_server;

/* Request states reported by ssrpa_server_poll. */
enum { SSRPA_REQ_QUEUED = 0, SSRPA_REQ_RUNNING = 1, SSRPA_REQ_DONE = 2,
       SSRPA_REQ_FAILED = 3 };

/* A server owns `max_running` (1..64) worker threads over `ctx`, each with
 * one HIP stream (non-blocking, default priority) created here and destroyed
 * by ssrpa_server_destroy after the workers have been joined.  Submitted
 * requests wait in arrival order; a free worker admits the first waiting
 * request whose ssrpa_footprint fits the memory not yet reserved (budget
 * minus the footprints of running requests) and runs it (system creation,
 * static chi0, subspace, E_c) on its stream, so the device work of different
 * requests overlaps.  A request that has waited longer than `max_bypass_s`
 * seconds is not overtaken by later ones.  Each result is independent of the
 * mix: kernels and reduction orders depend only on the request's own sizes.
 * SSRPA_ERR_HIP if a stream or event cannot be created. */
SSRPA_API ssrpa_status ssrpa_server_create(ssrpa_context *ctx, int max_running,
                                           double max_bypass_s,
                                           ssrpa_server **out);

/* Queue one E_c solve.  The description's arrays, `omega` and `weight` are
 * copied (host memory only: coeff_on_device must be 0); n_eig >= N_G asks for
 * the full basis.  valence_block 0 picks the largest block that fits the
 * request's reservation.  *request_id identifies it for polling.
 * SSRPA_ERR_NOMEM if the request could never fit the context budget. */
SSRPA_API ssrpa_status ssrpa_server_submit(ssrpa_server *srv,
                                           const ssrpa_system_desc *desc,
                                           int n_eig, int n_freq,
                                           const double *omega,
                                           const double *weight,
                                           ssrpa_precision precision,
                                           uint64_t *request_id);

/* State of a request; when done, *ec and the times in seconds since the
 * server's creation (submit, admission to the device, completion).
 * Any output pointer may be NULL.  `status` receives the solve's status. */
SSRPA_API ssrpa_status ssrpa_server_poll(ssrpa_server *srv, uint64_t request_id,
                                         int *state, ssrpa_status *status,
                                         double *ec, double *t_submit,
                                         double *t_start, double *t_done);

/* Device times of a finished request, in milliseconds since the server was
 * created, from HIP events recorded on the request's stream before its first
 * and after its last device work (the device clock, so two requests whose
 * intervals intersect had work queued on the device at the same time).
 * SSRPA_ERR_STATE while the request has not finished; -1 if the events
 * could not be read. */
SSRPA_API ssrpa_status ssrpa_server_device_times(ssrpa_server *srv,
                                                 uint64_t request_id,
                                                 double *start_ms,
                                                 double *end_ms);

/* Error text of a failed request (the message of the call that failed);
 * "" for any other state or an unknown id.  Valid until the server is
 * destroyed. */
SSRPA_API const char *ssrpa_server_error(ssrpa_server *srv, uint64_t request_id);

/* Block until every submitted request has finished. */
SSRPA_API ssrpa_status ssrpa_server_drain(ssrpa_server *srv);

/* Peak device memory reserved by admitted requests (bytes), and the
 * context's measured high-water mark. */
SSRPA_API ssrpa_status ssrpa_server_memory(ssrpa_server *srv, size_t *reserved_peak,
                                           size_t *high_water);

/* Drain and destroy. */
SSRPA_API ssrpa_status ssrpa_server_destroy(ssrpa_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* SSRPA_H */
