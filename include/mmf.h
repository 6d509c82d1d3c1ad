/*
 * mmf.h -- C ABI of the MI355X multimode Floquet library (libmmf.so).
 *
 * Implements the computational path of G. A. Sinuco-Leon, "OPENMMF: a library
 * for multimode driven quantum systems" (arXiv:2005.03426):
 *   mmf_build_floquet  -- the truncated multimode Floquet matrix H_F
 *                         (Sec. 2, Eq. 6; block layout of Appendix A)
 *   mmf_eigh           -- its dense Hermitian eigendecomposition (Sec. 3.2,
 *                         the diagonalisation the paper delegates to LAPACK)
 *   mmf_evolve         -- the bare-basis time-evolution operator U(t,t0)
 *                         (Eqs. 3-5) from the eigenpairs
 *   mmf_micromotion    -- the micromotion operator U_F(t) (Eq. 5)
 *   mmf_avg_prob       -- time/phase-averaged transition probabilities
 *                         (multimodetransitionavg of the Python-wrapper example)
 * plus the stages of mmf_eigh (tridiagonal reduction, tridiagonal
 * divide-and-conquer, back-transformation) as separate calls.
 *
 * Conventions (all calls):
 *   - hbar = 1.  H(t) = E + sum_k [ V_k e^{+i h_k w_{l_k} t} + V_k^H e^{-i h_k w_{l_k} t} ]
 *     (Eq. 1 with harmonic couplings k = (axis l_k, harmonic h_k >= 1, V_k)).
 *   - Complex numbers are interleaved (re, im) doubles (mmf_z), identical in
 *     layout to std::complex<double> and torch.complex128.
 *   - Matrices are column-major with an explicit leading dimension (ld >= rows).
 *   - Floquet row index r = i + D*s, site s = sum_l (N_l - n_l) prod_{l'<l}(2N_{l'}+1):
 *     descending Fourier index, fundamental 0 innermost (Appendix A order).
 *   - "dev" pointers are device (HBM) memory owned by the caller; "host"
 *     pointers are host memory read during the call only.  The library never
 *     allocates or frees caller-visible memory and keeps no global state
 *     (apart from the opt-in benchmark timer at the end of this header):
 *     every call is reentrant.  Kernels are enqueued on `stream` (a
 *     hipStream_t, NULL = default stream) and the call returns without
 *     synchronising (a call that enqueues tens of thousands of launches,
 *     like the two-stage eigensolve, can wait for room in the launch queue:
 *     at M = 20808 it returns after about 1.6 s of a 5 s solve).  The two-stage band reduction (mmf_eigh,
 *     mmf_eigh_window, mmf_eigvalsh_batched at large orders) also uses a
 *     stream of its own (one per host thread and device, default priority,
 *     created on first use and kept), forked from and joined back into
 *     `stream` with per-call events: all its work is ordered after the
 *     earlier work of `stream` and before the later.
 *   - Return value: 0 on success; -k when argument k (1-based) is invalid
 *     (checked on the host before anything is enqueued); a positive MMF_ERR_*
 *     code on a runtime failure.  Numerical failures found on the device are
 *     reported through a device status word where a call has one.
 */
#ifndef MMF_H
#define MMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } mmf_z;

/* Problem statement (Eq. 1; the ATOM / MODES_NUMBER / MODE data of Sec. 3.1). */
typedef struct {
  int32_t D;            /* bare Hilbert-space dimension, 1 <= D <= 4096 (<= 64 for
                           mmf_evolve, mmf_micromotion, mmf_avg_prob: MMF_ERR_TOO_LARGE) */
  int32_t F;            /* number of incommensurate fundamentals, 0 <= F <= 8             */
  int32_t K;            /* number of harmonic couplings, 0 <= K <= 64                     */
  const double  *omega; /* host [F]: fundamental angular frequencies                      */
  const int32_t *N;     /* host [F]: truncation, n_l in [-N_l, N_l], N_l >= 0              */
  const int32_t *axis;  /* host [K]: fundamental index l_k in [0, F)                      */
  const int32_t *harm;  /* host [K]: harmonic order h_k >= 1                              */
  const mmf_z   *E;     /* host [D*D]: static Hamiltonian, column-major, Hermitian: an
                           imaginary part on the diagonal or |E_ij - conj(E_ji)| above
                           1e-14 max(1, max|E|) makes the problem invalid (-k)            */
  const mmf_z   *V;     /* host [K*D*D]: V_k column-major at offset k*D*D (any complex)   */
} mmf_problem;
/* The whole problem statement is host memory, read during a call only.  Only
 * mmf_build_floquet reads E and V (it stages them on the device); the other
 * calls use the sizes, frequencies and truncations. */

/* eigensolver precision */
enum {
  MMF_C128 = 0,          /* complex128 throughout                                        */
  MMF_C64_REFINED = 1,   /* complex64 reduction/back-transform + FP64 refinement          */
  MMF_C64_RAW = 2        /* complex64 reduction/back-transform, no refinement             */
};
/* MMF_C64_REFINED iterates (at most twelve times) until max |s_ij - lam_j g_ij|
 * <= 1e-13 max(1, max |lam|) and max |g_ij - delta_ij| <= 1e-12 for
 * S = X^H A X, G = X^H X; otherwise dev_info is set to MMF_ERR_NO_CONVERGENCE
 * and the last iterate is returned. */

/* positive error codes */
enum {
  MMF_OK = 0,
  MMF_ERR_HIP = 1,             /* a HIP runtime call failed                               */
  MMF_ERR_WORKSPACE = 2,       /* workspace smaller than the size query returned         */
  MMF_ERR_NOT_IMPLEMENTED = 3, /* option not available in this library                   */
  MMF_ERR_NO_CONVERGENCE = 4,  /* device status: an iteration did not converge           */
  MMF_ERR_SELECTION = 5,       /* micromotion: not exactly D orbit representatives found */
  MMF_ERR_TOO_LARGE = 6,       /* size beyond what the library supports                   */
  MMF_ERR_DEGENERATE = 7       /* device status of mmf_avg_prob: quasienergies closer than
                                  1e-8 max(1, max|w|) share weight on the zero Fourier site,
                                  so P depends on the eigenvector basis (no unique value)    */
};

/* Human-readable text for a return code (static storage). */
const char *mmf_strerror(int code);

/* Floquet dimension M = D * prod_l (2 N_l + 1) of problem p (host only).
 * Errors: -1 p NULL or malformed, -2 M NULL, MMF_ERR_TOO_LARGE if M > 2^31-1. */
int mmf_floquet_dim(const mmf_problem *p, int64_t *M);

/* Workspace bytes of mmf_build_floquet: the device copy of E and the V_k,
 * (1 + K) D^2 complex numbers.  Errors: -1 bad problem, -2 bytes NULL. */
int mmf_build_floquet_workspace(const mmf_problem *p, size_t *bytes);

/* Assemble H_F (Sec. 2, Eq. 6 with the conjugate term indexed U^{n-m};
 * Appendix A layout):
 *   HF[(i,n),(j,m)] = H^{[n-m]}_{ij} + delta_{nm} delta_{ij} (n . w),
 *   H^{[0]} = E, H^{[+h e_l]} = sum of V_k with (l_k,h_k) = (l,h) (ascending k),
 *   H^{[-h e_l]} = sum of V_k^H over the same k, zero otherwise.
 * The diagonal is evaluated as ((E_ii + n_0 w_0) + n_1 w_1) + ... in FP64.
 * All M x M entries are written (both triangles).
 * HF: dev, M x M, column-major, ldh >= M.
 * work: dev, at least mmf_build_floquet_workspace() bytes; E and V are copied
 * into it on `stream` (from pageable host memory: the host arrays may be
 * released when the call returns) and the assembly kernel reads them there.
 * Errors: -1 bad problem (including a non-Hermitian E, checked on the host),
 * -2 HF NULL, -3 ldh < M, -4/-5 workspace NULL or too small, MMF_ERR_HIP. */
int mmf_build_floquet(const mmf_problem *p, mmf_z *HF, int64_t ldh, void *work, size_t work_bytes,
                      void *stream);

/* mmf_build_floquet with E and V already on the device, laid out as its
 * workspace holds them after a call (E, then V_k at offset (1 + k) D^2,
 * column-major): no host copy is made, the call is one kernel launch (so it
 * can be recorded in a HIP graph).  p is validated as by mmf_build_floquet,
 * its host E included; EV is taken to hold the same matrices.
 * Errors: -1 bad problem, -2 EV NULL, -3 HF NULL, -4 ldh < M, MMF_ERR_HIP. */
int mmf_build_floquet_dev(const mmf_problem *p, const mmf_z *EV, mmf_z *HF, int64_t ldh, void *stream);

/* Batches of small problems (parameter sweeps): the assembly, U(t, t0) and
 * the averaged probabilities of `count` problems in a fixed number of launches
 * whatever the count (a device table of the problems, written per call with
 * kernel-argument launches of 14 entries each).  Problems: D <= 64, at most 4
 * fundamentals and 8 couplings (MMF_ERR_TOO_LARGE otherwise).  Results equal
 * the single calls' to rounding (other reduction order), not bitwise.
 *
 * Workspace bytes for both calls below (count problems, T times). */
int mmf_batched_workspace(int64_t count, const mmf_problem *p, int32_t T, size_t *bytes);

/* H_F of every problem c (Sec. 2, Eq. 6; as mmf_build_floquet_dev): p[c]
 * host problem statements (E validated), EV[c] device copies of E and V in
 * mmf_build_floquet's workspace layout, HF[c] dev M_c x M_c (ldh[c] >= M_c);
 * EV, HF, ldh are host arrays [count].  work: at least count * 272 bytes of
 * the mmf_batched_workspace size.
 * Errors: -1 count < 0, -2 a bad problem, -3 EV, -4 HF, -5 ldh, -6/-7
 * workspace NULL or too small, MMF_ERR_TOO_LARGE, MMF_ERR_HIP. */
int mmf_build_floquet_batched(int64_t count, const mmf_problem *p, const mmf_z *const *EV, mmf_z *const *HF,
                              const int64_t *ldh, void *work, size_t work_bytes, void *stream);

/* U(t_q, t0) at T times per problem and the averaged transition
 * probabilities (Eqs. 3-5; as mmf_evolve and mmf_avg_prob) for every problem
 * c: Phi[c] eigenvectors (ld[c]), w[c] ascending eigenvalues, t[c] dev [T]
 * times, U[c] dev [T][D*D], P[c] dev [D*D], dev_status [count] (0 or
 * MMF_ERR_DEGENERATE, as mmf_avg_prob).  Host arrays of device pointers.
 * D * T <= 2048.  work: mmf_batched_workspace(count, p, T) bytes.
 * Errors: -1 count, -2 problem, -3 Phi, -4 ld, -5 w, -7 T < 1, -8 t, -9 U,
 * -10 P, -11 dev_status, -12/-13 workspace, MMF_ERR_TOO_LARGE, MMF_ERR_HIP. */
int mmf_observables_batched(int64_t count, const mmf_problem *p, const mmf_z *const *Phi, const int64_t *ld,
                            const double *const *w, double t0, int32_t T, const double *const *t,
                            mmf_z *const *U, double *const *P, int32_t *dev_status, void *work,
                            size_t work_bytes, void *stream);

/* Workspace bytes that mmf_eigh needs for an M x M problem at precision prec. */
int mmf_eigh_workspace(int64_t M, int prec, size_t *bytes);

/* Dense Hermitian eigendecomposition A = Phi diag(w) Phi^H (Sec. 3.2).
 * A:   dev M x M, ld lda >= M; on entry the Hermitian matrix (only the lower
 *      triangle is read); on exit column a holds the orthonormal eigenvector
 *      of w[a] (the paper's U_F array).
 * w:   dev [M], eigenvalues in ascending order.
 * work/work_bytes: dev scratch of at least mmf_eigh_workspace() bytes.
 * dev_info: dev int32, set to 0 or to MMF_ERR_NO_CONVERGENCE by the kernels.
 * Method: order <= 64: one workgroup holding the matrix and its
 * eigenvectors in LDS, parallel cyclic Jacobi (complex128).  Above that:
 * Householder reduction to a real symmetric tridiagonal matrix,
 * Cuppen divide and conquer with Gu-Eisenstat eigenvector recomputation,
 * back-transformation.  Below order mmf_eigh_two_stage_min() the reduction is
 * one-stage (blocked, trailing updates and back-transformation on the FP64
 * matrix cores); from that order up it is two-stage: dense -> band of
 * half-width 64 (matrix-core GEMMs), band -> tridiagonal by bulge chasing,
 * then the two back-transformations.  Both give the same results to rounding.
 * Errors: -1 M < 0, -2 A NULL, -3 lda < M, -4 w NULL, -5 prec unknown,
 *         -6/-7 workspace NULL or too small, -8 dev_info NULL, MMF_ERR_HIP,
 *         MMF_ERR_NOT_IMPLEMENTED for a precision not built. */
int mmf_eigh(int64_t M, mmf_z *A, int64_t lda, double *w, int prec,
             void *work, size_t work_bytes, int32_t *dev_info, void *stream);

/* Iteration limits of the eigensolver (a zero field keeps its default).  For
 * callers that need a different budget, and for testing the failure report:
 * a limit that is reached sets dev_info to MMF_ERR_NO_CONVERGENCE. */
typedef struct {
  int32_t refine_max_iters;   /* MMF_C64_REFINED refinement iterations, default 12, at most 64 */
  int32_t secular_max_iters;  /* divide and conquer: steps per secular-equation root, default
                                 200, at most 100000                                            */
  int32_t leaf_max_iters;     /* divide and conquer: implicit-QL steps per eigenvalue of a leaf,
                                 default 60, at most 100000                                     */
} mmf_eigh_opts;

/* mmf_eigh with iteration limits (opts may be NULL: the defaults, identical
 * to mmf_eigh).  Arguments as for mmf_eigh with opts inserted after prec.
 * Errors: as mmf_eigh with the workspace, size and dev_info positions moved
 * to -7, -8 and -9; -6 a limit out of range. */
int mmf_eigh_ex(int64_t M, mmf_z *A, int64_t lda, double *w, int prec, const mmf_eigh_opts *opts,
                void *work, size_t work_bytes, int32_t *dev_info, void *stream);

/* Order from which mmf_eigh and mmf_eigh_window take the two-stage reduction
 * (default 5888, the measured crossover; the environment variable
 * MMF_EIGH_TWO_STAGE_MIN, read at every call, overrides it and also the
 * eigenvalue-only thresholds of mmf_eigvalsh_batched).  Query the workspace
 * size and call the solver under the same setting.  Host-only, never fails. */
int64_t mmf_eigh_two_stage_min(void);

/* Workspace bytes that mmf_eigh_batched needs for `count` problems of orders
 * n[0..count) (host array) at precision prec.
 * Errors: -1 count < 0, -2 n NULL or an n[c] < 0, -3 prec unknown, -4 bytes NULL. */
int mmf_eigh_batched_workspace(int64_t count, const int64_t *n, int prec, size_t *bytes);

/* Many independent eigendecompositions (Sec. 3.2) in one call, e.g. the
 * Floquet matrices of a parameter scan.  Problem c is exactly the mmf_eigh
 * problem (n[c], A[c], lda[c], w[c]) and gets the same result; the stages
 * run grouped, so each kernel launch advances every matrix of the batch
 * (sizes may differ; launches cover the largest).  Every problem takes the
 * grouped one-stage path, also from mmf_eigh_two_stage_min() up (where the
 * single call takes the two-stage path; the results then agree to rounding,
 * not bit for bit).
 * n, lda: host arrays [count]; A, w: host arrays [count] of device pointers
 *   (A[c] n[c] x n[c] column-major, lower triangle read, eigenvectors on
 *   exit; w[c] eigenvalues ascending).  Problems with n[c] = 0 are skipped.
 * work/work_bytes: dev scratch of at least mmf_eigh_batched_workspace().
 * dev_info: dev int32 [count]; entry c set to 0 or MMF_ERR_NO_CONVERGENCE.
 * The host arrays are read during the call only.
 * Errors: -1 count < 0, -2 n NULL or n[c] < 0, -3 A NULL or A[c] NULL,
 *   -4 lda NULL or lda[c] < max(1, n[c]), -5 w NULL or w[c] NULL, -6 prec
 *   unknown, -7/-8 workspace NULL or too small, -9 dev_info NULL, MMF_ERR_HIP. */
int mmf_eigh_batched(int64_t count, const int64_t *n, mmf_z *const *A, const int64_t *lda,
                     double *const *w, int prec, void *work, size_t work_bytes,
                     int32_t *dev_info, void *stream);

/* Tile table of the batched eigensolver, per order bucket b = (n - 1) / 8
 * (orders 1-8, 9-16, ..., 57-64): the workgroup size (64, 128, 256 or 512
 * threads) of the one-workgroup solver that keeps the whole matrix and its
 * eigenvectors in LDS (parallel cyclic Jacobi), or 0 to send the bucket to
 * the grouped Householder / divide-and-conquer path.  Written by the
 * project's autotuner from measurements (paper_2005_03426_amd/autotune.py);
 * without one the library uses 64 threads up to order 16, 128 up to 32 and
 * 256 up to 64 (the same rule mmf_eigh applies to a single matrix of order
 * <= 64). */
typedef struct {
  int32_t small_threads[8];
} mmf_batch_opts;

/* mmf_eigh_batched with a tile table (opts NULL: the built-in rule).
 * complex128 problems whose bucket has a nonzero entry are solved by one
 * persistent launch per workgroup size: its workgroups take problems from a
 * device work queue (largest first), each with its matrix in LDS.  The
 * eigenpairs agree with the other path's to rounding (not bitwise).
 * Arguments as for mmf_eigh_batched with opts inserted after prec.
 * Errors: as mmf_eigh_batched, with -7 an invalid table entry and the
 * workspace, size and dev_info positions moved to -8, -9 and -10. */
int mmf_eigh_batched_ex(int64_t count, const int64_t *n, mmf_z *const *A, const int64_t *lda,
                        double *const *w, int prec, const mmf_batch_opts *opts, void *work, size_t work_bytes,
                        int32_t *dev_info, void *stream);

/* Workspace bytes of mmf_eigh_window for order M and at most kmax vectors. */
int mmf_eigh_window_workspace(int64_t M, int64_t kmax, size_t *bytes);

/* Partial spectrum (Sec. 3.2 restricted to a quasienergy window, the role of
 * the paper's sparse partial-spectrum path): the eigenvalues of the Hermitian
 * A in [vl, vu) and their eigenvectors.  Reduction and divide and conquer run
 * as in mmf_eigh; only the window's k columns are back-transformed (8 M^2 k
 * instead of 8 M^3 real flops).  For a single-drive Floquet matrix the window
 * [-w/2, w/2) holds one state per Fourier orbit (the Floquet states).
 * A: dev M x M (lda), lower triangle read, destroyed (reflectors).
 * w: dev [kmax] ascending eigenvalues of the window; Z: dev M x kmax (ldz),
 * column t the eigenvector of w[t]; count: dev int32, the number k of
 * eigenvalues in the window (only min(k, kmax) are returned; columns beyond
 * that are zero).  dev_info as for mmf_eigh.
 * Errors: -1 M < 0, -2 A NULL, -3 lda, -4 not vl < vu, -6 kmax < 0, -7 w NULL,
 *   -8 Z NULL, -9 ldz < M, -10 count NULL, -11/-12 workspace, -13 dev_info NULL. */
int mmf_eigh_window(int64_t M, mmf_z *A, int64_t lda, double vl, double vu, int64_t kmax,
                    double *w, mmf_z *Z, int64_t ldz, int32_t *count, void *work,
                    size_t work_bytes, int32_t *dev_info, void *stream);

/* Workspace bytes of mmf_eigh_band for order M and half-bandwidth b.
 * Errors: -1 M < 0, -2 b < 0, -3 bytes NULL. */
int mmf_eigh_band_workspace(int64_t M, int64_t b, size_t *bytes);

/* Band-aware eigendecomposition (Sec. 3.2; the band half of the paper's sparse
 * path): mmf_eigh (complex128) for a Hermitian A whose entries vanish below
 * its b-th subdiagonal, b stated by the caller (entries beyond it are not
 * read).  A Floquet matrix of one drive with harmonics up to h is banded with
 * b = D h + D - 1 (Eq. 6 in the block order of App. A).  With b <= 64 and
 * M > 64 the band goes straight to the bulge chase of the two-stage solver: no dense ->
 * band stage and no first back-transformation, so the eigensolve costs the
 * chase, divide and conquer and the 8 M^3 of the second back-transformation.
 * Otherwise the call is mmf_eigh with prec MMF_C128.  A: dev M x M (lda),
 * lower band read; on exit column a holds the eigenvector of w[a].
 * w: dev [M] ascending.  dev_info as for mmf_eigh.
 * Errors: -1 M < 0, -2 A NULL, -3 lda < M, -4 b < 0, -5 w NULL, -6/-7
 * workspace NULL or too small, -8 dev_info NULL, MMF_ERR_HIP. */
int mmf_eigh_band(int64_t M, mmf_z *A, int64_t lda, int64_t b, double *w, void *work, size_t work_bytes,
                  int32_t *dev_info, void *stream);

/* Workspace bytes of mmf_eigh_band_window for order M, half-bandwidth b and at
 * most kmax vectors.  Errors: -1 M < 0, -2 b < 0, -3 kmax < 0, -4 bytes NULL. */
int mmf_eigh_band_window_workspace(int64_t M, int64_t b, int64_t kmax, size_t *bytes);

/* Partial spectrum of a banded Hermitian matrix (Sec. 3.2: both halves of the
 * paper's sparse path): mmf_eigh_window for an A whose entries vanish below
 * its b-th subdiagonal.  With b <= 64 and M > 64 the band goes straight to the
 * bulge chase and only the window's k eigenvectors are back-transformed by the
 * chase reflectors (8 M^2 k flops, nothing else of order M^3), and A is only
 * read; otherwise the call is mmf_eigh_window (which destroys A).  Arguments
 * as for mmf_eigh_window with b after lda.
 * Errors: -1 M < 0, -2 A NULL, -3 lda, -4 b < 0, -5 not vl < vu, -7 kmax < 0,
 *   -8 w NULL, -9 Z NULL, -10 ldz < M, -11 count NULL, -12/-13 workspace,
 *   -14 dev_info NULL. */
int mmf_eigh_band_window(int64_t M, const mmf_z *A, int64_t lda, int64_t b, double vl, double vu, int64_t kmax,
                         double *w, mmf_z *Z, int64_t ldz, int32_t *count, void *work, size_t work_bytes,
                         int32_t *dev_info, void *stream);

/* Workspace bytes that mmf_eigvalsh_batched needs (count, n as for
 * mmf_eigh_batched_workspace; prec MMF_C128 or MMF_C64_RAW).
 * Errors: -1 count < 0, -2 n NULL or an n[c] < 0, -3 prec unsupported, -4 bytes NULL. */
int mmf_eigvalsh_batched_workspace(int64_t count, const int64_t *n, int prec, size_t *bytes);

/* Eigenvalues only of many Hermitian matrices (Sec. 3.2 without the
 * eigenvectors; the quasienergy scans of Sec. 4.2): each A[c] (n[c] x n[c],
 * lower triangle read, destroyed) is reduced to a real tridiagonal matrix by
 * the grouped Householder reduction (complex128, or complex64 for
 * MMF_C64_RAW, from a complex64 copy; A[c] then stays intact; complex128
 * problems take the grouped two-stage reduction, dense -> band ->
 * tridiagonal, from order 4608 up, or from 1280 up when the call holds at
 * least 8 problems of order >= 1280), and all
 * eigenvalues are found by bisection on Sturm counts in FP64; w[c] receives
 * them in ascending order.  Arguments, ownership and errors as for
 * mmf_eigh_batched (-6: prec not MMF_C128 / MMF_C64_RAW); dev_info[c] is set
 * to 0. */
int mmf_eigvalsh_batched(int64_t count, const int64_t *n, mmf_z *const *A, const int64_t *lda,
                         double *const *w, int prec, void *work, size_t work_bytes,
                         int32_t *dev_info, void *stream);

/* Stage 1 of mmf_eigh: Householder reduction Q^H A Q = T with T real
 * symmetric tridiagonal.  On exit d[n] (dev) is the diagonal, e[n-1] (dev) the
 * off-diagonal, the reflector v_i (v_i[i+1] = 1, zero above) is stored in
 * A[i+1:, i] and tau[n-1] (dev, complex) holds its scalar, so that
 * Q = H_0 H_1 ... H_{n-2}, H_i = I - tau_i v_i v_i^H.
 * work: at least mmf_eigh_workspace(n, MMF_C128) bytes. */
int mmf_hetrd(int64_t n, mmf_z *A, int64_t lda, double *d, double *e, mmf_z *tau,
              void *work, size_t work_bytes, void *stream);

/* Stage 2: eigenpairs of the real symmetric tridiagonal matrix (d, e):
 * on exit d holds the eigenvalues ascending and Z (dev, n x n, ldz >= n,
 * real) the orthonormal eigenvectors.  e is not modified.
 * work: at least mmf_eigh_workspace(n, MMF_C128) bytes. */
int mmf_stedc(int64_t n, double *d, const double *e, double *Z, int64_t ldz,
              void *work, size_t work_bytes, int32_t *dev_info, void *stream);

/* Stage 3: Phi = Q Z for the reflectors left by mmf_hetrd in V (dev, n x n,
 * ldv) and tau; Z real n x n (ldz); Phi (dev, n x n, ldphi) must not overlap
 * V or Z.  work: at least mmf_eigh_workspace(n, MMF_C128) bytes. */
int mmf_unmtr(int64_t n, const mmf_z *V, int64_t ldv, const mmf_z *tau,
              const double *Z, int64_t ldz, mmf_z *Phi, int64_t ldphi,
              void *work, size_t work_bytes, void *stream);

/* Workspace bytes for mmf_evolve / mmf_micromotion with T times. */
int mmf_evolve_workspace(const mmf_problem *p, int32_t T, size_t *bytes);

/* Bare-basis time-evolution operators (Eqs. 3-5 over all M eigenpairs):
 *   U_ij(t,t0) = sum_n e^{i n.w t} sum_a Phi[(i,n),a] e^{-i w_a (t-t0)} conj(Phi[(j,0),a])
 * Phi: dev M x M eigenvectors (ld), w: dev [M] eigenvalues, t: dev [T] times,
 * U: dev [T][D*D], U[tau*D*D + i + D*j] (i final state, j initial state).
 * Errors: -1 problem, -2 Phi, -3 ld, -4 w, -6 T < 0, -7 t, -8 U, -9/-10 workspace. */
int mmf_evolve(const mmf_problem *p, const mmf_z *Phi, int64_t ld, const double *w,
               double t0, int32_t T, const double *t, mmf_z *U,
               void *work, size_t work_bytes, void *stream);

/* Micromotion operator (Eq. 5) U_F(t)_{ib} = sum_n Phi[(i,n),b] e^{i n.w t} over
 * one eigenvector b per w-translation orbit: the columns whose Fourier centre
 * of mass sum_n n sum_i |Phi[(i,n),b]|^2 rounds (half away from zero) to the
 * zero vector; if more than D qualify the D of smallest |w_b| (ties: lower b).
 * UF: dev [T][D*D] (UF[tau*D*D + i + D*b]); eps_sel: dev [D] (ascending b);
 * sel: dev int32 [D] selected columns; dev_info: dev int32, 0 or
 * MMF_ERR_SELECTION when fewer than D columns qualify. */
int mmf_micromotion(const mmf_problem *p, const mmf_z *Phi, int64_t ld, const double *w,
                    int32_t T, const double *t, mmf_z *UF, double *eps_sel, int32_t *sel,
                    void *work, size_t work_bytes, int32_t *dev_info, void *stream);

/* Evolution in a dressed basis (Sec. 4.1: the basis of a subset of the modes,
 * Eq. 4 with that subset's micromotion operator):
 *   Ud[q] = UF2[q]^H  U[q]  UF1,   q = 0 .. T-1,
 * UF2: dev [T][D*D] micromotion operator of the dressing subset at the times
 *      t_q (mmf_micromotion of the subset problem, same layout);
 * U:   dev [T][D*D] bare evolution U(t_q, t1) of the full problem (mmf_evolve);
 * UF1: dev [D*D]    micromotion operator of the dressing subset at t1;
 * Ud:  dev [T][D*D] output (Ud[q*D*D + i + D*j], i final, j initial dressed state).
 * Errors: -1 D outside [1, 64], -2 T < 0, -3..-6 a NULL pointer, MMF_ERR_HIP. */
int mmf_dressed_evolution(int32_t D, int32_t T, const mmf_z *UF2, const mmf_z *U,
                          const mmf_z *UF1, mmf_z *Ud, void *stream);

/* Workspace bytes for mmf_avg_prob. */
int mmf_avg_prob_workspace(const mmf_problem *p, size_t *bytes);

/* Time- and drive-phase-averaged transition probabilities:
 *   P[i + D*j] = sum_a ( sum_n |Phi[(i,n),a]|^2 ) |Phi[(j,0),a]|^2
 * (long-time average of |U_ij|^2 for a nondegenerate quasienergy spectrum;
 * columns sum to one for any orthonormal Phi).  Deterministic (fixed
 * reduction order).  P: dev [D*D] doubles, i final, j initial.
 * w: dev [M] ascending eigenvalues of Phi's columns, used for the cluster
 * check: with z_a = sum_j |Phi[(j,0),a]|^2, a pair a < b with
 * w[b] - w[a] <= 1e-8 max(1, |w[0]|, |w[M-1]|) and z_a z_b > 1e-20 makes the
 * exact average depend on the basis chosen inside the degenerate subspace
 * (cross terms of size up to sqrt(z_a z_b) survive the time average); then
 * dev_status is set to MMF_ERR_DEGENERATE, else to 0.  P is written either way.
 * Errors: -1 problem, -2 Phi, -3 ld, -4 w, -5 P, -6 dev_status NULL,
 * -7/-8 workspace NULL or too small, MMF_ERR_HIP. */
int mmf_avg_prob(const mmf_problem *p, const mmf_z *Phi, int64_t ld, const double *w, double *P,
                 int32_t *dev_status, void *work, size_t work_bytes, void *stream);

/* mmf_avg_prob without a workspace, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation).  The partial sums and flags live in a 32 MiB array
 * inside the library (one per GPU, allocated when the library's code is
 * loaded on that GPU and held until the process ends); the call allocates and
 * frees nothing.  Every call on one GPU shares that array: calls that overlap
 * on one GPU (other streams, other host threads) race and must be
 * serialised by the caller.  Partials: min(2048, M) workgroups as in
 * mmf_avg_prob when they fit in the array (D <= 45: results bitwise equal to
 * mmf_avg_prob's), else 32 MiB / (8 D^2 + 4) of them (equal up to rounding).
 * Arguments and status as mmf_avg_prob without work/work_bytes.
 * Errors: -1 problem, -2 Phi, -3 ld, -4 w, -5 P, -6 dev_status NULL,
 * MMF_ERR_TOO_LARGE if the partials cannot fit, MMF_ERR_HIP. */
int mmf_avg_prob_noalloc(const mmf_problem *p, const mmf_z *Phi, int64_t ld, const double *w, double *P,
                         int32_t *dev_status, void *stream);

/* Benchmark instrumentation (not needed for computation).  mmf_ktimer_arm
 * starts recording HIP events around every launch of one kernel class on
 * the stream it is launched on, together with the algorithmic work of each
 * launch: "hemv" (the Hermitian matrix-vector product of the one-stage
 * reduction; work = bytes read) or "bt2" (the back-transformation by the
 * bulge-chasing reflectors of the two-stage reduction; work = real flops,
 * 16 per reflector entry and eigenvector column).  mmf_ktimer_read disarms,
 * waits for the events and returns the launch count, the summed kernel time
 * in ms and the summed work.  Process-wide state: use from one host thread, never concurrently
 * with other library calls on other threads.
 * Errors: arm: -1 name NULL or longer than 63 chars; read: -k pointer k NULL,
 * MMF_ERR_HIP. */
int mmf_ktimer_arm(const char *kernel);
int mmf_ktimer_read(int64_t *launches, double *total_ms, double *work);

/* Profiling aid (not needed for computation): with n > 0 the library waits
 * for the whole device (hipDeviceSynchronize) after every n of its kernel
 * launches, so that at most n of its dispatches are pending at once -- for
 * hardware-counter collection tools that cannot hold the tens of thousands
 * of pending dispatches one eigensolve enqueues.  n <= 0 turns it off (the
 * default).  Process-wide; never fails. */
int mmf_profile_sync_every(int64_t n);

#ifdef __cplusplus
}
#endif
#endif /* MMF_H */
