/*
 * matsgw.h -- C ABI of the MI355X Matsubara-time GW hot path.
 *
 * The operations follow Chu et al., "All-electron self-consistent GW in the
 * Matsubara-time domain" (arXiv:1602.02313):
 *   polarization P(q,tau)            eq. irpol (with G(-tau) = -G(beta-tau), Basics of the Theory)
 *   tau <-> i omega transforms       eq. trans (cubic-spline quadrature, "Analytic continuation")
 *   screened interaction W~(q,i nu)  eq. scrv and the W~ Dyson equation ("Screened Coulomb potential"),
 *                                    solved on the bosonic Matsubara axis
 *   correlation self-energy          eq. sigc
 *   exchange self-energy             Sigma^x = -G(0-) v delta(tau), product-basis form of eq. sigx
 *   Dyson update of G                eqs. dysongf, zxjk, zcjk, solved on the fermionic axis
 *
 * Conventions shared by every call
 *   - Every call returns int: MSGW_OK (0) or a negative MSGW_E* code; nothing
 *     throws across the ABI.  msgw_last_error() gives a message for the last
 *     failure on a context.
 *   - Arguments are validated on the host before anything is enqueued; a
 *     failing call enqueues nothing.
 *   - Device calls are asynchronous on the caller's stream (a hipStream_t
 *     passed as void*, NULL = the default stream) and never synchronise the
 *     device unless stated.
 *   - Ownership: the caller owns every device buffer, including the workspace.
 *     The library allocates no device memory; the context owns its host-side
 *     tables.  One context serves one host thread.
 *   - Layouts: row-major, 0-based.  Complex data are interleaved (re, im):
 *     "c128" = 2 x double, "c64" = 2 x float.  Hermitian outputs are stored in
 *     full.
 *   - Indices: n is a band at k, m a band at k-q.  M^I_nm(k,q) is the paper's
 *     M^{k-q}_{mn}(G_I, q) (eq. mmatrix).  s = problem.scale = -1/(Omega N_k).
 *   - tau[0] = 0 holds the 0+ limit and tau[ntau-1] = beta the beta- limit.
 *
 * Array shapes used below (nbmax = max_k Nb_k):
 *   G_tau      f64  [nk][nbmax][ntau]     entries n >= Nb_k are ignored / written 0
 *   M (per q)  c128 or c64, for k = 0..nk-1 a block [NI_q][Nb_k][Nb_{k-q}];
 *              q blocks are packed one after another starting at q0
 *              (msgw_m_layout gives the offsets)
 *   P_tau      c128 [q][ntau][NI_q][NI_q]     packed over the q range of the call
 *   P_iw, Wt_iw, R_iw  c128 [q][niw_b][NI_q][NI_q]
 *   Wt_tau     c128 [q][ntau][NI_q][NI_q]
 *   v          f64  [q][NI_q]                packed over the q range of the call
 *   Sigma_tau  f64  [nk][nbmax][ntau] (DIAG)  or c128 [nk][nbmax][nbmax][ntau] (FULL)
 *   Sigma_x    f64  [nk][nbmax]       (DIAG)  or c128 [nk][nbmax][nbmax]       (FULL)
 *   eps, sigma_static        f64 [nk][nbmax]
 *   Sigma_c_iw, G_iw         c128 [nk][nbmax][niw_f]
 */
#ifndef MATSGW_H
#define MATSGW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define MSGW_OK        0
#define MSGW_EINVAL   (-1)   /* bad argument (null pointer, out-of-range enum or index) */
#define MSGW_ESHAPE   (-2)   /* inconsistent sizes, tau mesh not mirror symmetric, ...  */
#define MSGW_EHIP     (-3)   /* a HIP runtime call failed (message has the HIP error)    */
#define MSGW_ENOMEM   (-4)   /* workspace missing or too small for the request           */
#define MSGW_ENOCONV  (-5)   /* reserved: iteration did not converge                      */
#define MSGW_ENOTSUP  (-6)   /* combination not supported (limits are in the message)     */

/* precision of the two contractions (polarization, self_energy) */
#define MSGW_FP64    0   /* FP64 arithmetic throughout                                  */
#define MSGW_FP32    1   /* FP32 MFMA, FP32 accumulation per k, FP64 across k            */
#define MSGW_BF16X3  2   /* 3-term BF16 split (hi*hi + hi*lo + lo*hi) on MFMA, FP32 accumulate */
#define MSGW_F16X3   3   /* 3-term FP16 split of power-of-two-scaled operands on MFMA, FP32
                            accumulate: M scaled per q, the weights (g for P, W~ for Sigma) per
                            (q, tau), so that the largest element is near 2^14; hi = f16(x),
                            lo = f16(x - hi), x.y ~ hi*hi + hi*lo + lo*hi (about 2^-21 relative
                            per product against 2^-16 for BF16X3); the scales are undone in FP64 */

/* storage type of M */
#define MSGW_C128    0
#define MSGW_C64     1

/* statistics of a transform */
#define MSGW_FERMION 0   /* omega_n = (2n+1) pi / beta */
#define MSGW_BOSON   1   /* nu_n    =  2n    pi / beta */

/* self-energy mode */
#define MSGW_SIGMA_DIAG 0   /* Sigma_nn(k,tau), the diagonal approximation of the paper */
#define MSGW_SIGMA_FULL 1   /* Sigma_nn'(k,tau), full band matrix (FP64 or F16X3)      */

/* chemical potential handling in msgw_dyson */
#define MSGW_MU_FIXED  0
#define MSGW_MU_SEARCH 1

/* bits of the device flag word written by msgw_dyson */
#define MSGW_FLAG_NAN        1   /* a non-finite value in Sigma or G   */
#define MSGW_FLAG_NOBRACKET  2   /* n_target outside [N(lo), N(hi)]     */
#define MSGW_FLAG_NOCONV     4   /* a quasiparticle equation did not converge */
#define MSGW_FLAG_SINGULAR   8   /* msgw_screen: an exactly zero pivot of 1 - v^1/2 P v^1/2 */

/* hard limits (checked by set_problem / the calls) */
#define MSGW_MAX_NI   1024   /* product-basis size per q (the screen keeps panel rows in registers) */
#define MSGW_MAX_NB   1024
#define MSGW_MIN_NTAU 4      /* not-a-knot spline needs four points */

typedef struct msgw_ctx msgw_ctx;

typedef struct {
    int           nk;         /* number of k points = number of q points                        */
    const int*    kmq;        /* host [nk*nk]: kmq[q*nk + k] = index of k - q                       */
    const int*    nb;         /* host [nk]: Nb_k, bands at k                                         */
    const int*    ni;         /* host [nk]: NI_q, product-basis size at q                            */
    int           ntau;       /* points of the tau mesh, including 0 and beta                        */
    const double* tau;        /* host [ntau]: 0 = tau_0 < ... < tau_{ntau-1} = beta, mirror symmetric */
    double        beta;       /* inverse temperature                                                 */
    int           niw_f;      /* positive fermionic Matsubara frequencies                            */
    int           niw_b;      /* non-negative bosonic Matsubara frequencies (nu_0 = 0 included)      */
    double        scale;      /* s = -1/(Omega N_k), prefactor of P, Sigma^c and Sigma^x             */
    int           sigma_mode; /* MSGW_SIGMA_DIAG or MSGW_SIGMA_FULL                                  */
} msgw_problem;

/* ---- context ---------------------------------------------------------------------------- */

/* Create a context bound to HIP device `hip_device`.  *out is NULL on failure. */
int msgw_create(msgw_ctx** out, int hip_device);
/* Destroy a context (NULL is accepted).  Does not touch caller-owned device memory. */
int msgw_destroy(msgw_ctx* c);
/* Message of the last failed call on c ("" if none).  Valid until the next call on c. */
const char* msgw_last_error(const msgw_ctx* c);

/* Set the problem.  Host-synchronous; copies every input.  Builds the FP64 transform
 * weights (not-a-knot cubic spline integrated exactly against e^{i omega tau}).
 * ESHAPE: ntau < 4, tau not increasing, tau[0] != 0, tau[ntau-1] != beta, or
 * |tau_i + tau_{ntau-1-i} - beta| > 1e-12 beta for some i.  Invalidates the workspace. */
int msgw_set_problem(msgw_ctx* c, const msgw_problem* p);

/* Bytes of device workspace needed for calls covering at most nq_max q points at once. */
int msgw_workspace_size(msgw_ctx* c, int nq_max, size_t* bytes);
/* Attach caller-owned device workspace (>= msgw_workspace_size for some nq_max) and upload
 * the constant tables into it.  Host-synchronous.  The buffer must outlive its use. */
int msgw_set_workspace(msgw_ctx* c, void* dptr, size_t bytes);

/* Layout of M: offsets (in complex elements) of the (q,k) block relative to the start of
 * q's block, and the size of q's block.  off may be NULL. */
int msgw_m_layout(const msgw_ctx* c, int q, int64_t* off /*[nk] or NULL*/, int64_t* qsize);

/* ---- hot path ------------------------------------------------------------------------------ */

/* a1. Reference Green's function (eq. for G^0_j(k|tau)):
 * G_tau[k][n][i] = -exp(-E tau_i) (1 - n_F(E)), E = eps[k][n] - mu, for n < Nb_k (0 otherwise),
 * evaluated in the overflow-free form.  eps: device f64 [nk][nbmax]; G_tau: device. */
int msgw_green0(msgw_ctx* c, void* stream, const double* eps, double mu, double* G_tau);

/* a2. Polarization (eq. irpol):
 * P_IJ(q,tau_i) = s sum_k sum_{n<Nb_k} sum_{m<Nb_{k-q}} M^I_nm G_n(k,tau_i) G_m(k-q,tau_{ntau-1-i}) conj(M^J_nm)
 * for q = q0..q0+nq-1.  M (device, m_dtype) starts at q0's block; G_tau device; P_tau (device c128)
 * is overwritten.  precision MSGW_FP64 needs MSGW_C128 M; FP32/BF16X3/F16X3 need MSGW_C64 M. */
int msgw_polarization(msgw_ctx* c, void* stream, int q0, int nq, const void* M, int m_dtype,
                      const double* G_tau, int precision, void* P_tau);

/* a3, a7 and G(tau) -> G(i omega).  Forward transform (eq. trans) along the tau axis:
 * f_iw[b][n][e] = int_0^beta e^{i w_n tau} f(tau) dtau, with f given at the mesh points as
 * f_tau[b][i][e] (b < nblk, i < ntau, e < len; real f64 if !f_is_complex, else c128), integrated
 * as the not-a-knot cubic spline.  stat selects omega_n (niw_f values) or nu_n (niw_b values).
 * e_ref (device f64 [nblk*len], FERMION only, may be NULL): the spline is applied to
 * f - G0(e_ref) and the exact 1/(i w_n - e_ref) is added, so a 0/beta jump is carried exactly.
 * f_iw: device c128 [nblk][niw][len]. */
int msgw_tau_to_iw(msgw_ctx* c, void* stream, int stat, int64_t nblk, int64_t len,
                   const void* f_tau, int f_is_complex, const double* e_ref, void* f_iw);

/* Inverse transform (truncated Matsubara sum), f_iw[b][n][e] -> f_tau[b][i][e]:
 *   FERMION (mat_n == 0, real output f64):
 *     f(tau_i) = G0(e_ref,tau_i) + (2/beta) sum_{n<niw_f} Re[e^{-i w_n tau_i}(f(i w_n) - 1/(i w_n - e_ref))]
 *     (e_ref may be NULL: no reference term).
 *   BOSON (mat_n > 0, len == mat_n^2, Hermitian pair f(-i nu) = f(i nu)^H, c128 output):
 *     f(tau_i) = add(tau_i) + (1/beta)[f_0 + sum_{n>=1}(e^{-i nu_n tau_i} f_n + e^{i nu_n tau_i} f_n^H)]
 *     add_tau (device c128 [nblk][ntau][len] or NULL).
 *     MSGW_ENOTSUP for BOSON when niw_b > 146 (the phases of a chunk of tau points are kept in LDS) or
 *     nblk > 65535. */
int msgw_iw_to_tau(msgw_ctx* c, void* stream, int stat, int64_t nblk, int64_t len, int mat_n,
                   const void* f_iw, const void* add_tau, const double* e_ref, void* f_tau);

/* a4. Screened interaction on the bosonic axis (W~ Dyson equation, eq. scrv, on i nu):
 * chi~ = v^1/2 P v^1/2;  W~ = v^1/2 [(1 - chi~)^-1 - 1] v^1/2;  R = W~ - v P v.
 * (1 - chi~) is inverted in FP64, all nq * niw_b matrices of the call together: a matrix whose
 * anti-Hermitian part is at most 1e-6 of max |chi~| is taken as Hermitian, and its Hermitian part is
 * inverted by the blocked sweep without pivoting (valid while it is positive definite, as for P <= 0;
 * every pivot is checked); the others, and those whose sweep met a non-positive pivot, by blocked
 * Gauss-Jordan with partial (row) pivoting (FP64 MFMA updates either way).  R keeps the P given.  The
 * state of both uses the workspace's scratch: MSGW_ENOMEM unless the workspace was sized for
 * nq_max >= nq.  MSGW_ENOTSUP, before anything is enqueued, for more than 65535 matrices
 * (nq * niw_b) in one call or more 64 x 64 update tiles than one launch takes
 * (8 ceil(nq niw_b / 8) ceil(NI/64)^2 * 256 threads >= 2^32): split the q range.
 * P_iw, Wt_iw, R_iw: device c128 [q][niw_b][NI_q][NI_q]; v: device f64 [q][NI_q]; R_iw may be NULL.
 * info: device int [nq*niw_b], 0 or 1 + the first column whose pivot was exactly zero (the outputs of
 * that matrix are then not finite).  flags: device int or NULL; MSGW_FLAG_SINGULAR is OR-ed into it
 * when some info is not 0, so that one word can collect the status of every q batch of a pass. */
int msgw_screen(msgw_ctx* c, void* stream, int q0, int nq, const void* P_iw, const double* v,
                void* Wt_iw, void* R_iw, int* info, int* flags);

/* a5. W~(q,tau_i) = v P(q,tau_i) v + (1/beta)[R(i nu_0) + sum_{n>=1}(e^{-i nu_n tau_i} R(i nu_n)
 *                    + e^{i nu_n tau_i} R(i nu_n)^H)]
 * (R(-i nu) = R(i nu)^H because P(tau) is Hermitian).  R_iw, P_tau, v as above; Wt_tau device c128. */
int msgw_screened_tau(msgw_ctx* c, void* stream, int q0, int nq, const void* R_iw,
                      const void* P_tau, const double* v, void* Wt_tau);

/* a6. Correlation self-energy (eq. sigc), ACCUMULATED into Sigma_tau:
 * DIAG: Sigma_n(k,tau_i) += s sum_q sum_m G_m(k-q,tau_i) Re sum_IJ conj(M^I_nm) W~_IJ(q,tau_i) M^J_nm
 * FULL: Sigma_nn'(k,tau_i) += s sum_q sum_m G_m(k-q,tau_i) sum_IJ conj(M^I_nm) W~_IJ M^J_n'm, in MSGW_FP64
 * (M c128) or MSGW_F16X3 (M c64: W~ M split into FP16 pairs on MFMA, the contraction with conj(M) G in
 * FP64; other precisions return MSGW_ENOTSUP; the whole k range only).
 * The caller zeroes Sigma_tau before the first q.  Wt_tau: device c128 [q][ntau][NI_q][NI_q]. */
int msgw_self_energy(msgw_ctx* c, void* stream, int q0, int nq, const void* M, int m_dtype,
                     const double* G_tau, const void* Wt_tau, int precision, void* Sigma_tau);

/* a6b. Exchange self-energy, ACCUMULATED (product-basis form of eq. sigx with f = G(0-)):
 * DIAG: Sigma^x_n(k) += s sum_q sum_m f_m(k-q) sum_I v_I |M^I_nm|^2 ; FULL: the n,n' matrix
 * s sum_q sum_m f_m sum_I v_I conj(M^I_nm) M^I_n'm.  The occupations are read from the Green's
 * function, f_m(k) = G_m(k, 0-) = -G_tau[k][m][ntau-1].  FP64 arithmetic for either M dtype. */
int msgw_sigma_x(msgw_ctx* c, void* stream, int q0, int nq, const void* M, int m_dtype,
                 const double* G_tau, const double* v, void* Sigma_x);

/* a8. Dyson update of the diagonal G on the fermionic axis and the chemical potential:
 * E = eps + sigma_static - mu;  G(i w_n) = 1/(i w_n - E - Sigma^c(i w_n));
 * N(mu) = sum_nk [n_F(E) + (2/beta) sum_{n<niw_f} Re(G - 1/(i w_n - E))];
 * MSGW_MU_SEARCH: mu so that N(mu) = n_target, on the bracket [min(eps+sigma_static) - 50/beta,
 * max(...) + 50/beta], by 8 fixed rounds of 256-section (N at 257 points of the bracket per round,
 * the bracket shrinks by 2^64 in all; device-side, a fixed number of launches, graph-capturable);
 * MSGW_MU_FIXED: mu is read from *mu.  Then G(tau) by the FERMION inverse transform with
 * e_ref = E.  mu, n_out: device f64 scalars (mu in/out); flags: device int (MSGW_FLAG_*).
 * G_iw may be NULL. */
int msgw_dyson(msgw_ctx* c, void* stream, const double* eps, const double* sigma_static,
               const void* Sigma_c_iw, double n_target, int mu_mode, double* mu, void* G_iw,
               double* G_tau, double* n_out, int* flags);

/* f3. Dyson update with off-diagonal band matrices, the generalisation of the diagonal approximation
 * (eqs. dysongf, zxjk, zcjk with Sigma_nn', solved on the fermionic axis):
 *   H0(k) = diag(eps_k) + Sigma_static(k);  G(k, i w_n) = [(i w_n + mu) 1 - H0(k) - Sigma^c(k, i w_n)]^-1
 *   over the bands n < Nb_k, inverted in FP64 (Gauss-Jordan with partial pivoting);
 *   with D = G - diag(1 / (i w - E_jj)), E_jj = Re H0_jj - mu:
 *   N(mu) = sum_k [sum_j n_F(E_jj) + (2/beta) sum_n Re Tr D(i w_n)],
 *   G(tau) = diag(G0(E_jj, tau)) + (1/beta) sum_n [e^{-i w_n tau} D_n + e^{i w_n tau} D_n^H]
 *   (negative frequencies D(-i w) = D(i w)^H, as for a Hermitian Sigma(tau)).
 * MSGW_MU_SEARCH: mu by 64 fixed bisection rounds on the Gershgorin bracket of H0 widened by 50/beta
 * (a fixed sequence of launches); MSGW_MU_FIXED: mu read from *mu.
 * eps f64 [nk][nbmax]; sigma_static c128 [nk][nbmax][nbmax] (e.g. the FULL Sigma^x); Sigma_c_iw c128
 * [nk][nbmax][nbmax][niw_f] (the FULL Sigma^c(tau) through msgw_tau_to_iw); G_iw c128
 * [nk][nbmax][nbmax][niw_f]; G_tau c128 [nk][nbmax][nbmax][ntau]; mu, n_out device f64; flags device int
 * (MSGW_FLAG_NAN for non-finite input or an exactly singular matrix, MSGW_FLAG_NOBRACKET).  nbmax <= 64
 * (MSGW_ENOTSUP).  Uses the workspace's scratch. */
int msgw_dyson_matrix(msgw_ctx* c, void* stream, const double* eps, const void* sigma_static,
                      const void* Sigma_c_iw, double n_target, int mu_mode, double* mu, void* G_iw,
                      void* G_tau, double* n_out, int* flags);

/* For callers that cannot allocate device memory at the time of the call (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): msgw_dyson with the same arguments,
 * results and errors, whose per-call scratch (the E array and the mu search state) lives in a static
 * device array of 1 MiB that each device keeps until the process ends, instead of the workspace.  It
 * calls no allocating routine.  The context still needs its workspace for the constant tables (set
 * once at setup).  Limit: nk * nbmax <= 130048 states, else MSGW_ENOTSUP and nothing is enqueued.
 * Every call on a device shares that device's array: calls that overlap on one device (two streams,
 * two contexts, two threads) race and must be ordered by the caller. */
int msgw_dyson_noalloc(msgw_ctx* c, void* stream, const double* eps, const double* sigma_static,
                       const void* Sigma_c_iw, double n_target, int mu_mode, double* mu, void* G_iw,
                       double* G_tau, double* n_out, int* flags);

/* a9 (loop control).  Matsubara-axis gap proxy used to follow the self-consistent loop:
 * E^QP_nk = eps + sigma_static + Re Sigma^c_nk(i w_0) - mu over all (n < Nb_k, k), and
 * *gap = E_(N+1) - E_(N) (ascending order, 1-based) with N = n_index, 1 <= N < number of states.
 * The paper reads gaps off analytically continued spectra instead; this proxy involves no
 * continuation.  Sigma_c_iw: device c128 [nk][nbmax][niw_f]; mu: device scalar; gap: device f64. */
int msgw_gap(msgw_ctx* c, void* stream, const double* eps, const double* sigma_static,
             const void* Sigma_c_iw, const double* mu, int n_index, double* gap);

/* ---- the paper's tau-domain solvers (cross-checks of a4-a5 and a8), FP64 --------------------- */

#define MSGW_TS_WTILDE 0   /* msgw_wt_tau_system   */
#define MSGW_TS_DYSON  1   /* msgw_dyson_tau       */

/* Bytes of the device work buffer that msgw_wt_tau_system (which = MSGW_TS_WTILDE, q range
 * [first, first + count)) or msgw_dyson_tau (MSGW_TS_DYSON, k range [first, first + count)) needs:
 * mostly the augmented systems, 16 * n * (n + rhs) bytes each.  The same range limits as the calls. */
int msgw_tau_solver_work_size(msgw_ctx* c, int which, int first, int count, size_t* bytes);

/* f2. W~(q, tau) from the paper's linear system on the tau mesh (eq. tildeW, "Screened Coulomb
 * potential" in Sec. III.B), for q in [q0, q0 + nq):
 *   sum_r [delta_pr 1 - v P(tau_p - tau_r) dtau_r] W~(tau_r) = v P(tau_p) v,
 * dtau_r = (tau_{r+1} - tau_{r-1}) / 2 (half intervals at the ends), P at a difference of mesh points
 * from the not-a-knot cubic spline of P(tau) on the mesh (a difference below zero is taken at
 * + beta: P is bosonic).  One dense complex system of order ntau * NI_q per q (<= 4096, else
 * MSGW_ENOTSUP), solved by the batched blocked Gauss-Jordan elimination of the screen.
 * P_tau, Wt_tau: device c128 [q][ntau][NI_q][NI_q] (the layout of msgw_polarization); v: device f64
 * [q][NI_q]; info: device int [nq], 0 or 1 + the first column whose pivot was exactly zero; work: device,
 * 256-byte aligned, at least msgw_tau_solver_work_size(MSGW_TS_WTILDE, q0, nq) bytes, owned by the
 * caller.  The call uploads its host-built tables into work on `stream` and waits for the stream
 * before returning (host-synchronous). */
int msgw_wt_tau_system(msgw_ctx* c, void* stream, int q0, int nq, const void* P_tau, const double* v,
                       void* Wt_tau, int* info, void* work, size_t work_bytes);

/* f2. G_n(k, tau) of every state (n < Nb_k) of k in [k0, k0 + nkc) from the paper's Dyson equation in
 * the tau domain (eqs. dysongf, zxjk, zcjk, dysong), solved on the dense uniform grid t_a = a h,
 * h = tau_1 - tau_0, a = 0..N, N h = beta:
 *   sum_r [delta_pr - dt_r Z(t_p, t_r)] G(t_r) = G0(t_p),
 *   Z(t, t2) = G0(t - t2) sigma_static + int_0^beta dt1 G0(t - t1) Sigma^c(t1 - t2),
 * G0 the reference Green's function at E = eps - mu, Sigma^c the not-a-knot spline of Sigma_c_tau on
 * the grid, dt the trapezoid increments of the grid (also for the t1 integral); arguments below zero
 * are antiperiodic; at a zero argument an interior node takes the mean of the two limits, an end node
 * of the integration range the limit inside the range.  One real system of order N + 1 per state.
 * MSGW_ESHAPE unless beta and every tau_i are multiples of h (as on a uniform or uniform power mesh);
 * MSGW_ENOTSUP above 2048 grid points or 65535 states.
 * eps, sigma_static: device f64 [nk][nbmax]; mu: device scalar; Sigma_c_tau: device f64
 * [nk][nbmax][ntau]; G_tau: device f64 [nk][nbmax][ntau], rows n < Nb_k of k in the range written;
 * info: device int [nkc][nbmax], 0 or 1 + the first zero pivot of the state's system (0 for n >= Nb_k);
 * work as for msgw_wt_tau_system (MSGW_TS_DYSON, k0, nkc).  Host-synchronous like msgw_wt_tau_system. */
int msgw_dyson_tau(msgw_ctx* c, void* stream, int k0, int nkc, const double* eps, const double* sigma_static,
                   const double* mu, const double* Sigma_c_tau, double* G_tau, int* info, void* work,
                   size_t work_bytes);

/* ---- symmetry ------------------------------------------------------------------------------ */

/* The caller asserts (on != 0) that its inputs give P(q, tau_{N-1-i}) = P(q, tau_i), i.e. P(tau) =
 * P(beta - tau) on the mirror-symmetric mesh: time-reversal symmetry of the matrix elements, as in
 * crystals without spin-orbit coupling and for msgw_synth_M's symmetric generator (the tau-mirror
 * saving of the paper's use of symmetry, Sec. III.C).  The split-BF16 pair-space polarization then
 * computes the points i <= (N - 1) / 2 and copies the others; the other paths compute every point.
 * With inputs that lack the symmetry the copied points are wrong.  Default off. */
int msgw_set_tau_mirror(msgw_ctx* c, int on);

/* f1. Crystal symmetry: q in the irreducible wedge (Sec. III.C, eqs. rso and qibz2bz with the relations
 * for M, P and W~ that follow them).  For a point group whose operations R map the k grid onto itself,
 * with M^{I'}_nm(R k, R q) = M^I_nm(k, q) for G_{I'} = R G_I (a symmorphic crystal: no fractional
 * translations), R-invariant v and band energies, P and W~ at R q are those at q with permuted basis
 * indices, and the contribution of q' = R q to Sigma_n(k) is that of q to Sigma_n(R^-1 k).  So P, W~ and
 * the contractions run for the irreducible q only, and each irreducible q's contributions to every k are
 * added over its star with rotated k (msgw_sigma_star); DIAG mode.
 *
 * msgw_set_symmetry: rot_k host int [nrot][nk], rot_k[r][k] = index of R_r k (1 <= nrot <= 48).  Each
 * row must be a permutation with R (k - q) = R k - R q on the problem's kmq table, else MSGW_EINVAL.
 * Every orbit {R q} is represented by its smallest q; its star lists each member once, reached by the
 * first r (in the given order) that maps the representative onto it.  Host-synchronous: the maps go
 * into the workspace (call after msgw_set_workspace, with no work on the context in flight); setting a
 * problem or a workspace clears them. */
int msgw_set_symmetry(msgw_ctx* c, int nrot, const int* rot_k);

/* The irreducible q (increasing) and the size of each one's star: host int arrays of nk entries or
 * NULL; *n_ibz receives their number.  MSGW_EINVAL before msgw_set_symmetry. */
int msgw_ibz(const msgw_ctx* c, int* n_ibz, int* q_ibz, int* star_size);

/* Sigma_tau[k][n][i] += sum over the star of q_ibz of C_tau[R^-1 k][n][i], and the same for Sigma_x from
 * C_x (both NULL or both given): C_tau / C_x are the contributions of the single q_ibz to every k
 * (msgw_self_energy / msgw_sigma_x of q_ibz alone into zeroed buffers).  Device f64 [nk][nbmax][ntau]
 * and [nk][nbmax]; the star members are summed in a fixed order. */
int msgw_sigma_star(msgw_ctx* c, void* stream, int q_ibz, const double* C_tau, const double* C_x,
                    double* Sigma_tau, double* Sigma_x);

/* ---- after the path: analytic continuation ---------------------------------------------------- */

/* Analytic continuation of Sigma^c to the real axis by a Pade approximant (the route the paper
 * compares with its continuous-pole expansion, analytic continuation subsection of Sec. III.B):
 * for every state (n < Nb_k, k) the continued fraction of Vidberg and Serene through the n_pade
 * lowest positive Matsubara points, C(z) = a_0 / (1 + a_1 (z - z_0) / (1 + ...)), z_j = i w_j; then
 *   E_qp = x + mu with x the root of x = e0 + Re C(x + i eta), e0 = eps + sigma_static - mu, reached
 *          by Newton's method from x = e0 (at most 100 steps, |step| <= 1e-12 (1 + |x|));
 *   A[state][j] = -(1/pi) Im 1 / (omega_j + i eta - e0 - C(omega_j + i eta)) when A is not NULL.
 * eps, sigma_static: device f64 [nk][nbmax]; Sigma_c_iw: device c128 [nk][nbmax][niw_f]; mu: device
 * scalar; omega: device f64 [n_omega], energies from mu (NULL when n_omega == 0); A: device f64
 * [nk][nbmax][n_omega] or NULL; E_qp: device f64 [nk][nbmax] (NaN for n >= Nb_k); flags: device int,
 * set to 0 then MSGW_FLAG_NOCONV if some state's iteration did not converge.
 * 1 <= n_pade <= min(niw_f, 128); eta >= 0.  Pade coefficients of noisy data can be ill-conditioned:
 * the usual n_pade is a few tens. */
int msgw_continue_pade(msgw_ctx* c, void* stream, int n_pade, double eta, const double* eps,
                       const double* sigma_static, const void* Sigma_c_iw, const double* mu, int n_omega,
                       const double* omega, double* A, double* E_qp, int* flags);

/* Analytic continuation by the continuous-pole expansion, the paper's own route (analytic continuation
 * subsection of Sec. III.B): Im Sigma^c(w) <= 0 is expanded in hat functions h_l at the interior
 * points of the uniform grid of n_real points on [w_min, w_max] (energies from mu),
 *   Sigma^c(z) = -(1/pi) sum_l a_l int h_l(w) / (w - z) dw,  a_l >= 0,
 * with the a_l minimising sum_n |Sigma^c(i w_n) - Sigma(i w_n)|^2 + lam |a|^2 over all niw_f positive
 * Matsubara points, lam = ridge * max_l of the diagonal of the normal matrix (the ridge makes the
 * minimiser unique).  Then, as for msgw_continue_pade, E_qp = x + mu with x = e0 + Re Sigma(x + i eta)
 * (Newton from e0) and, when A is not NULL, A on the omega grid.  coef: device f64
 * [nk][nbmax][n_real - 2] (the a_l) or NULL.  4 <= n_real <= 98, eta > 0, ridge >= 0.  flags gets
 * MSGW_FLAG_NOCONV if a fit or a quasiparticle iteration did not finish.  Uses the workspace. */
int msgw_continue_cpe(msgw_ctx* c, void* stream, int n_real, double w_min, double w_max, double ridge, double eta,
                      const double* eps, const double* sigma_static, const void* Sigma_c_iw, const double* mu,
                      int n_omega, const double* omega, double* A, double* E_qp, double* coef, int* flags);

/* Gap of given energies: *gap = E_(N+1) - E_(N) over the states n < Nb_k in ascending order
 * (N = n_index, 1 <= N < number of states).  E: device f64 [nk][nbmax]; gap: device f64. */
int msgw_gap_of(msgw_ctx* c, void* stream, const double* E, int n_index, double* gap);

/* ---- tile shapes of the MFMA paths (used by the autotuner) ---------------------------------- */

#define MSGW_OP_POLARIZATION 0
#define MSGW_OP_SELF_ENERGY  1

/* Number of compiled tile-shape variants for an op (MSGW_OP_*) in MSGW_FP32 or MSGW_BF16X3, or a
 * negative error code.  Every variant computes the same result to rounding. */
int msgw_variant_count(int op, int precision);
/* Static description of a variant ("WI2 WJ2 T4": 16*WI x 16*WJ output tile per wave, T tau points
 * per work-group), or NULL when out of range. */
const char* msgw_variant_name(int op, int precision, int variant);
/* Select the variant used by subsequent calls on c (default 0). */
int msgw_set_variant(msgw_ctx* c, int op, int precision, int variant);
/* The variant currently selected on c for (op, precision), written to *variant (host int). */
int msgw_get_variant(const msgw_ctx* c, int op, int precision, int* variant);

/* Harness-only (the batching study): restrict the following MSGW_BF16X3 pair-space polarization and
 * self-energy calls on c to the k blocks k0 <= k < k1, so that a loop over k reproduces one full call
 * launch by launch.  A polarization with k0 > 0 ADDS its blocks to P_tau (k0 == 0 overwrites); the
 * self-energy accumulates as always.  reuse_prepared != 0 skips the per-q preparations (the g planes
 * of the polarization, the weight blocks of the self-energy, the operand scales of MSGW_F16X3) and
 * reuses what the previous contraction call left in the workspace; that call must have been of the same
 * op, q range, precision and variant (the two ops share the scratch), else the call fails with
 * MSGW_EINVAL and enqueues nothing.  k1 <= 0 restores the full range.  While a partial range
 * is set, the other tile variants and precisions return MSGW_ENOTSUP.  The FP64 contractions honour a
 * partial range as well (DIAG self-energy; a polarization with k0 > 0 adds), without preparations. */
int msgw_set_k_range(msgw_ctx* c, int k0, int k1, int reuse_prepared);

/* Harness-only (measurement): the following polarization (op = MSGW_OP_POLARIZATION) or self-energy
 * (MSGW_OP_SELF_ENERGY) calls on c record the HIP event `start` (a hipEvent_t) on their stream just
 * before their contraction kernels and `stop` just after them, leaving out the per-q preparations, so
 * that the caller can time the kernels alone.  The events are the caller's; NULL, NULL stops it. */
int msgw_set_kernel_events(msgw_ctx* c, int op, void* start, void* stop);

/* ---- input generation (not part of the method) ---------------------------------------------- */

/* Synthetic M for q0..q0+nq-1 in the layout above (c128 or c64): complex Gaussian with
 * E|M^I|^2 = 1/(1+I/16), drawn by Philox4x32-10 (key = seed, counter = (orbit index lo, hi, I,
 * 0x4D475731)) and Box-Muller in FP64.  symmetric != 0: one draw per orbit of the time-reversal /
 * pair symmetry (k,q,n,m) -> (q-k,q,m,n) and (k,q,n,m) -> (-k,-q,n,m)+conj, keyed by the
 * orbit's smallest linear index ((q nk + k) nbmax + n) nbmax + m; an orbit fixed by a conjugating
 * element is real.  -k and q-k are read from kmq (k index 0 must be Gamma). */
int msgw_synth_M(msgw_ctx* c, void* stream, uint64_t seed, int q0, int nq, int symmetric,
                 int m_dtype, void* M);

/* Harness-only input generation with the symmetry of a symmorphic cubic crystal, the twin of the host
 * generator gwinputs.CubicGenerator: on an n x n x n grid (k = (i1 n + i2) n + i3) with one band count and
 * NI = the number of vectors G in closed shells of |G|^2 (product basis = those G, in the order |G|^2,
 * then lexicographic), one complex Gaussian per orbit of (k, q, G) under the 48 operations of O_h and band
 * pair (n, m): Philox4x32-10 counter (key low, key high, n nb + m, 0x4D435542) with the orbit's smallest
 * key (q' nk + k') NI + I', Box-Muller, E|M|^2 = 1 / (1 + |G|^2 / 4).  MSGW_ESHAPE for other shapes.
 * The first call per NI writes its tables into the workspace (host-synchronous). */
int msgw_synth_M_cubic(msgw_ctx* c, void* stream, uint64_t seed, int q0, int nq, int m_dtype, void* M);

#ifdef __cplusplus
}
#endif
#endif /* MATSGW_H */
