// Internal declarations shared by the host context and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <algorithm>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/matsgw.h"

namespace msgw {

// Error carrying an ABI return code.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define MSGW_HIP(call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::msgw::Error(MSGW_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// A grid dimension holds at most 2^32 - 1 work-items, and y / z at most 65535 work-groups: larger
// shapes are refused rather than launched truncated.
inline void check_grid(dim3 g, dim3 b, const char* what) {
    if (uint64_t(g.x) * b.x > 0xFFFFFFFFull || g.y > 65535u || g.z > 65535u)
        throw Error(MSGW_ENOTSUP, std::string(what) + ": launch grid exceeds the dispatch limits");
}

#define MSGW_LAUNCH(kernel, grid, block, shm, stream, ...)               \
    do {                                                                 \
        ::msgw::check_grid((grid), (block), #kernel);                    \
        hipLaunchKernelGGL(kernel, grid, block, shm, stream, __VA_ARGS__); \
    } while (0)

// Device-resident constant tables (they live in the caller's workspace) plus the
// sizes every kernel needs.  Passed by value to the launchers.
struct Dev {
    int nk = 0, ntau = 0, niw_f = 0, niw_b = 0, nbmax = 0, nimax = 0;
    double beta = 0, scale = 0;
    const double* tau = nullptr;      // [ntau]
    const double2* wf = nullptr;      // [niw_f][ntau]  forward fermionic weights
    const double2* wb = nullptr;      // [niw_b][ntau]  forward bosonic weights
    const double2* ef = nullptr;      // [ntau][niw_f]  exp(-i w_n tau_i)
    const double2* eb = nullptr;      // [ntau][niw_b]  exp(-i nu_n tau_i)
    const int* kmq = nullptr;         // [nk*nk]
    const int* nb = nullptr;          // [nk]
    const int* ni = nullptr;          // [nk]
    const int64_t* moff = nullptr;    // [nk*nk] offset of block (q,k) inside q's M block
    const int64_t* mpre = nullptr;    // [nk+1]  prefix over q of M block sizes
    const int64_t* ppre = nullptr;    // [nk+1]  prefix over q of ntau*NI_q^2
    const int64_t* wpre = nullptr;    // [nk+1]  prefix over q of niw_b*NI_q^2
    const int64_t* vpre = nullptr;    // [nk+1]  prefix over q of NI_q
    // crystal symmetry tables (written by msgw_set_symmetry / msgw_synth_M_cubic)
    int* sym_kmap = nullptr;          // [nk][nk]  R^-1 k for the operation R that maps q's representative onto q
    int* sym_star = nullptr;          // [nk]      the q of every star, grouped by representative
    int* sym_rk = nullptr;            // [48][nk]  cubic generator: index of R k
    int* sym_rg = nullptr;            // [48][nimax] cubic generator: index of R G_I
    int* sym_g2 = nullptr;            // [nimax]   cubic generator: |G_I|^2
    char* scratch = nullptr;          // per-call scratch
    size_t scratch_bytes = 0;
    int kb0 = 0, kb1 = 0;             // k blocks [kb0, kb1) of the pair-space contractions
    int kreuse = 0;                   // 1: the per-q operands prepared by the previous call are reused
    int tau_mirror = 0;               // 1: P(q, tau_{N-1-i}) = P(q, tau_i) may be used (caller's assertion)
    // operand scales of the MSGW_F16X3 contractions (in the scratch, indexed by absolute q):
    unsigned long long* mx_m = nullptr;  // [nk]        bits of max |M^I_K|^2 over q's block (double >= 0)
    unsigned long long* mx_w = nullptr;  // [nk][ntau]  bits of max |Re|, |Im| of W~(q, tau) (double >= 0)
    double* g_max = nullptr;             // [nk][ntau]  max_n |G_n(k, tau)|
    int* e_g = nullptr;                  // [nk][ntau]  power-of-two exponent of the polarization weights
    // harness-only timing: HIP events recorded around the contraction kernels of each polarization
    // (index 0) and self-energy (index 1) call on the call's stream (null: none)
    hipEvent_t ev_start[2] = {nullptr, nullptr}, ev_stop[2] = {nullptr, nullptr};
};

// records d's kernel-timing event of op (0 polarization, 1 self-energy) on s, if one is set
inline void record_kernel_event(const Dev& d, int op, bool stop, hipStream_t s) {
    hipEvent_t e = stop ? d.ev_stop[op] : d.ev_start[op];
    if (e) MSGW_HIP(hipEventRecord(e, s));
}

// Host mirror of the problem (used for launch shapes and validation).
struct Host {
    int nk = 0, ntau = 0, niw_f = 0, niw_b = 0, nbmax = 0, nimax = 0, sigma_mode = 0;
    double beta = 0, scale = 0;
    std::vector<int> kmq, nb, ni;
    std::vector<double> tau;
    std::vector<int64_t> moff, mpre, ppre, wpre, vpre;
};

// ---- launchers (defined in the kernel files) ----
void launch_green0(const Dev& d, hipStream_t s, const double* eps, double mu, double* G);
void launch_synth_M(const Dev& d, const Host& h, hipStream_t s, uint64_t seed, int q0, int nq,
                    int symmetric, int m_dtype, void* M);
void launch_fwd(const Dev& d, hipStream_t s, int stat, int64_t nblk, int64_t len, const void* f,
                int f_cplx, const double* eref, void* out);
void launch_inv_fermion(const Dev& d, hipStream_t s, int64_t nblk, int64_t len, const void* F,
                        const double* eref, double* out);
void launch_inv_boson(const Dev& d, hipStream_t s, int64_t nblk, int mat_n, const void* F,
                      const void* add, const double* v, void* out);
// scratch: screen_scratch_bytes(h, nq) bytes (the pivot rows of every (q, nu) matrix, and the state of
// the Hermitian path, k_hscreen.hip)
size_t screen_scratch_bytes(const Host& h, int nq);
// throws MSGW_ENOTSUP for a call the screen's launches cannot take (NI above 4096, more than 65535
// matrices, an update grid beyond 2^32 threads); called before anything is enqueued
void screen_validate(const Host& h, int q0, int nq);
void launch_screen(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* P_iw,
                   const double* v, void* Wt_iw, void* R_iw, int* info, int* flags, int* perm);
void launch_sigma_x(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
                    int m_dtype, const double* occ, const double* v, void* out, int full);
// E: [nk * nbmax] doubles, st: kMuSearchBytes of mu search state (every entry written before use)
void launch_dyson(const Dev& d, const Host& h, hipStream_t s, const double* eps,
                  const double* sstat, const void* sigc, double n_target, int search, double* mu,
                  void* G_iw, double* G_tau, double* n_out, int* flags, double* E, double* st);
// matrix Dyson (off-diagonal Sigma_nn'): scratch of 8 + nk * niw_f doubles
size_t mdyson_scratch_bytes(const Host& h);
void launch_dyson_matrix(const Dev& d, const Host& h, hipStream_t s, const double* eps, const double2* S0,
                         const double2* Sc, double n_target, int search, double* mu, double2* G_iw,
                         double2* G_tau, double* n_out, int* flags, double* scratch);
// bytes of the static scratch of msgw_dyson_noalloc, and its device address on `device` (looked up
// once per device, with that device made current for the lookup)
constexpr size_t kNoAllocScratchBytes = size_t(1) << 20;
void* noalloc_scratch(int device);
void launch_gap(const Dev& d, const Host& h, hipStream_t s, const double* eps,
                const double* sstat, const void* sigc, const double* mu, int n_index, double* gap);
void launch_gap_given(const Dev& d, const Host& h, hipStream_t s, const double* E, int n_index, double* gap);
size_t cpe_scratch_bytes(const Host& h, int n_real);
void launch_cpe(const Dev& d, const Host& h, hipStream_t s, int n_real, double w_min, double w_max, double ridge,
                double eta, const double* eps, const double* sstat, const void* sigc, const double* mu,
                int n_omega, const double* omega, double* A, double* Eqp, double* coef, int* flags);
void launch_pade(const Dev& d, const Host& h, hipStream_t s, int n_pade, double eta, const double* eps,
                 const double* sstat, const void* sigc, const double* mu, int n_omega, const double* omega,
                 double* A, double* Eqp, int* flags);
// contractions
void launch_pol_fp64(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
                     const double* G, void* P);
void launch_sig_fp64(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
                     const double* G, const void* W, void* Sig);
void launch_sig_full_fp64(const Dev& d, const Host& h, hipStream_t s, int q0, int nq,
                          const void* M, const double* G, const void* W, void* Sig);
// the FULL band-matrix self-energy in MSGW_F16X3 (k_sigfull.hip), M c64, W~ c128; scratch: the FP32
// product W~ M of one (q, k) for a chunk of tau points plus the operand maxima
size_t sigfull_split_scratch_bytes(const Host& h);
void launch_sig_full_split(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
                           const double* G, const void* W, void* Sig, char* scratch, size_t scratch_bytes);
int launch_pol_mfma(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
                    const double* G, int precision, int variant, void* P);
int launch_sig_mfma(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
                    const double* G, const void* W, int precision, int variant, void* Sig);
int mfma_variant_count(int op, int precision);
const char* mfma_variant_name(int op, int precision, int variant);
size_t mfma_scratch_bytes(const Host& h, int nq_max);

// Scratch layout: [E array of msgw_dyson: nk*nbmax doubles][mu search state: 8 KB][operand scales
// of the F16X3 contractions][MFMA conversion buffers].
constexpr size_t kMuSearchBytes = 8192;
inline size_t scratch_al(size_t x) { return (x + 255) & ~size_t(255); }
inline size_t scratch_scale_bytes(const Host& h) {
    const size_t nt = size_t(h.nk) * h.ntau;
    return scratch_al(8 * size_t(h.nk)) + scratch_al(8 * nt) + scratch_al(8 * nt) + scratch_al(4 * nt);
}
inline size_t scratch_E_bytes(const Host& h) {
    return scratch_al(sizeof(double) * size_t(h.nk) * h.nbmax) + kMuSearchBytes + scratch_scale_bytes(h);
}
inline double* scratch_E(const Dev& d) { return reinterpret_cast<double*>(d.scratch); }
inline double* scratch_mu_search(const Dev& d, const Host& h) {
    return reinterpret_cast<double*>(d.scratch + scratch_al(sizeof(double) * size_t(h.nk) * h.nbmax));
}
// points the scale tables of d into its scratch (after the mu search state)
inline void scratch_set_scales(Dev& d, const Host& h) {
    char* p = d.scratch + scratch_al(sizeof(double) * size_t(h.nk) * h.nbmax) + kMuSearchBytes;
    const size_t nt = size_t(h.nk) * h.ntau;
    d.mx_m = reinterpret_cast<unsigned long long*>(p);
    p += scratch_al(8 * size_t(h.nk));
    d.mx_w = reinterpret_cast<unsigned long long*>(p);
    p += scratch_al(8 * nt);
    d.g_max = reinterpret_cast<double*>(p);
    p += scratch_al(8 * nt);
    d.e_g = reinterpret_cast<int*>(p);
}
inline char* scratch_mfma(const Dev& d, const Host& h) { return d.scratch + scratch_E_bytes(h); }
inline size_t scratch_mfma_bytes(const Dev& d, const Host& h) {
    return d.scratch_bytes > scratch_E_bytes(h) ? d.scratch_bytes - scratch_E_bytes(h) : 0;
}

// ---- crystal symmetry (k_misc.hip) ----
constexpr int kMaxRot = 48;
void launch_synth_cubic(const Dev& d, const Host& h, hipStream_t s, uint64_t seed, int q0, int nq, int m_dtype,
                        void* M, const int* rk, const int* rg, const int* g2);
void launch_sigma_star(const Dev& d, const Host& h, hipStream_t s, const int* kmap, const int* star, int s0,
                       int s1, const double* C, const double* Cx, double* S, double* Sx);

// ---- batched Gauss-Jordan (k_gj.hip) ----
constexpr int GJ_INVERT = 0;  // A <- A^-1 (columns permuted by the pivot swaps)
constexpr int GJ_SOLVE = 1;   // [A | B] -> B <- A^-1 B
constexpr int kGjMaxN = 4096;
// A batch of matrices: either a table form (per-matrix order, row stride and offset in device arrays)
// or the screen's form (matrix b is (q0 + b / niw_b, nu = b % niw_b) of NI_q x NI_q at the screen's
// offsets).
struct GjArgs {
    double2* A = nullptr;
    int mode = GJ_INVERT;
    const int* tn = nullptr;           // [batch] order
    const int* tld = nullptr;          // [batch] row stride (>= order; order + rhs columns in GJ_SOLVE)
    const int64_t* toff = nullptr;     // [batch] offset of the matrix in A (elements)
    const int* ni = nullptr;           // screen form (when set): NI_q
    const int64_t* wpre = nullptr;     //   prefix over q of niw_b * NI_q^2
    int q0 = 0, niw_b = 0;
    int* perm = nullptr;               // [batch][pmax] pivot row chosen for each column
    int pmax = 0;
    int* info = nullptr;               // [batch] first zero pivot + 1, or 0
    const int* skip = nullptr;         // [batch] (when set) 1: leave the matrix alone (order 0)
};
__device__ __forceinline__ void gj_item(const GjArgs& g, int b, int& n, int& ld, int64_t& off) {
    if (g.skip && g.skip[b]) {
        n = ld = 0;
        off = 0;
        return;
    }
    if (g.ni) {
        const int q = g.q0 + b / g.niw_b;
        n = g.ni[q];
        ld = n;
        off = (g.wpre[q] - g.wpre[g.q0]) + int64_t(b % g.niw_b) * n * n;
    } else {
        n = g.tn[b];
        ld = g.tld[b];
        off = g.toff[b];
    }
}
// Enqueues the elimination of `batch` matrices of order <= nmax (row stride <= ldmax) on s.
void gj_run(const GjArgs& g, int batch, int nmax, int ldmax, hipStream_t s);
// the Hermitian path of the screen (k_hscreen.hip): scratch bytes for `batch` matrices of order <= nimax
size_t hp_scratch_bytes(int batch, int nimax);
// decides per matrix whether P(i nu) is Hermitian (to 1e-6 of max |v^1/2 P v^1/2|), and inverts those
// matrices (their Hermitian part) by the blocked sweep; on return skip_gj[b] = 1 for the matrices it
// finished and skip_rb[b] = 0 for those whose sweep met a non-positive pivot (their A must be rebuilt
// for the pivoting elimination)
void hp_run(const GjArgs& g, int batch, int nmax, int nimax, char* scratch, hipStream_t s, const int** skip_gj,
            const int** skip_rb);
// W~ and R of the matrices the sweep finished (from the upper triangle of -A^-1)
void hp_finish(const GjArgs& g, int batch, int nmax, int nimax, char* scratch, const double2* Piw, const double* v,
               const int64_t* vpre, double2* R, hipStream_t s);

// ---- the tau-domain solvers (k_tausys.hip) ----
constexpr int kDysonTauMaxGrid = 2048;  // dense grid points of the tau-domain Dyson solve
struct TauSysArgs {
    int ntau = 0, nbmax = 0, nd = 0, q0 = 0, k0 = 0;
    double beta = 0;
    const int* ni = nullptr;            // problem tables (device)
    const int64_t* ppre = nullptr;
    const int64_t* vpre = nullptr;
    const double* phi = nullptr;        // W~ system: spline weights [ntau][ntau][ntau] of P at tau_p - tau_r
    const double* dt = nullptr;         //   trapezoid increments of the mesh [ntau]
    const double* psi = nullptr;        // Dyson: spline weights [nd][ntau] of Sigma^c at the dense nodes
    const double* td = nullptr;         //   dense nodes [nd]
    const double* dtd = nullptr;        //   their trapezoid increments [nd]
    const int* idx = nullptr;           //   dense node of each mesh point [ntau]
    const int* st_k = nullptr;          //   state list (k, n) [nstates]
    const int* st_n = nullptr;
    double* gpos = nullptr;             //   G0(E, a h) per state [nstates][nd]
    double* scd = nullptr;              //   Sigma^c(a h) per state [nstates][nd]
    const int* tn = nullptr;            // systems: order, row stride, offset in K [count]
    const int* tld = nullptr;
    const int64_t* koff = nullptr;
    int* perm = nullptr;                // [count][max order]
    int* ginfo = nullptr;               // [count]
    double2* K = nullptr;               // the augmented systems
};
void launch_wt_tau_system(const TauSysArgs& a, hipStream_t s, int nq, int nmax, int ldmax, const void* P_tau,
                          const double* v, void* Wt_tau);
void launch_dyson_tau(const TauSysArgs& a, hipStream_t s, int nstates, int nkc, const double* eps,
                      const double* sstat, const double* mu, const double* Sigma_c_tau, double* G_tau, int* info);

// ---- small device helpers ----
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// Reference Green's function -exp(-E t)(1 - n_F(E)) in the overflow-free form.
__device__ __forceinline__ double g0_tau(double E, double t, double beta) {
    double a = fabs(E);
    double den = 1.0 + exp(-beta * a);
    return E >= 0.0 ? -exp(-a * t) / den : -exp(-a * (beta - t)) / den;
}

}  // namespace msgw
