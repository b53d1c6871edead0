// Dyson update with off-diagonal band matrices (the generalisation of the diagonal approximation to
// Sigma_nn'; eqs. dysongf, zxjk, zcjk with matrices, solved on the fermionic axis).  FP64.
//
//   H0(k) = diag(eps_k) + Sigma_static(k),  G(k, i w) = [(i w + mu) 1 - H0(k) - Sigma^c(k, i w)]^-1,
//   D = G - diag(1 / (i w - E_jj)), E_jj = Re H0_jj - mu,
//   N(mu) = sum_k [sum_j n_F(E_jj) + (2/beta) sum_n Re Tr D(i w_n)],
//   G(tau) = diag(G0(E_jj, tau)) + (1/beta) sum_n [e^{-i w_n tau} D_n + e^{i w_n tau} D_n^H].
//
// One work-group inverts one (k, i w_n) matrix in LDS (in-place Gauss-Jordan with partial row pivoting,
// the row interchanges undone as column interchanges at the end), Nb <= 64.  The chemical potential is
// found by a fixed number of bisection rounds on the Gershgorin bracket of H0 (each round: the
// inversions at the midpoint, then one work-group sums Re Tr D in a fixed order and halves the
// bracket), so the call is a fixed sequence of launches.
#include "internal.h"

namespace msgw {
namespace {

constexpr int MD_NB = 64;        // largest band count
constexpr int MD_ROUNDS = 64;    // bisection rounds (the bracket shrinks by 2^64)
constexpr int MD_T = 256;        // threads per work-group
constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ double md_fermi(double E, double beta) {
    const double x = beta * E;
    const double ex = exp(-fabs(x));
    return x >= 0.0 ? ex / (1.0 + ex) : 1.0 / (1.0 + ex);
}
__device__ __forceinline__ double2 md_div(double2 a, double2 b) {
    const double s = fmax(fabs(b.x), fabs(b.y));
    const double bx = b.x / s, by = b.y / s, den = bx * bx + by * by;
    return make_double2((a.x * bx + a.y * by) / (den * s), (a.y * bx - a.x * by) / (den * s));
}

struct MdArgs {
    const double* eps;      // [nk][nbmax]
    const double2* S0;      // [nk][nbmax][nbmax]
    const double2* Sc;      // [nk][nbmax][nbmax][niw]
    const int* nb;
    int nk, nbmax, niw;
    double beta, n_target;
};

// state (doubles): [0] lo, [1] hi, [2] N(lo), [3] N(hi), [4] flags, [5] mu, [6] N(mu)
constexpr int ST_LO = 0, ST_HI = 1, ST_NLO = 2, ST_NHI = 3, ST_FL = 4, ST_MU = 5, ST_N = 6;

// the bracket from the Gershgorin discs of H0 (widened by 50 / beta) and the NaN check
__global__ __launch_bounds__(MD_T) void k_md_prep(MdArgs a, double* st) {
    __shared__ double rlo[MD_T / 64], rhi[MD_T / 64];
    __shared__ int rbad[MD_T / 64];
    double lo = 1e300, hi = -1e300;
    int bad = 0;
    const int64_t rows = int64_t(a.nk) * a.nbmax;
    for (int64_t r = threadIdx.x; r < rows; r += MD_T) {
        const int k = int(r / a.nbmax), j = int(r % a.nbmax), n = a.nb[k];
        if (j >= n) continue;
        const double2* S = a.S0 + int64_t(k) * a.nbmax * a.nbmax;
        double rad = 0.0;
        for (int i = 0; i < n; ++i) {
            if (i == j) continue;
            const double2 v = S[int64_t(j) * a.nbmax + i];
            rad += sqrt(v.x * v.x + v.y * v.y);
        }
        const double d = a.eps[r] + S[int64_t(j) * a.nbmax + j].x;
        if (!isfinite(d) || !isfinite(rad)) bad = 1;
        lo = fmin(lo, d - rad);
        hi = fmax(hi, d + rad);
        const double2* Sc = a.Sc + (int64_t(k) * a.nbmax + j) * a.nbmax * a.niw;
        for (int i = 0; i < n * a.niw; ++i) {
            const double2 v = Sc[(i / a.niw) * a.niw + i % a.niw];
            if (!isfinite(v.x) || !isfinite(v.y)) bad = 1;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, o));
        hi = fmax(hi, __shfl_xor(hi, o));
        bad |= __shfl_xor(bad, o);
    }
    if ((threadIdx.x & 63) == 0) {
        rlo[threadIdx.x >> 6] = lo;
        rhi[threadIdx.x >> 6] = hi;
        rbad[threadIdx.x >> 6] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < MD_T / 64; ++i) {
            lo = fmin(lo, rlo[i]);
            hi = fmax(hi, rhi[i]);
            bad |= rbad[i];
        }
        st[ST_LO] = lo - 50.0 / a.beta;
        st[ST_HI] = hi + 50.0 / a.beta;
        st[ST_FL] = bad ? double(MSGW_FLAG_NAN) : 0.0;
    }
}

// which mu an evaluation uses
enum { MU_LO = 0, MU_HI = 1, MU_MID = 2, MU_GIVEN = 3 };

__device__ __forceinline__ double md_mu(const double* st, const double* mu_in, int which) {
    switch (which) {
        case MU_LO: return st[ST_LO];
        case MU_HI: return st[ST_HI];
        case MU_MID: return 0.5 * (st[ST_LO] + st[ST_HI]);
        default: return *mu_in;
    }
}

// one (k, i w_n) matrix per work-group: A = (i w + mu) 1 - H0 - Sigma^c inverted in LDS; Re Tr D to
// part[k][n]; with G_iw the inverse is written out.  A zero pivot sets MSGW_FLAG_NAN.
__global__ __launch_bounds__(MD_T) void k_md_eval(MdArgs a, double* st, const double* mu_in, int which,
                                                  double* part, double2* G_iw) {
    __shared__ double2 A[MD_NB][MD_NB + 1];
    __shared__ int perm[MD_NB];
    __shared__ double2 colj[MD_NB];
    __shared__ int ridx;
    const int k = blockIdx.x, iw = blockIdx.y, tid = threadIdx.x;
    const int n = a.nb[k], nbm = a.nbmax;
    const double mu = md_mu(st, mu_in, which);
    const double w = (2.0 * iw + 1.0) * kPi / a.beta;
    const double2* S0 = a.S0 + int64_t(k) * nbm * nbm;
    const double2* Sc = a.Sc + int64_t(k) * nbm * nbm * a.niw;
    bool singular = false;
    for (int e = tid; e < n * n; e += MD_T) {
        const int i = e / n, j = e % n;
        const double2 s0 = S0[int64_t(i) * nbm + j], sc = Sc[(int64_t(i) * nbm + j) * a.niw + iw];
        double2 v = make_double2(-s0.x - sc.x, -s0.y - sc.y);
        if (i == j) {
            v.x += mu - a.eps[int64_t(k) * nbm + i];
            v.y += w;
        }
        A[i][j] = v;
    }
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        // pivot: the largest |A_ij|, i >= j (first wave)
        if (tid < 64) {
            double best = -1.0;
            int bi = j;
            for (int i = j + tid; i < n; i += 64) {
                const double m = A[i][j].x * A[i][j].x + A[i][j].y * A[i][j].y;
                if (m > best) {
                    best = m;
                    bi = i;
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double ob = __shfl_xor(best, o);
                const int oi = __shfl_xor(bi, o);
                if (ob > best || (ob == best && oi < bi)) {
                    best = ob;
                    bi = oi;
                }
            }
            if (tid == 0) {
                ridx = bi;
                perm[j] = bi;
            }
        }
        __syncthreads();
        const int p = ridx;
        if (p != j)
            for (int c = tid; c < n; c += MD_T) {
                const double2 t = A[j][c];
                A[j][c] = A[p][c];
                A[p][c] = t;
            }
        __syncthreads();
        const double2 pv = A[j][j];
        if (pv.x == 0.0 && pv.y == 0.0) {  // uniform: every thread reads the same pivot
            singular = true;
            break;
        }
        // row j scaled by 1 / pivot, A_jj replaced by 1 / pivot; the column j saved for the update
        for (int c = tid; c < n; c += MD_T) {
            colj[c] = A[c][j];
            A[j][c] = md_div(c == j ? make_double2(1.0, 0.0) : A[j][c], pv);
        }
        __syncthreads();
        for (int e = tid; e < n * n; e += MD_T) {
            const int i = e / n, c = e % n;
            if (i == j) continue;
            const double2 f = colj[i];
            const double2 r = A[j][c];
            if (c == j) {
                A[i][c] = make_double2(-(f.x * r.x - f.y * r.y), -(f.x * r.y + f.y * r.x));
            } else {
                A[i][c].x -= f.x * r.x - f.y * r.y;
                A[i][c].y -= f.x * r.y + f.y * r.x;
            }
        }
        __syncthreads();
    }
    if (singular) {  // a NaN in part makes k_md_sum raise MSGW_FLAG_NAN
        if (tid == 0) part[int64_t(k) * a.niw + iw] = __longlong_as_double(0x7ff8000000000000ll);
        return;
    }
    // undo the row interchanges as column interchanges, last first
    for (int j = n - 1; j >= 0; --j) {
        const int p = perm[j];
        if (p != j)
            for (int r = tid; r < n; r += MD_T) {
                const double2 t = A[r][j];
                A[r][j] = A[r][p];
                A[r][p] = t;
            }
        __syncthreads();
    }
    if (tid < 64) {
        double tr = 0.0;
        for (int j = tid; j < n; j += 64) {
            const double E = a.eps[int64_t(k) * nbm + j] + S0[int64_t(j) * nbm + j].x - mu;
            const double2 ref = md_div(make_double2(1.0, 0.0), make_double2(-E, w));
            tr += A[j][j].x - ref.x;
        }
        for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o);
        if (tid == 0) part[int64_t(k) * a.niw + iw] = tr;
    }
    if (G_iw)
        for (int e = tid; e < nbm * nbm; e += MD_T) {
            const int i = e / nbm, j = e % nbm;
            G_iw[(int64_t(k) * nbm * nbm + e) * a.niw + iw] = (i < n && j < n) ? A[i][j] : make_double2(0.0, 0.0);
        }
}

// N(mu) = sum_k [sum_j n_F(E_jj) + (2/beta) sum_n part[k][n]], summed in a fixed order; then, by
// mode: 0 store as N(lo), 1 store as N(hi) and check the bracket, 2 halve the bracket, 3 the final
// mu (stored with N(mu), and the flags written out)
__global__ __launch_bounds__(MD_T) void k_md_sum(MdArgs a, double* st, const double* mu_in, int which,
                                                 int mode, const double* part, double* mu_out, double* n_out,
                                                 int* flags) {
    __shared__ double red[MD_T];
    const int tid = threadIdx.x;
    const double mu = md_mu(st, mu_in, which);
    double s = 0.0;
    int bad = 0;
    const int64_t nrow = int64_t(a.nk) * a.nbmax, npart = int64_t(a.nk) * a.niw;
    for (int64_t r = tid; r < nrow; r += MD_T) {
        const int k = int(r / a.nbmax), j = int(r % a.nbmax);
        if (j >= a.nb[k]) continue;
        const double E = a.eps[r] + a.S0[(int64_t(k) * a.nbmax + j) * a.nbmax + j].x - mu;
        s += md_fermi(E, a.beta);
    }
    double t = 0.0;
    for (int64_t i = tid; i < npart; i += MD_T) {
        const double v = part[i];
        if (!isfinite(v)) bad = 1;
        t += v;
    }
    red[tid] = s + (2.0 / a.beta) * t;
    __syncthreads();
    for (int h = MD_T / 2; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    __shared__ int sbad;
    if (tid == 0) sbad = 0;
    __syncthreads();
    if (bad) atomicOr(&sbad, 1);
    __syncthreads();
    if (tid != 0) return;
    const double N = red[0];
    int fl = int(st[ST_FL]) | (sbad ? MSGW_FLAG_NAN : 0);
    if (mode == 0) {
        st[ST_NLO] = N;
    } else if (mode == 1) {
        st[ST_NHI] = N;
        if (!(a.n_target >= st[ST_NLO] && a.n_target <= N)) fl |= MSGW_FLAG_NOBRACKET;
    } else if (mode == 2) {
        if (N < a.n_target)
            st[ST_LO] = mu;
        else
            st[ST_HI] = mu;
    } else {
        st[ST_MU] = mu;
        st[ST_N] = N;
        *mu_out = mu;
        *n_out = N;
        *flags = fl;
    }
    st[ST_FL] = double(fl);
}

// G(tau) for every (k, n, n') and tau: the diagonal reference plus the inverse sum of D
__global__ __launch_bounds__(MD_T) void k_md_gtau(MdArgs a, const double* st, const double* __restrict__ tau,
                                                  int ntau, const double2* __restrict__ G_iw,
                                                  double2* __restrict__ G_tau) {
    const int64_t id = int64_t(blockIdx.x) * MD_T + threadIdx.x;
    const int nbm = a.nbmax;
    const int64_t total = int64_t(a.nk) * nbm * nbm * ntau;
    if (id >= total) return;
    const int t = int(id % ntau);
    const int64_t e = id / ntau;  // (k, i, j)
    const int j = int(e % nbm), i = int((e / nbm) % nbm), k = int(e / (int64_t(nbm) * nbm));
    const int n = a.nb[k];
    if (i >= n || j >= n) {
        G_tau[id] = make_double2(0.0, 0.0);
        return;
    }
    const double mu = st[ST_MU];
    const double2* Gij = G_iw + ((int64_t(k) * nbm + i) * nbm + j) * a.niw;
    const double2* Gji = G_iw + ((int64_t(k) * nbm + j) * nbm + i) * a.niw;
    double Ei = 0.0;
    if (i == j) Ei = a.eps[int64_t(k) * nbm + i] + a.S0[(int64_t(k) * nbm + i) * nbm + i].x - mu;
    const double tt = tau[t];
    double re = 0.0, im = 0.0;
    for (int w = 0; w < a.niw; ++w) {
        const double om = (2.0 * w + 1.0) * kPi / a.beta;
        double2 d = Gij[w], dt = Gji[w];  // D_ij and D_ji (the diagonal carries the reference)
        if (i == j) {
            const double2 ref = md_div(make_double2(1.0, 0.0), make_double2(-Ei, om));
            d.x -= ref.x;
            d.y -= ref.y;
            dt = d;
        }
        double sn, cs;
        sincos(om * tt, &sn, &cs);
        // e^{-i w t} D_ij + e^{i w t} conj(D_ji)
        re += cs * d.x + sn * d.y + cs * dt.x + sn * dt.y;
        im += cs * d.y - sn * d.x - cs * dt.y + sn * dt.x;
    }
    re /= a.beta;
    im /= a.beta;
    if (i == j) {
        const double b = a.beta, aE = fabs(Ei);
        const double den = 1.0 + exp(-b * aE);
        re += Ei >= 0.0 ? -exp(-aE * tt) / den : -exp(-aE * (b - tt)) / den;
    }
    G_tau[id] = make_double2(re, im);
}

inline unsigned md_blocks(int64_t n) { return unsigned((n + MD_T - 1) / MD_T); }

}  // namespace

size_t mdyson_scratch_bytes(const Host& h) { return sizeof(double) * (8 + size_t(h.nk) * h.niw_f); }

void launch_dyson_matrix(const Dev& d, const Host& h, hipStream_t s, const double* eps, const double2* S0,
                         const double2* Sc, double n_target, int search, double* mu, double2* G_iw,
                         double2* G_tau, double* n_out, int* flags, double* scratch) {
    if (h.nbmax > MD_NB) throw Error(MSGW_ENOTSUP, "msgw_dyson_matrix: at most 64 bands");
    MdArgs a{eps, S0, Sc, d.nb, h.nk, h.nbmax, h.niw_f, h.beta, n_target};
    double* st = scratch;
    double* part = scratch + 8;
    const dim3 grid(h.nk, h.niw_f);
    MSGW_LAUNCH(k_md_prep, dim3(1), dim3(MD_T), 0, s, a, st);
    if (search) {
        MSGW_LAUNCH(k_md_eval, grid, dim3(MD_T), 0, s, a, st, mu, MU_LO, part, nullptr);
        MSGW_LAUNCH(k_md_sum, dim3(1), dim3(MD_T), 0, s, a, st, mu, MU_LO, 0, part, mu, n_out, flags);
        MSGW_LAUNCH(k_md_eval, grid, dim3(MD_T), 0, s, a, st, mu, MU_HI, part, nullptr);
        MSGW_LAUNCH(k_md_sum, dim3(1), dim3(MD_T), 0, s, a, st, mu, MU_HI, 1, part, mu, n_out, flags);
        for (int r = 0; r < MD_ROUNDS; ++r) {
            MSGW_LAUNCH(k_md_eval, grid, dim3(MD_T), 0, s, a, st, mu, MU_MID, part, nullptr);
            MSGW_LAUNCH(k_md_sum, dim3(1), dim3(MD_T), 0, s, a, st, mu, MU_MID, 2, part, mu, n_out, flags);
        }
        MSGW_LAUNCH(k_md_eval, grid, dim3(MD_T), 0, s, a, st, mu, MU_MID, part, G_iw);
        MSGW_LAUNCH(k_md_sum, dim3(1), dim3(MD_T), 0, s, a, st, mu, MU_MID, 3, part, mu, n_out, flags);
    } else {
        MSGW_LAUNCH(k_md_eval, grid, dim3(MD_T), 0, s, a, st, mu, MU_GIVEN, part, G_iw);
        MSGW_LAUNCH(k_md_sum, dim3(1), dim3(MD_T), 0, s, a, st, mu, MU_GIVEN, 3, part, mu, n_out, flags);
    }
    const int64_t total = int64_t(h.nk) * h.nbmax * h.nbmax * h.ntau;
    MSGW_LAUNCH(k_md_gtau, dim3(md_blocks(total)), dim3(MD_T), 0, s, a, st, d.tau, h.ntau, G_iw, G_tau);
    MSGW_HIP(hipGetLastError());
}

}  // namespace msgw
