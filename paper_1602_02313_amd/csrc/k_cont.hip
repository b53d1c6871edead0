// Analytic continuation of Sigma^c(k, n, i w) to the real axis by a Pade approximant, FP64: the
// route the paper compares with its continuous-pole expansion (analytic continuation subsection of
// Sec. III.B), after the path.
//
// One 64-thread work-group (one wave) per state (k, n):
//   1. the continued-fraction coefficients of Vidberg and Serene through the n_pade lowest positive
//      Matsubara points z_j = i w_j: lane l keeps g(z_j) for j = l and j = l + 64; step p replaces
//      g(z_j), j >= p, by (g(z_{p-1}) - g(z_j)) / ((z_j - z_{p-1}) g(z_j)), with g(z_{p-1})
//      broadcast from its lane; when the steps are done g(z_j) = a_j;
//   2. C(w) = a_0 / (1 + a_1 (w - z_0) / (1 + a_2 (w - z_1) / ...)), nested from the last level,
//      with its derivative by the same recursion;
//   3. the quasiparticle equation x = e0 + Re C(x + i eta), e0 = eps + sigma_static - mu, by Newton
//      from x = e0 (every lane runs the same iteration), E = x + mu;
//   4. A(w_j) = -(1/pi) Im 1 / (w_j + i eta - e0 - C(w_j + i eta)), lanes over the grid.
#include "internal.h"

namespace msgw {
namespace {

constexpr int PADE_MAX = 128;
constexpr int QP_ITERS = 100;
constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// a / b with the larger component of b scaled to one (no overflow for large |b|)
__device__ __forceinline__ double2 cdivs(double2 a, double2 b) {
    const double s = fmax(fabs(b.x), fabs(b.y));
    const double bx = b.x / s, by = b.y / s;
    const double den = (bx * bx + by * by) * s;
    return make_double2((a.x * bx + a.y * by) / den, (a.y * bx - a.x * by) / den);
}

__device__ __forceinline__ double2 shfl2(double2 v, int src) {
    return make_double2(__shfl(v.x, src), __shfl(v.y, src));
}

__global__ __launch_bounds__(64) void k_pade(int nbmax, const int* __restrict__ nb, int niw, int n_pade, double beta,
                                             double eta, const double* __restrict__ eps,
                                             const double* __restrict__ sstat, const double2* __restrict__ sigc,
                                             const double* __restrict__ mu_p, int n_omega,
                                             const double* __restrict__ omega, double* __restrict__ A,
                                             double* __restrict__ Eqp, int* __restrict__ flags) {
    __shared__ double2 a[PADE_MAX];
    const int64_t b = blockIdx.x;
    const int k = int(b / nbmax), n = int(b % nbmax), lane = threadIdx.x;
    if (n >= nb[k]) {  // padding band: no state (uniform over the work-group)
        if (lane == 0) Eqp[b] = __longlong_as_double(0x7ff8000000000000LL);
        for (int j = lane; j < n_omega && A; j += 64) A[b * n_omega + j] = 0.0;
        return;
    }
    const double wstep = 2.0 * kPi / beta, w0 = kPi / beta;  // w_j = w0 + j wstep
    const double2* S = sigc + b * niw;
    double2 g[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int j = lane + 64 * s;
        g[s] = j < n_pade ? S[j] : make_double2(0.0, 0.0);
    }
    for (int p = 1; p < n_pade; ++p) {
        const int src = p - 1;
        const double2 prev = src < 64 ? shfl2(g[0], src) : shfl2(g[1], src - 64);  // g(z_{p-1}) = a_{p-1}
        const double zp = w0 + src * wstep;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int j = lane + 64 * s;
            if (j >= p && j < n_pade) {
                const double dz = (w0 + j * wstep) - zp;  // z_j - z_{p-1} = i dz
                const double2 den = make_double2(-dz * g[s].y, dz * g[s].x);  // i dz g(z_j)
                g[s] = cdivs(csub(prev, g[s]), den);
            }
        }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int j = lane + 64 * s;
        if (j < n_pade) a[j] = g[s];
    }
    __syncthreads();

    // C(w) and dC/dw by nesting: t = 1 + a_m (w - z_{m-1}) / t, m = n_pade - 1 .. 1; C = a_0 / t
    auto eval = [&](double2 w, double2& c, double2& dc) {
        double2 t = make_double2(1.0, 0.0), dt = make_double2(0.0, 0.0);
        for (int m = n_pade - 1; m >= 1; --m) {
            const double2 am = a[m];
            const double2 d = make_double2(w.x, w.y - (w0 + (m - 1) * wstep));  // w - z_{m-1}
            const double2 ad = cmul(am, d);
            const double2 q = cdivs(ad, t);                                     // a_m d / t
            // t' <- a_m / t - a_m d t' / t^2 = (a_m - q t') / t
            dt = cdivs(csub(am, cmul(q, dt)), t);
            t = make_double2(1.0 + q.x, q.y);
        }
        c = cdivs(a[0], t);
        dc = cdivs(make_double2(-(c.x * dt.x - c.y * dt.y), -(c.x * dt.y + c.y * dt.x)), t);  // -a_0 t' / t^2
    };

    const double mu = *mu_p;
    const double e0 = eps[b] + sstat[b] - mu;
    double x = e0;
    bool conv = false;
    for (int it = 0; it < QP_ITERS && !conv; ++it) {
        double2 c, dc;
        eval(make_double2(x, eta), c, dc);
        const double step = (x - e0 - c.x) / (1.0 - dc.x);
        x -= step;
        conv = fabs(step) <= 1e-12 * (1.0 + fabs(x));
    }
    if (lane == 0) {
        Eqp[b] = x + mu;
        if (!conv) atomicOr(flags, MSGW_FLAG_NOCONV);
    }
    for (int j = lane; j < n_omega && A; j += 64) {
        const double w = omega[j];
        double2 c, dc;
        eval(make_double2(w, eta), c, dc);
        const double2 den = make_double2(w - e0 - c.x, eta - c.y);  // w + i eta - e0 - C
        const double mag = den.x * den.x + den.y * den.y;
        A[b * n_omega + j] = den.y / mag / kPi;  // -Im(1/den) / pi
    }
}

__global__ void k_clear_flag(int* flags) { *flags = 0; }

}  // namespace

void launch_pade(const Dev& d, const Host& h, hipStream_t s, int n_pade, double eta, const double* eps,
                 const double* sstat, const void* sigc, const double* mu, int n_omega, const double* omega,
                 double* A, double* Eqp, int* flags) {
    MSGW_LAUNCH(k_clear_flag, dim3(1), dim3(1), 0, s, flags);
    MSGW_HIP(hipGetLastError());
    const int64_t nstate = int64_t(h.nk) * h.nbmax;
    if (nstate == 0) return;
    MSGW_LAUNCH(k_pade, dim3(unsigned(nstate)), dim3(64), 0, s, h.nbmax, d.nb, d.niw_f, n_pade, d.beta, eta, eps,
                sstat, (const double2*)sigc, mu, n_omega, omega, A, Eqp, flags);
    MSGW_HIP(hipGetLastError());
}


// =================================================================================================
// continuous-pole expansion (the paper's continuation, after Staar et al.)
// =================================================================================================
// Im Sigma(w) <= 0 is expanded in hat functions h_l at the interior points of a uniform real grid,
// Sigma(z) = -(1/pi) sum_l a_l Phi_l(z), Phi_l(z) = int h_l(w) / (w - z) dw (closed form below), and
// the a_l >= 0 minimise |B a - y|^2 + lam |a|^2 with B the real rows (Re, Im) of -Phi_l(i w_n) / pi,
// y the same rows of Sigma^c(i w_n) and lam = ridge * max_l (B^T B)_ll.  The design matrix and the
// Gram matrix Q = B^T B + lam I are shared by all states; each state solves its non-negative problem
// on the normal equations (Q, c = B^T y) by the active-set method of Lawson and Hanson.
namespace {

constexpr int CPE_MAX = 96;  // hats (interior grid points)

__device__ __forceinline__ double2 clog2(double2 a) { return make_double2(log(hypot(a.x, a.y)), atan2(a.y, a.x)); }

// Phi_l(z) and dPhi_l/dz for hat l (interior point l + 1 of the grid w_j = w0 + j dw)
__device__ void cpe_phi(double w0, double dw, int l, double2 z, double2& phi, double2& dphi) {
    const double lo = w0 + l * dw, mid = lo + dw, hi = mid + dw;
    // F(a, b, c) = (b - a) + (z - c) [ln(b - z) - ln(a - z)]; dF/dz = L + (z - c) (1/(a - z) - 1/(b - z))
    auto F = [&](double a, double b, double c, double2& v, double2& dv) {
        const double2 bz = make_double2(b - z.x, -z.y), az = make_double2(a - z.x, -z.y);
        const double2 lb = clog2(bz), la = clog2(az);
        const double2 L = make_double2(lb.x - la.x, lb.y - la.y);
        const double2 zc = make_double2(z.x - c, z.y);
        const double2 zl = cmul(zc, L);
        v = make_double2((b - a) + zl.x, zl.y);
        const double2 ia = cdivs(make_double2(1.0, 0.0), az), ib = cdivs(make_double2(1.0, 0.0), bz);
        const double2 t = cmul(zc, make_double2(ia.x - ib.x, ia.y - ib.y));
        dv = make_double2(L.x + t.x, L.y + t.y);
    };
    double2 f1, d1, f2, d2;
    F(lo, mid, lo, f1, d1);
    F(mid, hi, hi, f2, d2);
    phi = make_double2((f1.x - f2.x) / dw, (f1.y - f2.y) / dw);
    dphi = make_double2((d1.x - d2.x) / dw, (d1.y - d2.y) / dw);
}

// design matrix B [2 niw][nh]: one work-group per hat
__global__ __launch_bounds__(256) void k_cpe_basis(double w0, double dw, int nh, int niw, double beta,
                                                   double* __restrict__ B) {
    const int l = blockIdx.x;
    for (int n = threadIdx.x; n < niw; n += 256) {
        double2 phi, dphi;
        cpe_phi(w0, dw, l, make_double2(0.0, (2 * n + 1) * kPi / beta), phi, dphi);
        B[int64_t(n) * nh + l] = -phi.x / kPi;
        B[int64_t(niw + n) * nh + l] = -phi.y / kPi;
    }
}

// Gram matrix Q = B^T B: one work-group per row
__global__ __launch_bounds__(256) void k_cpe_gram(const double* __restrict__ B, int nh, int rows,
                                                  double* __restrict__ Q) {
    const int i = blockIdx.x;
    for (int j = threadIdx.x; j < nh; j += 256) {
        double s = 0.0;
        for (int r = 0; r < rows; ++r) s += B[int64_t(r) * nh + i] * B[int64_t(r) * nh + j];
        Q[int64_t(i) * nh + j] = s;
    }
}

// lam = ridge * max_l Q_ll, added to the diagonal
__global__ __launch_bounds__(64) void k_cpe_ridge(double* __restrict__ Q, int nh, double ridge) {
    if (threadIdx.x != 0) return;
    double m = 0.0;
    for (int l = 0; l < nh; ++l) m = fmax(m, Q[int64_t(l) * nh + l]);
    for (int l = 0; l < nh; ++l) Q[int64_t(l) * nh + l] += ridge * m;
}

// one work-group per state: the non-negative fit, then the quasiparticle energy and A(w)
__global__ __launch_bounds__(256) void k_cpe_state(int nbmax, const int* __restrict__ nb, int niw, int nh,
                                                   double w0, double dw, double eta,
                                                   const double* __restrict__ B, const double* __restrict__ Q,
                                                   const double* __restrict__ eps, const double* __restrict__ sstat,
                                                   const double2* __restrict__ sigc, const double* __restrict__ mu_p,
                                                   int n_omega, const double* __restrict__ omega,
                                                   double* __restrict__ A, double* __restrict__ Eqp,
                                                   double* __restrict__ coef, int* __restrict__ flags) {
    __shared__ double Lf[CPE_MAX][CPE_MAX + 1];  // Cholesky factor of Q restricted to the passive set
    __shared__ double c[CPE_MAX], x[CPE_MAX], s[CPE_MAX], w[CPE_MAX];
    __shared__ int pidx[CPE_MAX], inP[CPE_MAX];
    __shared__ int np_s, jmax_s, done_s, ok_s;
    __shared__ double red[4], red2[4];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int k = int(b / nbmax), n = int(b % nbmax);
    if (n >= nb[k]) {  // padding band (uniform over the work-group)
        if (tid == 0) Eqp[b] = __longlong_as_double(0x7ff8000000000000LL);
        for (int j = tid; j < n_omega && A; j += 256) A[b * n_omega + j] = 0.0;
        for (int l = tid; l < nh && coef; l += 256) coef[b * nh + l] = 0.0;
        return;
    }
    const double2* S = sigc + b * niw;
    for (int l = tid; l < nh; l += 256) {
        double acc = 0.0;
        for (int r = 0; r < niw; ++r) acc += B[int64_t(r) * nh + l] * S[r].x + B[int64_t(niw + r) * nh + l] * S[r].y;
        c[l] = acc;
        x[l] = 0.0;
        inP[l] = 0;
    }
    if (tid == 0) {
        np_s = 0;
        ok_s = 1;
    }
    __syncthreads();
    double cmax = 0.0;
    for (int l = 0; l < nh; ++l) cmax = fmax(cmax, fabs(c[l]));
    const double tol = 1e-13 * cmax;

    // s_P = Q_PP^-1 c_P by a Cholesky factorisation of Q_PP (all threads), s = 0 off P
    auto solve_passive = [&]() {
        const int p = np_s;
        for (int e = tid; e < p * p; e += 256) {
            const int i = e / p, j = e % p;
            Lf[i][j] = Q[int64_t(pidx[i]) * nh + pidx[j]];
        }
        __syncthreads();
        for (int kk = 0; kk < p; ++kk) {
            if (tid == 0) Lf[kk][kk] = sqrt(fmax(Lf[kk][kk], 1e-300));
            __syncthreads();
            for (int i = kk + 1 + tid; i < p; i += 256) Lf[i][kk] /= Lf[kk][kk];
            __syncthreads();
            for (int e = tid; e < (p - kk - 1) * (p - kk - 1); e += 256) {
                const int i = kk + 1 + e / (p - kk - 1), j = kk + 1 + e % (p - kk - 1);
                if (j <= i) Lf[i][j] -= Lf[i][kk] * Lf[j][kk];
            }
            __syncthreads();
        }
        if (tid == 0) {
            double y[CPE_MAX];
            for (int i = 0; i < p; ++i) {  // L y = c_P
                double t = c[pidx[i]];
                for (int j = 0; j < i; ++j) t -= Lf[i][j] * y[j];
                y[i] = t / Lf[i][i];
            }
            for (int i = p - 1; i >= 0; --i) {  // L^T s = y
                double t = y[i];
                for (int j = i + 1; j < p; ++j) t -= Lf[j][i] * y[j];
                y[i] = t / Lf[i][i];
            }
            for (int l = 0; l < nh; ++l) s[l] = 0.0;
            for (int i = 0; i < p; ++i) s[pidx[i]] = y[i];
        }
        __syncthreads();
    };

    for (int outer = 0; outer < 3 * nh; ++outer) {
        // gradient w = c - Q x; the most positive w_j off the passive set enters it
        for (int l = tid; l < nh; l += 256) {
            double t = c[l];
            for (int j = 0; j < nh; ++j) t -= Q[int64_t(l) * nh + j] * x[j];
            w[l] = t;
        }
        __syncthreads();
        if (tid == 0) {
            int jm = -1;
            double best = tol;
            for (int l = 0; l < nh; ++l)
                if (!inP[l] && w[l] > best) {
                    best = w[l];
                    jm = l;
                }
            jmax_s = jm;
            if (jm >= 0) {
                inP[jm] = 1;
                pidx[np_s++] = jm;
            }
        }
        __syncthreads();
        if (jmax_s < 0) break;  // optimal
        for (int inner = 0; inner <= nh; ++inner) {
            solve_passive();
            if (tid == 0) {
                // feasible: accept; else step towards s until a passive coefficient reaches zero
                double alpha = 2.0;
                int im = -1;
                for (int i = 0; i < np_s; ++i) {
                    const int l = pidx[i];
                    if (s[l] <= 0.0) {
                        const double t = x[l] / (x[l] - s[l]);
                        if (t < alpha) {
                            alpha = t;
                            im = l;
                        }
                    }
                }
                if (im < 0) {
                    for (int i = 0; i < np_s; ++i) x[pidx[i]] = s[pidx[i]];
                    done_s = 1;
                } else {
                    for (int i = 0; i < np_s; ++i) {
                        const int l = pidx[i];
                        x[l] += alpha * (s[l] - x[l]);
                    }
                    x[im] = 0.0;
                    int q2 = 0;  // drop the coefficients that reached zero from the passive set
                    for (int i = 0; i < np_s; ++i) {
                        const int l = pidx[i];
                        if (x[l] > 0.0) {
                            pidx[q2++] = l;
                        } else {
                            inP[l] = 0;
                            x[l] = 0.0;
                        }
                    }
                    np_s = q2;
                    done_s = 0;
                }
            }
            __syncthreads();
            if (done_s) break;
            if (inner == nh && tid == 0) ok_s = 0;
        }
        if (outer == 3 * nh - 1 && tid == 0) ok_s = 0;
    }
    __syncthreads();
    for (int l = tid; l < nh && coef; l += 256) coef[b * nh + l] = x[l];

    // Sigma(z) = -(1/pi) sum_l x_l Phi_l(z) (and its derivative), reduced over the work-group
    auto sigma = [&](double2 z, double2& sg, double2& dsg) {
        double sr = 0.0, si = 0.0, dr = 0.0, di = 0.0;
        for (int l = tid; l < nh; l += 256) {
            if (x[l] == 0.0) continue;
            double2 phi, dphi;
            cpe_phi(w0, dw, l, z, phi, dphi);
            sr -= x[l] * phi.x / kPi;
            si -= x[l] * phi.y / kPi;
            dr -= x[l] * dphi.x / kPi;
            di -= x[l] * dphi.y / kPi;
        }
        for (int o = 32; o > 0; o >>= 1) {
            sr += __shfl_xor(sr, o);
            si += __shfl_xor(si, o);
            dr += __shfl_xor(dr, o);
            di += __shfl_xor(di, o);
        }
        __syncthreads();
        if ((tid & 63) == 0) {
            red[tid >> 6] = sr;
            red2[tid >> 6] = dr;
        }
        __syncthreads();
        sg = make_double2(red[0] + red[1] + red[2] + red[3], 0.0);
        dsg = make_double2(red2[0] + red2[1] + red2[2] + red2[3], 0.0);
        __syncthreads();
        if ((tid & 63) == 0) {
            red[tid >> 6] = si;
            red2[tid >> 6] = di;
        }
        __syncthreads();
        sg.y = red[0] + red[1] + red[2] + red[3];
        dsg.y = red2[0] + red2[1] + red2[2] + red2[3];
    };
    const double mu = *mu_p;
    const double e0 = eps[b] + sstat[b] - mu;
    double xq = e0;
    bool conv = false;
    for (int it = 0; it < QP_ITERS && !conv; ++it) {  // every thread runs the same iteration
        double2 sg, dsg;
        sigma(make_double2(xq, eta), sg, dsg);
        const double step = (xq - e0 - sg.x) / (1.0 - dsg.x);
        xq -= step;
        conv = fabs(step) <= 1e-12 * (1.0 + fabs(xq));
    }
    if (tid == 0) {
        Eqp[b] = xq + mu;
        if (!conv || !ok_s) atomicOr(flags, MSGW_FLAG_NOCONV);
    }
    for (int j = tid; j < n_omega && A; j += 256) {  // A(w): one thread per grid point
        const double om = omega[j];
        double sr = 0.0, si = 0.0;
        for (int l = 0; l < nh; ++l) {
            if (x[l] == 0.0) continue;
            double2 phi, dphi;
            cpe_phi(w0, dw, l, make_double2(om, eta), phi, dphi);
            sr -= x[l] * phi.x / kPi;
            si -= x[l] * phi.y / kPi;
        }
        const double2 den = make_double2(om - e0 - sr, eta - si);
        A[b * n_omega + j] = den.y / (den.x * den.x + den.y * den.y) / kPi;
    }
}

}  // namespace

size_t cpe_scratch_bytes(const Host& h, int n_real) {
    const int nh = n_real - 2;
    return sizeof(double) * (size_t(2) * h.niw_f * nh + size_t(nh) * nh);
}

void launch_cpe(const Dev& d, const Host& h, hipStream_t s, int n_real, double w_min, double w_max, double ridge,
                double eta, const double* eps, const double* sstat, const void* sigc, const double* mu,
                int n_omega, const double* omega, double* A, double* Eqp, double* coef, int* flags) {
    const int nh = n_real - 2;
    if (nh > CPE_MAX) throw Error(MSGW_ENOTSUP, "continue_cpe: at most 98 real grid points");
    if (cpe_scratch_bytes(h, n_real) > scratch_mfma_bytes(d, h))
        throw Error(MSGW_ENOMEM, "workspace too small for the CPE design matrix");
    double* B = reinterpret_cast<double*>(scratch_mfma(d, h));
    double* Q = B + int64_t(2) * h.niw_f * nh;
    const double dw = (w_max - w_min) / (n_real - 1);
    MSGW_LAUNCH(k_clear_flag, dim3(1), dim3(1), 0, s, flags);
    MSGW_LAUNCH(k_cpe_basis, dim3(nh), dim3(256), 0, s, w_min, dw, nh, h.niw_f, d.beta, B);
    MSGW_LAUNCH(k_cpe_gram, dim3(nh), dim3(256), 0, s, (const double*)B, nh, 2 * h.niw_f, Q);
    MSGW_LAUNCH(k_cpe_ridge, dim3(1), dim3(64), 0, s, Q, nh, ridge);
    const int64_t nstate = int64_t(h.nk) * h.nbmax;
    MSGW_LAUNCH(k_cpe_state, dim3(unsigned(nstate)), dim3(256), 0, s, h.nbmax, d.nb, h.niw_f, nh, w_min, dw, eta,
                (const double*)B, (const double*)Q, eps, sstat, (const double2*)sigc, mu, n_omega, omega, A, Eqp,
                coef, flags);
    MSGW_HIP(hipGetLastError());
}

}  // namespace msgw
