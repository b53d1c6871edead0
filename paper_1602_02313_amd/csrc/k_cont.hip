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

}  // namespace msgw
