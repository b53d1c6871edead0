// The paper's own tau-domain solvers, FP64: cross-checks of the Matsubara-axis path.
//
// W~ linear system (eq. tildeW): for one q, with A = v P and the trapezoid increments dtau_r,
//     sum_r [delta_pr 1 - A(tau_p - tau_r) dtau_r] W~(tau_r) = A(tau_p) v,
// one dense system of order Ntau * NI.  A at a difference of mesh points is the not-a-knot spline of
// P(tau) there (a difference below zero taken at + beta), contracted with host-built weights Phi:
//   k_wsys_build    the system [K | rhs] of each q, one work-group per (tau_p, tau_r) block;
//   gj_run          Gauss-Jordan with the right-hand sides (k_gj.hip);
//   k_wsys_extract  W~(q, tau_p)_IJ = X[(p, I), J].
//
// G Dyson on the dense uniform grid (eqs. dysongf, zxjk, zcjk, dysong): for one state (k, n), on the
// grid t_a = a h, h = tau_1 - tau_0, a = 0..N, with trapezoid increments dt_a,
//     sum_r [delta_pr - dt_r (G0(t_p - t_r) dsig + sum_s dt_s G0(t_p - t_s) Sigma^c(t_s - t_r))] G(t_r)
//         = G0(t_p),
// G0 the reference Green's function at E = eps - mu, dsig the static self-energy, Sigma^c splined
// onto the grid (weights Psi); negative arguments are antiperiodic; at a zero argument an interior
// node takes the mean of the two limits and an end node of the integration range the limit inside
// it (t_r at the ends of the t_2 integral, t_s at the ends of the t_1 integral):
//   k_dtau_vec      G0(E, a h) and Sigma^c(a h) of each state;
//   k_dtau_build    the system [K | G0] of each state, a thread per (p, r);
//   gj_run          Gauss-Jordan with the right-hand side;
//   k_dtau_extract  G at the mesh points (dense node idx_i = tau_i / h) and the status.
#include "internal.h"

namespace msgw {
namespace {

__global__ __launch_bounds__(256) void k_wsys_build(TauSysArgs a, const double2* __restrict__ P,
                                                    const double* __restrict__ v) {
    const int nt = a.ntau;
    const int p = blockIdx.x / nt, r = blockIdx.x % nt;
    const int qi = blockIdx.y, q = a.q0 + qi;
    const int NI = a.ni[q];
    const int n = nt * NI, ld = n + NI;
    const double2* Pq = P + (a.ppre[q] - a.ppre[a.q0]);
    const double* vq = v + (a.vpre[q] - a.vpre[a.q0]);
    double2* K = a.K + a.koff[qi];
    const double* phi = a.phi + (int64_t(p) * nt + r) * nt;
    const double dtr = a.dt[r];
    const int64_t nn = int64_t(NI) * NI;
    for (int e = threadIdx.x; e < NI * NI; e += 256) {
        const int I = e / NI, J = e % NI;
        double2 s = make_double2(0.0, 0.0);
        for (int i = 0; i < nt; ++i) {
            const double w = phi[i];
            const double2 x = Pq[i * nn + e];
            s.x += w * x.x;
            s.y += w * x.y;
        }
        const double f = -vq[I] * dtr;
        double2 kv = make_double2(f * s.x, f * s.y);
        if (p == r && I == J) kv.x += 1.0;
        K[int64_t(p * NI + I) * ld + r * NI + J] = kv;
        if (r == 0) {
            const double2 x = Pq[p * nn + e];
            const double vv = vq[I] * vq[J];
            K[int64_t(p * NI + I) * ld + n + J] = make_double2(vv * x.x, vv * x.y);
        }
    }
}

__global__ __launch_bounds__(256) void k_wsys_extract(TauSysArgs a, double2* __restrict__ Wt) {
    const int p = blockIdx.x, qi = blockIdx.y, q = a.q0 + qi;
    const int NI = a.ni[q];
    const int n = a.ntau * NI, ld = n + NI;
    const double2* K = a.K + a.koff[qi];
    double2* W = Wt + (a.ppre[q] - a.ppre[a.q0]) + int64_t(p) * NI * NI;
    for (int e = threadIdx.x; e < NI * NI; e += 256) {
        const int I = e / NI, J = e % NI;
        W[e] = K[int64_t(p * NI + I) * ld + n + J];
    }
}

__global__ __launch_bounds__(256) void k_dtau_vec(TauSysArgs a, const double* __restrict__ eps,
                                                  const double* __restrict__ mu, const double* __restrict__ sig) {
    const int s = blockIdx.x;
    const int k = a.st_k[s], nband = a.st_n[s];
    const int nd = a.nd, nt = a.ntau;
    const double E = eps[int64_t(k) * a.nbmax + nband] - *mu;
    const double* sg = sig + (int64_t(k) * a.nbmax + nband) * nt;
    double* gp = a.gpos + int64_t(s) * nd;
    double* sc = a.scd + int64_t(s) * nd;
    for (int m = threadIdx.x; m < nd; m += 256) {
        gp[m] = g0_tau(E, a.td[m], a.beta);
        const double* psi = a.psi + int64_t(m) * nt;
        double acc = 0.0;
        for (int i = 0; i < nt; ++i) acc += psi[i] * sg[i];
        sc[m] = acc;
    }
}

constexpr int DT_ROWS = 4;  // rows p of the system per work-group

__global__ __launch_bounds__(256) void k_dtau_build(TauSysArgs a, const double* __restrict__ sstat) {
    extern __shared__ double sh[];
    const int s = blockIdx.y;
    const int nd = a.nd, N = nd - 1, ld = nd + 1;
    double* gp = sh;           // G0(E, a h), a = 0..N
    double* sc = sh + nd;      // Sigma^c(a h)
    double* dt = sh + 2 * nd;  // trapezoid increments
    for (int m = threadIdx.x; m < nd; m += 256) {
        gp[m] = a.gpos[int64_t(s) * nd + m];
        sc[m] = a.scd[int64_t(s) * nd + m];
        dt[m] = a.dtd[m];
    }
    __syncthreads();
    const double dsig = sstat[int64_t(a.st_k[s]) * a.nbmax + a.st_n[s]];
    // the values at zero argument: the limits from above (0+) and below (0-, antiperiodic) and their mean
    const double g_p = gp[0], g_m = -gp[N], g_0 = 0.5 * (g_p + g_m);
    const double s_p = sc[0], s_m = -sc[N], s_0 = 0.5 * (s_p + s_m);
    // G0(t_x - t_y) as the integrand over t_y, Sigma^c(t_x - t_y) as the integrand over t_x
    auto G0c = [&](int x, int y) {
        if (x > y) return gp[x - y];
        if (x < y) return -gp[x - y + N];
        return x == 0 ? g_m : (x == N ? g_p : g_0);
    };
    auto Scr = [&](int x, int y) {
        if (x > y) return sc[x - y];
        if (x < y) return -sc[x - y + N];
        return x == 0 ? s_p : (x == N ? s_m : s_0);
    };
    double2* K = a.K + int64_t(s) * nd * ld;
    const int p0 = blockIdx.x * DT_ROWS;
    for (int e = threadIdx.x; e < DT_ROWS * ld; e += 256) {
        const int p = p0 + e / ld, r = e % ld;
        if (p >= nd) break;
        double val;
        if (r == nd) {
            val = gp[p];  // G0(t_p) on [0, beta]
        } else {
            double zc = 0.0;
            for (int t = 0; t < nd; ++t) zc += dt[t] * G0c(p, t) * Scr(t, r);
            val = (p == r ? 1.0 : 0.0) - dt[r] * (G0c(p, r) * dsig + zc);
        }
        K[int64_t(p) * ld + r] = make_double2(val, 0.0);
    }
}

__global__ __launch_bounds__(256) void k_dtau_extract(TauSysArgs a, double* __restrict__ G_tau,
                                                      int* __restrict__ info) {
    const int s = blockIdx.x;
    const int k = a.st_k[s], nband = a.st_n[s];
    const int nd = a.nd, ld = nd + 1;
    const double2* K = a.K + int64_t(s) * nd * ld;
    double* G = G_tau + (int64_t(k) * a.nbmax + nband) * a.ntau;
    for (int i = threadIdx.x; i < a.ntau; i += 256) G[i] = K[int64_t(a.idx[i]) * ld + nd].x;
    if (threadIdx.x == 0) info[(k - a.k0) * a.nbmax + nband] = a.ginfo[s];
}

__global__ void k_tau_zero(int* p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

}  // namespace

void launch_wt_tau_system(const TauSysArgs& a, hipStream_t s, int nq, int nmax, int ldmax, const void* P_tau,
                          const double* v, void* Wt_tau) {
    MSGW_LAUNCH(k_wsys_build, dim3(a.ntau * a.ntau, nq), dim3(256), 0, s, a, (const double2*)P_tau, v);
    GjArgs g;
    g.A = a.K;
    g.mode = GJ_SOLVE;
    g.tn = a.tn;
    g.tld = a.tld;
    g.toff = a.koff;
    g.perm = a.perm;
    g.pmax = nmax;
    g.info = a.ginfo;
    gj_run(g, nq, nmax, ldmax, s);
    MSGW_LAUNCH(k_wsys_extract, dim3(a.ntau, nq), dim3(256), 0, s, a, (double2*)Wt_tau);
    MSGW_HIP(hipGetLastError());
}

void launch_dyson_tau(const TauSysArgs& a, hipStream_t s, int nstates, int nkc, const double* eps,
                      const double* sstat, const double* mu, const double* Sigma_c_tau, double* G_tau, int* info) {
    MSGW_LAUNCH(k_tau_zero, dim3((nkc * a.nbmax + 255) / 256), dim3(256), 0, s, info, nkc * a.nbmax);
    if (nstates == 0) return;
    MSGW_LAUNCH(k_dtau_vec, dim3(nstates), dim3(256), 0, s, a, eps, mu, Sigma_c_tau);
    const size_t shm = sizeof(double) * 3 * size_t(a.nd);
    MSGW_LAUNCH(k_dtau_build, dim3((a.nd + DT_ROWS - 1) / DT_ROWS, nstates), dim3(256), shm, s, a, sstat);
    GjArgs g;
    g.A = a.K;
    g.mode = GJ_SOLVE;
    g.tn = a.tn;
    g.tld = a.tld;
    g.toff = a.koff;
    g.perm = a.perm;
    g.pmax = a.nd;
    g.info = a.ginfo;
    gj_run(g, nstates, a.nd, a.nd + 1, s);
    MSGW_LAUNCH(k_dtau_extract, dim3(nstates), dim3(256), 0, s, a, G_tau, info);
    MSGW_HIP(hipGetLastError());
}

}  // namespace msgw
