// Host side of the C ABI: context, validation, FP64 transform weights, workspace.
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <sstream>

#include "internal.h"

using cplx = std::complex<double>;
using namespace msgw;

struct msgw_ctx {
    int device = 0;
    void* noalloc = nullptr;  // device address of the static scratch of msgw_dyson_noalloc on `device`
    std::string err;
    bool have_problem = false;
    Host h;
    // host tables
    std::vector<cplx> wf, wb, ef, eb;
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_ready = false;
    Dev d;
    int variant[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};  // [op][precision] tile shape of the MFMA paths
    // what the last contraction call left in the split-precision scratch (the per-q operands a call
    // with reuse_prepared may reuse); op = -1: nothing reusable
    struct Prepared {
        int op = -1, q0 = 0, nq = 0, precision = 0, variant = 0;
    } prep;
    // crystal symmetry (msgw_set_symmetry): the irreducible q and the stars
    bool sym_set = false;
    int cubic_ni = 0;  // NI of the cubic generator's tables in the workspace (0: none)
    std::vector<int> sym_ibz, sym_off;  // representatives; star of sym_ibz[i] = sym_star[sym_off[i] .. sym_off[i+1])
    std::vector<int> sym_star, sym_rep_of;  // star members grouped; representative index of every q
};

namespace {

constexpr double kPi = 3.14159265358979323846;

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// ---- dense LU with partial pivoting (host, small systems) ----
void lu_solve_multi(std::vector<double> A, int n, std::vector<double>& B, int nrhs) {
    // A: n*n row-major; B: n*nrhs row-major, overwritten with the solution.
    std::vector<int> piv(n);
    for (int j = 0; j < n; ++j) {
        int p = j;
        for (int i = j + 1; i < n; ++i)
            if (std::fabs(A[i * n + j]) > std::fabs(A[p * n + j])) p = i;
        if (A[p * n + j] == 0.0) throw Error(MSGW_ESHAPE, "singular spline system (repeated tau?)");
        if (p != j) {
            for (int c = 0; c < n; ++c) std::swap(A[j * n + c], A[p * n + c]);
            for (int c = 0; c < nrhs; ++c) std::swap(B[j * nrhs + c], B[p * nrhs + c]);
        }
        for (int i = j + 1; i < n; ++i) {
            double f = A[i * n + j] / A[j * n + j];
            if (f == 0.0) continue;
            for (int c = j; c < n; ++c) A[i * n + c] -= f * A[j * n + c];
            for (int c = 0; c < nrhs; ++c) B[i * nrhs + c] -= f * B[j * nrhs + c];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        for (int c = 0; c < nrhs; ++c) {
            double s = B[i * nrhs + c];
            for (int k = i + 1; k < n; ++k) s -= A[i * n + k] * B[k * nrhs + c];
            B[i * nrhs + c] = s / A[i * n + i];
        }
    }
}

// Moments J_p(w, h) = int_0^h t^p e^{i w t} dt, p = 0..3.
void moments(double w, double h, cplx J[4]) {
    const cplx I(0.0, 1.0);
    if (std::fabs(w * h) < 0.5) {
        // series: J_p = h^{p+1} sum_j (i w h)^j / (j! (p + j + 1))
        cplx z = I * (w * h);
        for (int p = 0; p < 4; ++p) {
            cplx term = 1.0, acc = 0.0;
            for (int j = 0; j < 30; ++j) {
                if (j) term *= z / double(j);
                acc += term / double(p + j + 1);
            }
            J[p] = acc * std::pow(h, p + 1);
        }
    } else {
        cplx e = std::exp(I * (w * h));
        cplx iw = I * w;
        J[0] = (e - 1.0) / iw;
        for (int p = 1; p < 4; ++p) J[p] = (std::pow(h, p) * e - double(p) * J[p - 1]) / iw;
    }
}

// Second derivatives of the not-a-knot cubic spline of f on the mesh as a linear map of the values:
// sig = X f, X [n][n] row-major.
std::vector<double> spline_second_derivs(const std::vector<double>& tau) {
    const int n = (int)tau.size();
    std::vector<double> h(n - 1);
    for (int i = 0; i + 1 < n; ++i) h[i] = tau[i + 1] - tau[i];
    // A sig = Rm f with the not-a-knot end conditions (third derivative continuous at tau_1, tau_{n-2})
    std::vector<double> A(size_t(n) * n, 0.0), X(size_t(n) * n, 0.0);
    A[0 * n + 0] = -1.0 / h[0];
    A[0 * n + 1] = 1.0 / h[0] + 1.0 / h[1];
    A[0 * n + 2] = -1.0 / h[1];
    for (int i = 1; i < n - 1; ++i) {
        A[i * n + i - 1] = h[i - 1];
        A[i * n + i] = 2.0 * (h[i - 1] + h[i]);
        A[i * n + i + 1] = h[i];
        X[i * n + i + 1] += 6.0 / h[i];
        X[i * n + i] += -6.0 / h[i] - 6.0 / h[i - 1];
        X[i * n + i - 1] += 6.0 / h[i - 1];
    }
    A[(n - 1) * n + n - 3] = -1.0 / h[n - 3];
    A[(n - 1) * n + n - 2] = 1.0 / h[n - 3] + 1.0 / h[n - 2];
    A[(n - 1) * n + n - 1] = -1.0 / h[n - 2];
    lu_solve_multi(A, n, X, n);  // X[i][j] = d sig_i / d f_j
    return X;
}

// Weights w[j] with S(x) = sum_j w[j] f_j for the spline of f at x in [tau_0, tau_{n-1}]: on the
// interval [tau_i, tau_{i+1}], t = x - tau_i, S = f_i + b t + (s_i / 2) t^2 + (s_{i+1} - s_i) t^3 / (6 h)
// with b = (f_{i+1} - f_i) / h - h (2 s_i + s_{i+1}) / 6.
void spline_eval_weights(const std::vector<double>& tau, const std::vector<double>& X, double x, double* w) {
    const int n = (int)tau.size();
    int i = int(std::upper_bound(tau.begin(), tau.end(), x) - tau.begin()) - 1;
    i = std::min(std::max(i, 0), n - 2);
    const double h = tau[i + 1] - tau[i], t = x - tau[i];
    for (int j = 0; j < n; ++j) {
        const double si = X[size_t(i) * n + j], si1 = X[size_t(i + 1) * n + j];
        w[j] = t * (-h * (2.0 * si + si1) / 6.0) + t * t * (si / 2.0) + t * t * t * ((si1 - si) / (6.0 * h));
    }
    w[i] += 1.0 - t / h;
    w[i + 1] += t / h;
}

// Forward weights W[n][j]: F(i w_n) = sum_j W[n][j] f_j for the not-a-knot cubic spline of f
// integrated exactly against e^{i w tau} over [0, beta].
void spline_filon_weights(const std::vector<double>& tau, int niw, bool fermion, double beta,
                          std::vector<cplx>& W) {
    const int n = (int)tau.size();
    const int N = n - 1;  // intervals
    std::vector<double> h(N);
    for (int i = 0; i < N; ++i) h[i] = tau[i + 1] - tau[i];
    const std::vector<double> X = spline_second_derivs(tau);
    W.assign(size_t(niw) * n, cplx(0.0));
    for (int w = 0; w < niw; ++w) {
        double om = (fermion ? (2.0 * w + 1.0) : 2.0 * w) * kPi / beta;
        for (int i = 0; i < N; ++i) {
            cplx J[4];
            moments(om, h[i], J);
            cplx ph = std::exp(cplx(0.0, om * tau[i]));
            for (int p = 0; p < 4; ++p) J[p] *= ph;
            // a_i = f_i ; b_i = (f_{i+1}-f_i)/h - h (2 s_i + s_{i+1})/6 ; c_i = s_i/2 ;
            // d_i = (s_{i+1} - s_i)/(6h)
            cplx* row = &W[size_t(w) * n];
            row[i] += J[0];
            row[i + 1] += J[1] / h[i];
            row[i] -= J[1] / h[i];
            for (int j = 0; j < n; ++j) {
                double si = X[i * n + j], si1 = X[(i + 1) * n + j];
                if (si == 0.0 && si1 == 0.0) continue;
                row[j] += J[1] * (-h[i] * (2.0 * si + si1) / 6.0) + J[2] * (si / 2.0) +
                          J[3] * ((si1 - si) / (6.0 * h[i]));
            }
        }
    }
}

void set_err(msgw_ctx* c, const std::string& m) {
    if (c) c->err = m;
}

template <class F>
int guarded(msgw_ctx* c, F&& f) {
    if (!c) return MSGW_EINVAL;
    try {
        c->err.clear();
        f();
        return MSGW_OK;
    } catch (const Error& e) {
        set_err(c, e.what());
        return e.code;
    } catch (const std::exception& e) {
        set_err(c, e.what());
        return MSGW_EINVAL;
    }
}

void need(bool cond, int code, const std::string& msg) {
    if (!cond) throw Error(code, msg);
}

void require_ready(msgw_ctx* c) {
    need(c->have_problem, MSGW_EINVAL, "no problem set (msgw_set_problem)");
    need(c->ws_ready, MSGW_ENOMEM, "no workspace attached (msgw_set_workspace)");
    MSGW_HIP(hipSetDevice(c->device));
}

void check_qrange(msgw_ctx* c, int q0, int nq) {
    need(q0 >= 0 && nq >= 1 && q0 + nq <= c->h.nk, MSGW_EINVAL, "q range outside [0, nk)");
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ---- crystal symmetry: the 48 operations of O_h and the closed-shell product basis of the cubic
// input generator ----
struct IMat {
    int m[3][3];
};
std::vector<IMat> cubic_ops() {
    static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    std::vector<IMat> out;
    for (const auto& p : perms)
        for (int sgn = 0; sgn < 8; ++sgn) {
            IMat R{};
            for (int r = 0; r < 3; ++r) R.m[r][p[r]] = (sgn >> r) & 1 ? -1 : 1;
            out.push_back(R);
        }
    return out;
}
// the first ni vectors G of Z^3 by |G|^2, then lexicographically; empty if ni does not close a shell
std::vector<std::array<int, 3>> shell_basis(int ni) {
    int R = 1;
    while ((2 * R + 1) * (2 * R + 1) * (2 * R + 1) < 4 * ni || R * R * R < ni) ++R;
    std::vector<std::array<int, 3>> g;
    for (int a = -R; a <= R; ++a)
        for (int b = -R; b <= R; ++b)
            for (int c = -R; c <= R; ++c) g.push_back({a, b, c});
    auto n2 = [](const std::array<int, 3>& x) { return x[0] * x[0] + x[1] * x[1] + x[2] * x[2]; };
    std::sort(g.begin(), g.end(), [&](const std::array<int, 3>& x, const std::array<int, 3>& y) {
        return n2(x) != n2(y) ? n2(x) < n2(y) : x < y;
    });
    if (ni < (int)g.size() && n2(g[ni]) == n2(g[ni - 1])) return {};
    g.resize(ni);
    return g;
}

// ---- the tau-domain solvers: host tables and the layout of the caller's work buffer ----
// Trapezoid increments of a grid: (t_{i+1} - t_{i-1}) / 2 inside, half intervals at the ends.
std::vector<double> trapezoid_increments(const std::vector<double>& t) {
    const int n = (int)t.size();
    std::vector<double> d(n);
    for (int i = 1; i + 1 < n; ++i) d[i] = 0.5 * (t[i + 1] - t[i - 1]);
    d[0] = 0.5 * (t[1] - t[0]);
    d[n - 1] = 0.5 * (t[n - 1] - t[n - 2]);
    return d;
}

struct TauSysLayout {
    size_t total = 0;
    // offsets (bytes) of each table in the work buffer
    size_t phi = 0, dt = 0, psi = 0, td = 0, dtd = 0, idx = 0, st_k = 0, st_n = 0, gpos = 0, scd = 0;
    size_t tn = 0, tld = 0, koff = 0, perm = 0, ginfo = 0, K = 0;
    int count = 0, nmax = 0, ldmax = 0, nd = 0;
    std::vector<int> tn_h, tld_h, st_k_h, st_n_h;
    std::vector<int64_t> koff_h;
};

// Dense uniform grid of the Dyson solve: spacing tau_1 - tau_0 from 0 to beta; every mesh point must
// be one of its nodes.  Returns the number of nodes (0 if the mesh does not allow it) and idx.
int dense_grid(const Host& h, std::vector<int>* idx) {
    const double step = h.tau[1] - h.tau[0];
    const double nf = h.beta / step;
    const long N = std::lround(nf);
    if (N < 1 || std::fabs(N * step - h.beta) > 1e-9 * h.beta) return 0;
    if (N + 1 > kDysonTauMaxGrid) return int(std::min<long>(N + 1, 1L << 30));
    if (idx) idx->resize(h.ntau);
    for (int i = 0; i < h.ntau; ++i) {
        const long a = std::lround(h.tau[i] / step);
        if (std::fabs(a * step - h.tau[i]) > 1e-9 * h.beta) return 0;
        if (idx) (*idx)[i] = int(a);
    }
    return int(N + 1);
}

// which = MSGW_TS_WTILDE: first = q0, count = nq; MSGW_TS_DYSON: first = k0, count = nkc
TauSysLayout tau_sys_layout(const Host& h, int which, int first, int count) {
    TauSysLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const int nt = h.ntau;
    if (which == MSGW_TS_WTILDE) {
        L.count = count;
        for (int q = first; q < first + count; ++q) {
            const int n = nt * h.ni[q];
            need(n <= kGjMaxN, MSGW_ENOTSUP, "W~ tau system: ntau * NI_q above 4096");
            L.tn_h.push_back(n);
            L.tld_h.push_back(n + h.ni[q]);
            L.nmax = std::max(L.nmax, n);
            L.ldmax = std::max(L.ldmax, n + h.ni[q]);
        }
        L.phi = take(sizeof(double) * size_t(nt) * nt * nt);
        L.dt = take(sizeof(double) * nt);
    } else {
        const int nd = dense_grid(h, nullptr);
        need(nd > 0, MSGW_ESHAPE, "tau Dyson: beta and every tau_i must be multiples of tau_1 - tau_0");
        need(nd <= kDysonTauMaxGrid, MSGW_ENOTSUP, "tau Dyson: more than 2048 dense grid points");
        L.nd = nd;
        for (int k = first; k < first + count; ++k)
            for (int n = 0; n < h.nb[k]; ++n) {
                L.st_k_h.push_back(k);
                L.st_n_h.push_back(n);
                L.tn_h.push_back(nd);
                L.tld_h.push_back(nd + 1);
            }
        L.count = (int)L.tn_h.size();
        need(L.count <= 65535, MSGW_ENOTSUP, "tau Dyson: more than 65535 states in one call (use a smaller k range)");
        L.nmax = nd;
        L.ldmax = nd + 1;
        L.psi = take(sizeof(double) * size_t(nd) * nt);
        L.td = take(sizeof(double) * nd);
        L.dtd = take(sizeof(double) * nd);
        L.idx = take(sizeof(int) * nt);
        L.st_k = take(sizeof(int) * L.count);
        L.st_n = take(sizeof(int) * L.count);
        L.gpos = take(sizeof(double) * size_t(L.count) * nd);
        L.scd = take(sizeof(double) * size_t(L.count) * nd);
    }
    int64_t koff = 0;
    for (int b = 0; b < L.count; ++b) {
        L.koff_h.push_back(koff);
        koff += int64_t(L.tn_h[b]) * L.tld_h[b];
    }
    L.tn = take(sizeof(int) * L.count);
    L.tld = take(sizeof(int) * L.count);
    L.koff = take(sizeof(int64_t) * L.count);
    L.perm = take(sizeof(int) * size_t(L.count) * L.nmax);
    L.ginfo = take(sizeof(int) * L.count);
    L.K = take(sizeof(double2) * size_t(koff));
    L.total = off;
    return L;
}

}  // namespace

extern "C" {

int msgw_create(msgw_ctx** out, int hip_device) {
    if (!out) return MSGW_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return MSGW_EHIP;
    if (hip_device < 0 || hip_device >= n) return MSGW_EINVAL;
    auto* c = new (std::nothrow) msgw_ctx();
    if (!c) return MSGW_EINVAL;
    c->device = hip_device;
    try {
        c->noalloc = noalloc_scratch(hip_device);  // once per device, that device current for the lookup
    } catch (...) {
        delete c;
        return MSGW_EHIP;
    }
    *out = c;
    return MSGW_OK;
}

int msgw_destroy(msgw_ctx* c) {
    delete c;
    return MSGW_OK;
}

const char* msgw_last_error(const msgw_ctx* c) { return c ? c->err.c_str() : "null context"; }

int msgw_set_problem(msgw_ctx* c, const msgw_problem* p) {
    return guarded(c, [&] {
        need(p != nullptr, MSGW_EINVAL, "null problem");
        need(p->kmq && p->nb && p->ni && p->tau, MSGW_EINVAL, "null table in problem");
        need(p->nk >= 1, MSGW_ESHAPE, "nk must be >= 1");
        need(p->ntau >= MSGW_MIN_NTAU, MSGW_ESHAPE, "ntau must be >= 4 (not-a-knot spline)");
        need(p->niw_f >= 1 && p->niw_b >= 1, MSGW_ESHAPE, "niw_f and niw_b must be >= 1");
        need(p->beta > 0 && std::isfinite(p->beta), MSGW_EINVAL, "beta must be positive");
        need(std::isfinite(p->scale), MSGW_EINVAL, "scale must be finite");
        need(p->sigma_mode == MSGW_SIGMA_DIAG || p->sigma_mode == MSGW_SIGMA_FULL, MSGW_EINVAL,
             "bad sigma_mode");
        Host h;
        h.nk = p->nk;
        h.ntau = p->ntau;
        h.niw_f = p->niw_f;
        h.niw_b = p->niw_b;
        h.beta = p->beta;
        h.scale = p->scale;
        h.sigma_mode = p->sigma_mode;
        h.kmq.assign(p->kmq, p->kmq + size_t(p->nk) * p->nk);
        h.nb.assign(p->nb, p->nb + p->nk);
        h.ni.assign(p->ni, p->ni + p->nk);
        h.tau.assign(p->tau, p->tau + p->ntau);
        for (int v : h.kmq) need(v >= 0 && v < h.nk, MSGW_EINVAL, "kmq entry out of range");
        for (int v : h.nb) need(v >= 1 && v <= MSGW_MAX_NB, MSGW_ESHAPE, "Nb_k outside [1, 1024]");
        for (int v : h.ni) need(v >= 1 && v <= MSGW_MAX_NI, MSGW_ESHAPE, "NI_q outside [1, 1024]");
        need(h.tau[0] == 0.0, MSGW_ESHAPE, "tau[0] must be 0");
        need(std::fabs(h.tau.back() - h.beta) <= 1e-12 * h.beta, MSGW_ESHAPE, "tau[-1] must be beta");
        for (int i = 0; i + 1 < h.ntau; ++i)
            need(h.tau[i + 1] > h.tau[i], MSGW_ESHAPE, "tau must be strictly increasing");
        for (int i = 0; i < h.ntau; ++i)
            need(std::fabs(h.tau[i] + h.tau[h.ntau - 1 - i] - h.beta) <= 1e-12 * h.beta,
                 MSGW_ESHAPE, "tau mesh is not mirror symmetric (tau_i + tau_{N-i} != beta)");
        h.nbmax = *std::max_element(h.nb.begin(), h.nb.end());
        h.nimax = *std::max_element(h.ni.begin(), h.ni.end());
        const int nk = h.nk;
        h.moff.assign(size_t(nk) * nk, 0);
        h.mpre.assign(nk + 1, 0);
        h.ppre.assign(nk + 1, 0);
        h.wpre.assign(nk + 1, 0);
        h.vpre.assign(nk + 1, 0);
        for (int q = 0; q < nk; ++q) {
            int64_t off = 0;
            for (int k = 0; k < nk; ++k) {
                h.moff[size_t(q) * nk + k] = off;
                off += int64_t(h.ni[q]) * h.nb[k] * h.nb[h.kmq[size_t(q) * nk + k]];
            }
            h.mpre[q + 1] = h.mpre[q] + off;
            h.ppre[q + 1] = h.ppre[q] + int64_t(h.ntau) * h.ni[q] * h.ni[q];
            h.wpre[q + 1] = h.wpre[q] + int64_t(h.niw_b) * h.ni[q] * h.ni[q];
            h.vpre[q + 1] = h.vpre[q] + h.ni[q];
        }
        // transform tables
        std::vector<cplx> wf, wb;
        spline_filon_weights(h.tau, h.niw_f, true, h.beta, wf);
        spline_filon_weights(h.tau, h.niw_b, false, h.beta, wb);
        std::vector<cplx> ef(size_t(h.ntau) * h.niw_f), eb(size_t(h.ntau) * h.niw_b);
        for (int i = 0; i < h.ntau; ++i) {
            for (int n = 0; n < h.niw_f; ++n)
                ef[size_t(i) * h.niw_f + n] = std::exp(cplx(0.0, -(2.0 * n + 1.0) * kPi / h.beta * h.tau[i]));
            for (int n = 0; n < h.niw_b; ++n)
                eb[size_t(i) * h.niw_b + n] = std::exp(cplx(0.0, -(2.0 * n) * kPi / h.beta * h.tau[i]));
        }
        c->h = std::move(h);
        c->wf = std::move(wf);
        c->wb = std::move(wb);
        c->ef = std::move(ef);
        c->eb = std::move(eb);
        c->have_problem = true;
        c->sym_set = false;
        c->prep = msgw_ctx::Prepared();
        c->ws_ready = false;
        c->ws = nullptr;
        c->ws_bytes = 0;
    });
}

static size_t tables_bytes(const Host& h) {
    size_t b = 0;
    b += align_up(sizeof(int) * size_t(h.nk) * h.nk) + align_up(sizeof(int) * h.nk);      // symmetry maps
    b += align_up(sizeof(int) * size_t(kMaxRot) * h.nk) + align_up(sizeof(int) * size_t(kMaxRot) * h.nimax) +
         align_up(sizeof(int) * h.nimax);                                                    // cubic generator
    b += align_up(sizeof(double) * h.ntau);
    b += align_up(sizeof(double2) * size_t(h.niw_f) * h.ntau) * 2;
    b += align_up(sizeof(double2) * size_t(h.niw_b) * h.ntau) * 2;
    b += align_up(sizeof(int) * size_t(h.nk) * h.nk);
    b += align_up(sizeof(int) * h.nk) * 2;
    b += align_up(sizeof(int64_t) * size_t(h.nk) * h.nk);
    b += align_up(sizeof(int64_t) * (h.nk + 1)) * 4;
    return b;
}

static size_t scratch_needed(const Host& h, int nq_max) {
    return scratch_E_bytes(h) + align_up(std::max({mfma_scratch_bytes(h, nq_max), cpe_scratch_bytes(h, 98),
                                                   screen_scratch_bytes(h, nq_max),
                                                   sigfull_split_scratch_bytes(h)}));
}

int msgw_workspace_size(msgw_ctx* c, int nq_max, size_t* bytes) {
    return guarded(c, [&] {
        need(c->have_problem, MSGW_EINVAL, "no problem set");
        need(bytes != nullptr, MSGW_EINVAL, "null bytes");
        need(nq_max >= 1 && nq_max <= c->h.nk, MSGW_EINVAL, "nq_max outside [1, nk]");
        *bytes = tables_bytes(c->h) + scratch_needed(c->h, nq_max);
    });
}

int msgw_set_workspace(msgw_ctx* c, void* dptr, size_t bytes) {
    return guarded(c, [&] {
        need(c->have_problem, MSGW_EINVAL, "no problem set");
        need(dptr != nullptr, MSGW_EINVAL, "null workspace");
        need((reinterpret_cast<uintptr_t>(dptr) & 255) == 0, MSGW_EINVAL, "workspace must be 256-byte aligned");
        const Host& h = c->h;
        size_t tb = tables_bytes(h);
        need(bytes >= tb + scratch_needed(h, 1), MSGW_ENOMEM, "workspace smaller than msgw_workspace_size(nq_max=1)");
        MSGW_HIP(hipSetDevice(c->device));
        char* base = static_cast<char*>(dptr);
        size_t off = 0;
        auto put = [&](const void* src, size_t n) -> void* {
            void* p = base + off;
            if (n) MSGW_HIP(hipMemcpy(p, src, n, hipMemcpyHostToDevice));
            off += align_up(n);
            return p;
        };
        Dev d;
        d.nk = h.nk;
        d.ntau = h.ntau;
        d.niw_f = h.niw_f;
        d.niw_b = h.niw_b;
        d.nbmax = h.nbmax;
        d.nimax = h.nimax;
        d.beta = h.beta;
        d.scale = h.scale;
        d.tau = (const double*)put(h.tau.data(), sizeof(double) * h.ntau);
        d.wf = (const double2*)put(c->wf.data(), sizeof(double2) * c->wf.size());
        d.ef = (const double2*)put(c->ef.data(), sizeof(double2) * c->ef.size());
        d.wb = (const double2*)put(c->wb.data(), sizeof(double2) * c->wb.size());
        d.eb = (const double2*)put(c->eb.data(), sizeof(double2) * c->eb.size());
        d.kmq = (const int*)put(h.kmq.data(), sizeof(int) * h.kmq.size());
        d.nb = (const int*)put(h.nb.data(), sizeof(int) * h.nk);
        d.ni = (const int*)put(h.ni.data(), sizeof(int) * h.nk);
        d.moff = (const int64_t*)put(h.moff.data(), sizeof(int64_t) * h.moff.size());
        d.mpre = (const int64_t*)put(h.mpre.data(), sizeof(int64_t) * (h.nk + 1));
        d.ppre = (const int64_t*)put(h.ppre.data(), sizeof(int64_t) * (h.nk + 1));
        d.wpre = (const int64_t*)put(h.wpre.data(), sizeof(int64_t) * (h.nk + 1));
        d.vpre = (const int64_t*)put(h.vpre.data(), sizeof(int64_t) * (h.nk + 1));
        auto room = [&](size_t n) {
            void* p = base + off;
            off += align_up(n);
            return p;
        };
        d.sym_kmap = (int*)room(sizeof(int) * size_t(h.nk) * h.nk);
        d.sym_star = (int*)room(sizeof(int) * h.nk);
        d.sym_rk = (int*)room(sizeof(int) * size_t(kMaxRot) * h.nk);
        d.sym_rg = (int*)room(sizeof(int) * size_t(kMaxRot) * h.nimax);
        d.sym_g2 = (int*)room(sizeof(int) * h.nimax);
        need(off == tb, MSGW_EINVAL, "internal: table size mismatch");
        d.scratch = base + off;
        d.scratch_bytes = bytes - off;
        scratch_set_scales(d, h);
        d.kb0 = 0;
        d.kb1 = h.nk;
        c->d = d;
        c->ws = base;
        c->ws_bytes = bytes;
        c->ws_ready = true;
        c->sym_set = false;  // the tables live in the workspace
        c->cubic_ni = 0;
        c->prep = msgw_ctx::Prepared();
    });
}

int msgw_m_layout(const msgw_ctx* cc, int q, int64_t* off, int64_t* qsize) {
    msgw_ctx* c = const_cast<msgw_ctx*>(cc);
    return guarded(c, [&] {
        need(c->have_problem, MSGW_EINVAL, "no problem set");
        need(q >= 0 && q < c->h.nk, MSGW_EINVAL, "q out of range");
        need(qsize != nullptr, MSGW_EINVAL, "null qsize");
        if (off)
            for (int k = 0; k < c->h.nk; ++k) off[k] = c->h.moff[size_t(q) * c->h.nk + k];
        *qsize = c->h.mpre[q + 1] - c->h.mpre[q];
    });
}

int msgw_green0(msgw_ctx* c, void* stream, const double* eps, double mu, double* G_tau) {
    return guarded(c, [&] {
        require_ready(c);
        need(eps && G_tau, MSGW_EINVAL, "null pointer");
        need(std::isfinite(mu), MSGW_EINVAL, "mu must be finite");
        launch_green0(c->d, S(stream), eps, mu, G_tau);
    });
}

int msgw_synth_M(msgw_ctx* c, void* stream, uint64_t seed, int q0, int nq, int symmetric,
                 int m_dtype, void* M) {
    return guarded(c, [&] {
        require_ready(c);
        check_qrange(c, q0, nq);
        need(M != nullptr, MSGW_EINVAL, "null M");
        need(m_dtype == MSGW_C128 || m_dtype == MSGW_C64, MSGW_EINVAL, "bad m_dtype");
        launch_synth_M(c->d, c->h, S(stream), seed, q0, nq, symmetric, m_dtype, M);
    });
}

static bool full_k_range(const msgw_ctx* c) { return c->d.kb0 == 0 && c->d.kb1 == c->h.nk; }

// A call with reuse_prepared set must follow a call of the same op, q range, precision and variant
// (the polarization's g planes and the self-energy's weight blocks share the scratch); every other
// call that writes the scratch records itself (or clears the record).
static void check_reuse(msgw_ctx* c, int op, int q0, int nq, int precision) {
    const auto& p = c->prep;
    const int v = c->variant[op][precision];
    if (c->d.kreuse && precision != MSGW_FP64)  // the FP64 kernels prepare nothing
        need(p.op == op && p.q0 == q0 && p.nq == nq && p.precision == precision && p.variant == v, MSGW_EINVAL,
             "reuse_prepared: the scratch holds no operands of this op, q range, precision and variant");
}
static void record_prep(msgw_ctx* c, int op, int q0, int nq, int precision) {
    if (c->d.kreuse) return;
    if (precision == MSGW_FP64) {
        c->prep = msgw_ctx::Prepared();  // the FP64 kernels leave the scratch alone
        return;
    }
    c->prep.op = op;
    c->prep.q0 = q0;
    c->prep.nq = nq;
    c->prep.precision = precision;
    c->prep.variant = c->variant[op][precision];
}

int msgw_polarization(msgw_ctx* c, void* stream, int q0, int nq, const void* M, int m_dtype,
                      const double* G_tau, int precision, void* P_tau) {
    return guarded(c, [&] {
        require_ready(c);
        check_qrange(c, q0, nq);
        need(M && G_tau && P_tau, MSGW_EINVAL, "null pointer");
        need(full_k_range(c) || precision != MSGW_FP32, MSGW_ENOTSUP,
             "a partial k range is supported by the FP64 and the split-precision pair-space kernels only");
        check_reuse(c, MSGW_OP_POLARIZATION, q0, nq, precision);
        if (precision == MSGW_FP64) {
            need(m_dtype == MSGW_C128, MSGW_EINVAL, "MSGW_FP64 needs MSGW_C128 M");
            launch_pol_fp64(c->d, c->h, S(stream), q0, nq, M, G_tau, P_tau);
        } else if (precision == MSGW_FP32 || precision == MSGW_BF16X3 || precision == MSGW_F16X3) {
            need(m_dtype == MSGW_C64, MSGW_EINVAL, "MSGW_FP32 / MSGW_BF16X3 / MSGW_F16X3 need MSGW_C64 M");
            int rc = launch_pol_mfma(c->d, c->h, S(stream), q0, nq, M, G_tau, precision,
                                     c->variant[MSGW_OP_POLARIZATION][precision], P_tau);
            need(rc == MSGW_OK, rc, "polarization: unsupported shape for the MFMA path");
            record_prep(c, MSGW_OP_POLARIZATION, q0, nq, precision);
        } else {
            throw Error(MSGW_EINVAL, "bad precision");
        }
    });
}

int msgw_tau_to_iw(msgw_ctx* c, void* stream, int stat, int64_t nblk, int64_t len,
                   const void* f_tau, int f_is_complex, const double* e_ref, void* f_iw) {
    return guarded(c, [&] {
        require_ready(c);
        need(stat == MSGW_FERMION || stat == MSGW_BOSON, MSGW_EINVAL, "bad stat");
        need(nblk >= 0 && len >= 0, MSGW_EINVAL, "negative size");
        need(f_tau && f_iw, MSGW_EINVAL, "null pointer");
        need(!(e_ref && stat == MSGW_BOSON), MSGW_EINVAL, "e_ref is for FERMION data");
        if (nblk == 0 || len == 0) return;
        launch_fwd(c->d, S(stream), stat, nblk, len, f_tau, f_is_complex, e_ref, f_iw);
    });
}

int msgw_iw_to_tau(msgw_ctx* c, void* stream, int stat, int64_t nblk, int64_t len, int mat_n,
                   const void* f_iw, const void* add_tau, const double* e_ref, void* f_tau) {
    return guarded(c, [&] {
        require_ready(c);
        need(f_iw && f_tau, MSGW_EINVAL, "null pointer");
        need(nblk >= 0 && len >= 0, MSGW_EINVAL, "negative size");
        if (stat == MSGW_FERMION) {
            need(mat_n == 0, MSGW_EINVAL, "FERMION inverse transform is scalar (mat_n = 0)");
            need(add_tau == nullptr, MSGW_EINVAL, "add_tau is for BOSON matrices");
            if (nblk == 0 || len == 0) return;
            launch_inv_fermion(c->d, S(stream), nblk, len, f_iw, e_ref, (double*)f_tau);
        } else if (stat == MSGW_BOSON) {
            need(mat_n > 0 && int64_t(mat_n) * mat_n == len, MSGW_ESHAPE, "BOSON needs len == mat_n^2");
            need(e_ref == nullptr, MSGW_EINVAL, "e_ref is for FERMION data");
            if (nblk == 0) return;
            launch_inv_boson(c->d, S(stream), nblk, mat_n, f_iw, add_tau, nullptr, f_tau);
        } else {
            throw Error(MSGW_EINVAL, "bad stat");
        }
    });
}

int msgw_screen(msgw_ctx* c, void* stream, int q0, int nq, const void* P_iw, const double* v,
                void* Wt_iw, void* R_iw, int* info, int* flags) {
    return guarded(c, [&] {
        require_ready(c);
        check_qrange(c, q0, nq);
        need(P_iw && v && Wt_iw && info, MSGW_EINVAL, "null pointer");
        need(P_iw != Wt_iw, MSGW_EINVAL, "P_iw and Wt_iw must not alias");
        screen_validate(c->h, q0, nq);
        need(screen_scratch_bytes(c->h, nq) <= scratch_mfma_bytes(c->d, c->h), MSGW_ENOMEM,
             "screen: workspace too small for nq (size it with msgw_workspace_size(nq_max >= nq))");
        c->prep = msgw_ctx::Prepared();  // the pivot record uses the split-precision scratch
        launch_screen(c->d, c->h, S(stream), q0, nq, P_iw, v, Wt_iw, R_iw, info, flags,
                      reinterpret_cast<int*>(scratch_mfma(c->d, c->h)));
    });
}

int msgw_screened_tau(msgw_ctx* c, void* stream, int q0, int nq, const void* R_iw,
                      const void* P_tau, const double* v, void* Wt_tau) {
    return guarded(c, [&] {
        require_ready(c);
        check_qrange(c, q0, nq);
        need(R_iw && P_tau && v && Wt_tau, MSGW_EINVAL, "null pointer");
        const Host& h = c->h;
        for (int q = q0; q < q0 + nq; ++q) {
            int n = h.ni[q];
            const char* R = (const char*)R_iw + sizeof(double2) * (h.wpre[q] - h.wpre[q0]);
            const char* P = (const char*)P_tau + sizeof(double2) * (h.ppre[q] - h.ppre[q0]);
            char* W = (char*)Wt_tau + sizeof(double2) * (h.ppre[q] - h.ppre[q0]);
            const double* vq = v + (h.vpre[q] - h.vpre[q0]);
            launch_inv_boson(c->d, S(stream), 1, n, R, P, vq, W);
        }
    });
}

int msgw_self_energy(msgw_ctx* c, void* stream, int q0, int nq, const void* M, int m_dtype,
                     const double* G_tau, const void* Wt_tau, int precision, void* Sigma_tau) {
    return guarded(c, [&] {
        require_ready(c);
        check_qrange(c, q0, nq);
        need(M && G_tau && Wt_tau && Sigma_tau, MSGW_EINVAL, "null pointer");
        need(full_k_range(c) || (precision != MSGW_FP32 && c->h.sigma_mode != MSGW_SIGMA_FULL), MSGW_ENOTSUP,
             "a partial k range is supported by the FP64 (DIAG) and the split-precision pair-space kernels only");
        check_reuse(c, MSGW_OP_SELF_ENERGY, q0, nq, precision);
        if (c->h.sigma_mode == MSGW_SIGMA_FULL) {
            if (precision == MSGW_FP64) {
                need(m_dtype == MSGW_C128, MSGW_EINVAL, "MSGW_FP64 needs MSGW_C128 M");
                launch_sig_full_fp64(c->d, c->h, S(stream), q0, nq, M, G_tau, Wt_tau, Sigma_tau);
                return;
            }
            need(precision == MSGW_F16X3 && m_dtype == MSGW_C64, MSGW_ENOTSUP,
                 "MSGW_SIGMA_FULL runs in MSGW_FP64 (MSGW_C128 M) or MSGW_F16X3 (MSGW_C64 M)");
            launch_sig_full_split(c->d, c->h, S(stream), q0, nq, M, G_tau, Wt_tau, Sigma_tau,
                                  scratch_mfma(c->d, c->h), scratch_mfma_bytes(c->d, c->h));
            c->prep = msgw_ctx::Prepared();  // the scratch no longer holds prepared operands
            return;
        }
        if (precision == MSGW_FP64) {
            need(m_dtype == MSGW_C128, MSGW_EINVAL, "MSGW_FP64 needs MSGW_C128 M");
            launch_sig_fp64(c->d, c->h, S(stream), q0, nq, M, G_tau, Wt_tau, Sigma_tau);
        } else if (precision == MSGW_FP32 || precision == MSGW_BF16X3 || precision == MSGW_F16X3) {
            need(m_dtype == MSGW_C64, MSGW_EINVAL, "MSGW_FP32 / MSGW_BF16X3 / MSGW_F16X3 need MSGW_C64 M");
            int rc = launch_sig_mfma(c->d, c->h, S(stream), q0, nq, M, G_tau, Wt_tau, precision,
                                     c->variant[MSGW_OP_SELF_ENERGY][precision], Sigma_tau);
            need(rc == MSGW_OK, rc, "self_energy: workspace too small or unsupported shape for the MFMA path");
            record_prep(c, MSGW_OP_SELF_ENERGY, q0, nq, precision);
        } else {
            throw Error(MSGW_EINVAL, "bad precision");
        }
    });
}

int msgw_sigma_x(msgw_ctx* c, void* stream, int q0, int nq, const void* M, int m_dtype,
                 const double* G_tau, const double* v, void* Sigma_x) {
    return guarded(c, [&] {
        require_ready(c);
        check_qrange(c, q0, nq);
        need(M && G_tau && v && Sigma_x, MSGW_EINVAL, "null pointer");
        need(m_dtype == MSGW_C128 || m_dtype == MSGW_C64, MSGW_EINVAL, "bad m_dtype");
        launch_sigma_x(c->d, c->h, S(stream), q0, nq, M, m_dtype, G_tau, v, Sigma_x,
                       c->h.sigma_mode == MSGW_SIGMA_FULL);
    });
}

int msgw_dyson(msgw_ctx* c, void* stream, const double* eps, const double* sigma_static,
               const void* Sigma_c_iw, double n_target, int mu_mode, double* mu, void* G_iw,
               double* G_tau, double* n_out, int* flags) {
    return guarded(c, [&] {
        require_ready(c);
        need(eps && sigma_static && Sigma_c_iw && mu && G_tau && n_out && flags, MSGW_EINVAL,
             "null pointer");
        need(mu_mode == MSGW_MU_FIXED || mu_mode == MSGW_MU_SEARCH, MSGW_EINVAL, "bad mu_mode");
        need(std::isfinite(n_target) && n_target >= 0, MSGW_EINVAL, "bad n_target");
        launch_dyson(c->d, c->h, S(stream), eps, sigma_static, Sigma_c_iw, n_target,
                     mu_mode == MSGW_MU_SEARCH, mu, G_iw, G_tau, n_out, flags, scratch_E(c->d),
                     scratch_mu_search(c->d, c->h));
    });
}

int msgw_dyson_matrix(msgw_ctx* c, void* stream, const double* eps, const void* sigma_static,
                      const void* Sigma_c_iw, double n_target, int mu_mode, double* mu, void* G_iw,
                      void* G_tau, double* n_out, int* flags) {
    return guarded(c, [&] {
        require_ready(c);
        need(eps && sigma_static && Sigma_c_iw && mu && G_iw && G_tau && n_out && flags, MSGW_EINVAL,
             "null pointer");
        need(mu_mode == MSGW_MU_FIXED || mu_mode == MSGW_MU_SEARCH, MSGW_EINVAL, "bad mu_mode");
        need(std::isfinite(n_target) && n_target >= 0, MSGW_EINVAL, "bad n_target");
        need(c->h.nbmax <= 64, MSGW_ENOTSUP, "msgw_dyson_matrix: at most 64 bands (one matrix in LDS)");
        need(int64_t(c->h.nk) <= 65535 && c->h.niw_f <= 65535, MSGW_ENOTSUP, "msgw_dyson_matrix: grid limits");
        need(mdyson_scratch_bytes(c->h) <= scratch_mfma_bytes(c->d, c->h), MSGW_ENOMEM,
             "msgw_dyson_matrix: workspace too small");
        c->prep = msgw_ctx::Prepared();  // uses the split-precision scratch
        launch_dyson_matrix(c->d, c->h, S(stream), eps, (const double2*)sigma_static, (const double2*)Sigma_c_iw,
                            n_target, mu_mode == MSGW_MU_SEARCH, mu, (double2*)G_iw, (double2*)G_tau, n_out,
                            flags, reinterpret_cast<double*>(scratch_mfma(c->d, c->h)));
    });
}

int msgw_dyson_noalloc(msgw_ctx* c, void* stream, const double* eps, const double* sigma_static,
                       const void* Sigma_c_iw, double n_target, int mu_mode, double* mu, void* G_iw,
                       double* G_tau, double* n_out, int* flags) {
    return guarded(c, [&] {
        need(c->have_problem, MSGW_EINVAL, "no problem set (msgw_set_problem)");
        const size_t eb = align_up(sizeof(double) * size_t(c->h.nk) * c->h.nbmax);
        if (eb + kMuSearchBytes > kNoAllocScratchBytes) {
            std::ostringstream m;
            m << "msgw_dyson_noalloc: nk * nbmax = " << size_t(c->h.nk) * c->h.nbmax
              << " states exceed its static scratch (at most "
              << (kNoAllocScratchBytes - kMuSearchBytes) / sizeof(double) << " states); use msgw_dyson";
            throw Error(MSGW_ENOTSUP, m.str());
        }
        require_ready(c);
        need(eps && sigma_static && Sigma_c_iw && mu && G_tau && n_out && flags, MSGW_EINVAL,
             "null pointer");
        need(mu_mode == MSGW_MU_FIXED || mu_mode == MSGW_MU_SEARCH, MSGW_EINVAL, "bad mu_mode");
        need(std::isfinite(n_target) && n_target >= 0, MSGW_EINVAL, "bad n_target");
        need(c->noalloc != nullptr, MSGW_EHIP, "static scratch address unknown");
        char* base = static_cast<char*>(c->noalloc);
        launch_dyson(c->d, c->h, S(stream), eps, sigma_static, Sigma_c_iw, n_target,
                     mu_mode == MSGW_MU_SEARCH, mu, G_iw, G_tau, n_out, flags, reinterpret_cast<double*>(base),
                     reinterpret_cast<double*>(base + eb));
    });
}

int msgw_set_tau_mirror(msgw_ctx* c, int on) {
    return guarded(c, [&] {
        require_ready(c);
        c->d.tau_mirror = on ? 1 : 0;
    });
}

int msgw_continue_pade(msgw_ctx* c, void* stream, int n_pade, double eta, const double* eps,
                       const double* sigma_static, const void* Sigma_c_iw, const double* mu, int n_omega,
                       const double* omega, double* A, double* E_qp, int* flags) {
    return guarded(c, [&] {
        require_ready(c);
        need(eps && sigma_static && Sigma_c_iw && mu && E_qp && flags, MSGW_EINVAL, "null pointer");
        need(n_pade >= 1 && n_pade <= c->h.niw_f && n_pade <= 128, MSGW_EINVAL,
             "n_pade outside [1, min(niw_f, 128)]");
        need(std::isfinite(eta) && eta >= 0.0, MSGW_EINVAL, "eta must be finite and >= 0");
        need(n_omega >= 0, MSGW_EINVAL, "negative n_omega");
        need(n_omega == 0 || (omega && A), MSGW_EINVAL, "n_omega > 0 needs omega and A");
        launch_pade(c->d, c->h, S(stream), n_pade, eta, eps, sigma_static, Sigma_c_iw, mu, n_omega,
                    n_omega ? omega : nullptr, n_omega ? A : nullptr, E_qp, flags);
    });
}

int msgw_continue_cpe(msgw_ctx* c, void* stream, int n_real, double w_min, double w_max, double ridge, double eta,
                      const double* eps, const double* sigma_static, const void* Sigma_c_iw, const double* mu,
                      int n_omega, const double* omega, double* A, double* E_qp, double* coef, int* flags) {
    return guarded(c, [&] {
        require_ready(c);
        need(eps && sigma_static && Sigma_c_iw && mu && E_qp && flags, MSGW_EINVAL, "null pointer");
        need(n_real >= 4 && n_real <= 98, MSGW_EINVAL, "n_real outside [4, 98]");
        need(std::isfinite(w_min) && std::isfinite(w_max) && w_min < w_max, MSGW_EINVAL, "need w_min < w_max");
        need(std::isfinite(ridge) && ridge >= 0.0, MSGW_EINVAL, "ridge must be finite and >= 0");
        need(std::isfinite(eta) && eta > 0.0, MSGW_EINVAL, "eta must be finite and > 0");
        need(n_omega >= 0, MSGW_EINVAL, "negative n_omega");
        need(n_omega == 0 || (omega && A), MSGW_EINVAL, "n_omega > 0 needs omega and A");
        launch_cpe(c->d, c->h, S(stream), n_real, w_min, w_max, ridge, eta, eps, sigma_static, Sigma_c_iw, mu,
                   n_omega, n_omega ? omega : nullptr, n_omega ? A : nullptr, E_qp, coef, flags);
        c->prep = msgw_ctx::Prepared();  // its design matrix overwrites the split-precision scratch
    });
}

int msgw_gap_of(msgw_ctx* c, void* stream, const double* E, int n_index, double* gap) {
    return guarded(c, [&] {
        require_ready(c);
        need(E && gap, MSGW_EINVAL, "null pointer");
        int64_t nstate = 0;
        for (int k = 0; k < c->h.nk; ++k) nstate += c->h.nb[k];
        need(n_index >= 1 && n_index < nstate, MSGW_EINVAL, "n_index outside [1, number of states)");
        launch_gap_given(c->d, c->h, S(stream), E, n_index, gap);
    });
}

int msgw_variant_count(int op, int precision) {
    if (op != MSGW_OP_POLARIZATION && op != MSGW_OP_SELF_ENERGY) return MSGW_EINVAL;
    if (precision != MSGW_FP32 && precision != MSGW_BF16X3 && precision != MSGW_F16X3) return MSGW_EINVAL;
    return mfma_variant_count(op, precision);
}

const char* msgw_variant_name(int op, int precision, int variant) {
    return mfma_variant_name(op, precision, variant);
}

int msgw_set_variant(msgw_ctx* c, int op, int precision, int variant) {
    return guarded(c, [&] {
        int n = msgw_variant_count(op, precision);
        need(n > 0, MSGW_EINVAL, "bad op or precision");
        need(variant >= 0 && variant < n, MSGW_EINVAL, "variant out of range");
        c->variant[op][precision] = variant;
    });
}

int msgw_set_k_range(msgw_ctx* c, int k0, int k1, int reuse_prepared) {
    return guarded(c, [&] {
        require_ready(c);
        if (k1 <= 0) {
            k0 = 0;
            k1 = c->h.nk;
            reuse_prepared = 0;
        }
        need(k0 >= 0 && k0 < k1 && k1 <= c->h.nk, MSGW_EINVAL, "k range outside [0, nk]");
        c->d.kb0 = k0;
        c->d.kb1 = k1;
        c->d.kreuse = reuse_prepared ? 1 : 0;
    });
}

int msgw_set_kernel_events(msgw_ctx* c, int op, void* start, void* stop) {
    return guarded(c, [&] {
        require_ready(c);
        need(op == MSGW_OP_POLARIZATION || op == MSGW_OP_SELF_ENERGY, MSGW_EINVAL, "bad op");
        need((start == nullptr) == (stop == nullptr), MSGW_EINVAL, "give both events or neither");
        c->d.ev_start[op] = static_cast<hipEvent_t>(start);
        c->d.ev_stop[op] = static_cast<hipEvent_t>(stop);
    });
}

int msgw_get_variant(const msgw_ctx* c, int op, int precision, int* variant) {
    if (!c || !variant) return MSGW_EINVAL;
    if (msgw_variant_count(op, precision) <= 0) return MSGW_EINVAL;
    *variant = c->variant[op][precision];
    return MSGW_OK;
}

int msgw_gap(msgw_ctx* c, void* stream, const double* eps, const double* sigma_static,
             const void* Sigma_c_iw, const double* mu, int n_index, double* gap) {
    return guarded(c, [&] {
        require_ready(c);
        need(eps && sigma_static && Sigma_c_iw && mu && gap, MSGW_EINVAL, "null pointer");
        int64_t nstate = 0;
        for (int k = 0; k < c->h.nk; ++k) nstate += c->h.nb[k];
        need(n_index >= 1 && n_index < nstate, MSGW_EINVAL, "n_index outside [1, number of states)");
        launch_gap(c->d, c->h, S(stream), eps, sigma_static, Sigma_c_iw, mu, n_index, gap);
    });
}

int msgw_tau_solver_work_size(msgw_ctx* c, int which, int first, int count, size_t* bytes) {
    return guarded(c, [&] {
        need(c->have_problem, MSGW_EINVAL, "no problem set");
        need(bytes != nullptr, MSGW_EINVAL, "null bytes");
        need(which == MSGW_TS_WTILDE || which == MSGW_TS_DYSON, MSGW_EINVAL, "bad solver");
        need(first >= 0 && count >= 1 && first + count <= c->h.nk, MSGW_EINVAL, "range outside [0, nk)");
        *bytes = tau_sys_layout(c->h, which, first, count).total;
    });
}

static void upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes) MSGW_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
}

int msgw_wt_tau_system(msgw_ctx* c, void* stream, int q0, int nq, const void* P_tau, const double* v,
                       void* Wt_tau, int* info, void* work, size_t work_bytes) {
    return guarded(c, [&] {
        require_ready(c);
        check_qrange(c, q0, nq);
        need(P_tau && v && Wt_tau && info && work, MSGW_EINVAL, "null pointer");
        need((reinterpret_cast<uintptr_t>(work) & 255) == 0, MSGW_EINVAL, "work must be 256-byte aligned");
        const Host& h = c->h;
        const TauSysLayout L = tau_sys_layout(h, MSGW_TS_WTILDE, q0, nq);
        need(work_bytes >= L.total, MSGW_ENOMEM, "work smaller than msgw_tau_solver_work_size");
        const int nt = h.ntau;
        // spline weights of P at tau_p - tau_r (+ beta below zero) and the trapezoid increments
        const std::vector<double> X = spline_second_derivs(h.tau);
        std::vector<double> phi(size_t(nt) * nt * nt);
        for (int p = 0; p < nt; ++p)
            for (int r = 0; r < nt; ++r) {
                double x = h.tau[p] - h.tau[r];
                if (x < 0.0) x += h.beta;
                spline_eval_weights(h.tau, X, x, &phi[(size_t(p) * nt + r) * nt]);
            }
        const std::vector<double> dt = trapezoid_increments(h.tau);
        char* w = static_cast<char*>(work);
        hipStream_t st = S(stream);
        upload(w + L.phi, phi.data(), sizeof(double) * phi.size(), st);
        upload(w + L.dt, dt.data(), sizeof(double) * nt, st);
        upload(w + L.tn, L.tn_h.data(), sizeof(int) * L.count, st);
        upload(w + L.tld, L.tld_h.data(), sizeof(int) * L.count, st);
        upload(w + L.koff, L.koff_h.data(), sizeof(int64_t) * L.count, st);
        TauSysArgs a;
        a.ntau = nt;
        a.nbmax = h.nbmax;
        a.q0 = q0;
        a.beta = h.beta;
        a.ni = c->d.ni;
        a.ppre = c->d.ppre;
        a.vpre = c->d.vpre;
        a.phi = reinterpret_cast<const double*>(w + L.phi);
        a.dt = reinterpret_cast<const double*>(w + L.dt);
        a.tn = reinterpret_cast<const int*>(w + L.tn);
        a.tld = reinterpret_cast<const int*>(w + L.tld);
        a.koff = reinterpret_cast<const int64_t*>(w + L.koff);
        a.perm = reinterpret_cast<int*>(w + L.perm);
        a.ginfo = info;
        a.K = reinterpret_cast<double2*>(w + L.K);
        launch_wt_tau_system(a, st, nq, L.nmax, L.ldmax, P_tau, v, Wt_tau);
        MSGW_HIP(hipStreamSynchronize(st));  // the host tables above are released on return
    });
}

int msgw_dyson_tau(msgw_ctx* c, void* stream, int k0, int nkc, const double* eps, const double* sigma_static,
                   const double* mu, const double* Sigma_c_tau, double* G_tau, int* info, void* work,
                   size_t work_bytes) {
    return guarded(c, [&] {
        require_ready(c);
        need(k0 >= 0 && nkc >= 1 && k0 + nkc <= c->h.nk, MSGW_EINVAL, "k range outside [0, nk)");
        need(eps && sigma_static && mu && Sigma_c_tau && G_tau && info && work, MSGW_EINVAL, "null pointer");
        need((reinterpret_cast<uintptr_t>(work) & 255) == 0, MSGW_EINVAL, "work must be 256-byte aligned");
        const Host& h = c->h;
        const TauSysLayout L = tau_sys_layout(h, MSGW_TS_DYSON, k0, nkc);
        need(work_bytes >= L.total, MSGW_ENOMEM, "work smaller than msgw_tau_solver_work_size");
        const int nt = h.ntau, nd = L.nd;
        std::vector<int> idx;
        dense_grid(h, &idx);
        const double step = h.tau[1] - h.tau[0];
        std::vector<double> td(nd);
        for (int a = 0; a < nd; ++a) td[a] = a * step;
        td[nd - 1] = h.beta;
        for (int i = 0; i < nt; ++i) td[idx[i]] = h.tau[i];  // the mesh's own values at its nodes
        const std::vector<double> dtd = trapezoid_increments(td);
        const std::vector<double> X = spline_second_derivs(h.tau);
        std::vector<double> psi(size_t(nd) * nt);
        for (int a = 0; a < nd; ++a) spline_eval_weights(h.tau, X, td[a], &psi[size_t(a) * nt]);
        char* w = static_cast<char*>(work);
        hipStream_t st = S(stream);
        upload(w + L.psi, psi.data(), sizeof(double) * psi.size(), st);
        upload(w + L.td, td.data(), sizeof(double) * nd, st);
        upload(w + L.dtd, dtd.data(), sizeof(double) * nd, st);
        upload(w + L.idx, idx.data(), sizeof(int) * nt, st);
        upload(w + L.st_k, L.st_k_h.data(), sizeof(int) * L.count, st);
        upload(w + L.st_n, L.st_n_h.data(), sizeof(int) * L.count, st);
        upload(w + L.tn, L.tn_h.data(), sizeof(int) * L.count, st);
        upload(w + L.tld, L.tld_h.data(), sizeof(int) * L.count, st);
        upload(w + L.koff, L.koff_h.data(), sizeof(int64_t) * L.count, st);
        TauSysArgs a;
        a.ntau = nt;
        a.nbmax = h.nbmax;
        a.nd = nd;
        a.k0 = k0;
        a.beta = h.beta;
        a.psi = reinterpret_cast<const double*>(w + L.psi);
        a.td = reinterpret_cast<const double*>(w + L.td);
        a.dtd = reinterpret_cast<const double*>(w + L.dtd);
        a.idx = reinterpret_cast<const int*>(w + L.idx);
        a.st_k = reinterpret_cast<const int*>(w + L.st_k);
        a.st_n = reinterpret_cast<const int*>(w + L.st_n);
        a.gpos = reinterpret_cast<double*>(w + L.gpos);
        a.scd = reinterpret_cast<double*>(w + L.scd);
        a.tn = reinterpret_cast<const int*>(w + L.tn);
        a.tld = reinterpret_cast<const int*>(w + L.tld);
        a.koff = reinterpret_cast<const int64_t*>(w + L.koff);
        a.perm = reinterpret_cast<int*>(w + L.perm);
        a.ginfo = reinterpret_cast<int*>(w + L.ginfo);
        a.K = reinterpret_cast<double2*>(w + L.K);
        launch_dyson_tau(a, st, L.count, nkc, eps, sigma_static, mu, Sigma_c_tau, G_tau, info);
        MSGW_HIP(hipStreamSynchronize(st));  // the host tables above are released on return
    });
}

int msgw_set_symmetry(msgw_ctx* c, int nrot, const int* rot_k) {
    return guarded(c, [&] {
        require_ready(c);
        const Host& h = c->h;
        const int nk = h.nk;
        need(rot_k != nullptr, MSGW_EINVAL, "null rot_k");
        need(nrot >= 1 && nrot <= kMaxRot, MSGW_EINVAL, "nrot outside [1, 48]");
        // every row a permutation of the grid that commutes with k - q
        for (int r = 0; r < nrot; ++r) {
            std::vector<char> hit(nk, 0);
            for (int k = 0; k < nk; ++k) {
                const int x = rot_k[size_t(r) * nk + k];
                need(x >= 0 && x < nk && !hit[x], MSGW_EINVAL, "rot_k: a row is not a permutation of the k grid");
                hit[x] = 1;
            }
            for (int q = 0; q < nk; ++q)
                for (int k = 0; k < nk; ++k) {
                    const int* R = rot_k + size_t(r) * nk;
                    need(h.kmq[size_t(R[q]) * nk + R[k]] == R[h.kmq[size_t(q) * nk + k]], MSGW_EINVAL,
                         "rot_k: R (k - q) != R k - R q");
                }
        }
        // stars: each orbit represented by its smallest q, members with the first operation reaching them
        std::vector<int> ibz, off(1, 0), star, rep_of(nk, -1), op_of(nk, -1);
        for (int q = 0; q < nk; ++q) {
            if (rep_of[q] >= 0) continue;
            ibz.push_back(q);
            for (int r = 0; r < nrot; ++r) {
                const int qp = rot_k[size_t(r) * nk + q];
                if (rep_of[qp] >= 0) continue;
                rep_of[qp] = q;
                op_of[qp] = r;
                star.push_back(qp);
            }
            off.push_back((int)star.size());
        }
        need((int)star.size() == nk, MSGW_EINVAL, "rot_k: the operations do not close into orbits");
        // kmap[q'][k] = R^-1 k for the operation R that maps the representative of q' onto q'
        std::vector<int> kmap(size_t(nk) * nk);
        for (int qp = 0; qp < nk; ++qp) {
            const int* R = rot_k + size_t(op_of[qp]) * nk;
            for (int k = 0; k < nk; ++k) kmap[size_t(qp) * nk + R[k]] = k;
        }
        MSGW_HIP(hipMemcpy(c->d.sym_kmap, kmap.data(), sizeof(int) * kmap.size(), hipMemcpyHostToDevice));
        MSGW_HIP(hipMemcpy(c->d.sym_star, star.data(), sizeof(int) * nk, hipMemcpyHostToDevice));
        c->sym_ibz = ibz;
        c->sym_off = off;
        c->sym_star = star;
        c->sym_rep_of = rep_of;
        c->sym_set = true;
    });
}

int msgw_ibz(const msgw_ctx* cc, int* n_ibz, int* q_ibz, int* star_size) {
    msgw_ctx* c = const_cast<msgw_ctx*>(cc);
    return guarded(c, [&] {
        need(c->sym_set, MSGW_EINVAL, "no symmetry set (msgw_set_symmetry)");
        need(n_ibz != nullptr, MSGW_EINVAL, "null n_ibz");
        *n_ibz = (int)c->sym_ibz.size();
        for (size_t i = 0; i < c->sym_ibz.size(); ++i) {
            if (q_ibz) q_ibz[i] = c->sym_ibz[i];
            if (star_size) star_size[i] = c->sym_off[i + 1] - c->sym_off[i];
        }
    });
}

int msgw_sigma_star(msgw_ctx* c, void* stream, int q_ibz, const double* C_tau, const double* C_x, double* Sigma_tau,
                    double* Sigma_x) {
    return guarded(c, [&] {
        require_ready(c);
        need(c->sym_set, MSGW_EINVAL, "no symmetry set (msgw_set_symmetry)");
        need(c->h.sigma_mode == MSGW_SIGMA_DIAG, MSGW_ENOTSUP, "msgw_sigma_star: MSGW_SIGMA_DIAG only");
        need(C_tau && Sigma_tau, MSGW_EINVAL, "null pointer");
        need((C_x == nullptr) == (Sigma_x == nullptr), MSGW_EINVAL, "give both C_x and Sigma_x or neither");
        const auto it = std::find(c->sym_ibz.begin(), c->sym_ibz.end(), q_ibz);
        need(it != c->sym_ibz.end(), MSGW_EINVAL, "q_ibz is not an irreducible q");
        const int i = int(it - c->sym_ibz.begin());
        launch_sigma_star(c->d, c->h, S(stream), c->d.sym_kmap, c->d.sym_star, c->sym_off[i], c->sym_off[i + 1], C_tau,
                          C_x, Sigma_tau, Sigma_x);
    });
}

int msgw_synth_M_cubic(msgw_ctx* c, void* stream, uint64_t seed, int q0, int nq, int m_dtype, void* M) {
    return guarded(c, [&] {
        require_ready(c);
        check_qrange(c, q0, nq);
        need(M != nullptr, MSGW_EINVAL, "null M");
        need(m_dtype == MSGW_C128 || m_dtype == MSGW_C64, MSGW_EINVAL, "bad m_dtype");
        const Host& h = c->h;
        int n = 1;
        while (n * n * n < h.nk) ++n;
        need(n * n * n == h.nk, MSGW_ESHAPE, "the cubic generator needs an n x n x n grid (k = (i1 n + i2) n + i3)");
        for (int k = 0; k < h.nk; ++k) need(h.nb[k] == h.nb[0], MSGW_ESHAPE, "the cubic generator needs one band count");
        for (int q = 0; q < h.nk; ++q) need(h.ni[q] == h.ni[0], MSGW_ESHAPE, "the cubic generator needs one NI");
        const int ni = h.ni[0];
        const auto g = shell_basis(ni);
        need(!g.empty(), MSGW_ESHAPE, "NI does not close a shell of reciprocal-lattice vectors");
        if (c->cubic_ni == ni) {  // tables already in the workspace
            launch_synth_cubic(c->d, h, S(stream), seed, q0, nq, m_dtype, M, c->d.sym_rk, c->d.sym_rg, c->d.sym_g2);
            return;
        }
        const auto ops = cubic_ops();
        std::map<std::array<int, 3>, int> index;
        for (int i = 0; i < ni; ++i) index[g[i]] = i;
        std::vector<int> rk(size_t(kMaxRot) * h.nk), rg(size_t(kMaxRot) * ni), g2(ni);
        for (int r = 0; r < kMaxRot; ++r) {
            const IMat& R = ops[r];
            for (int k = 0; k < h.nk; ++k) {
                const int ik[3] = {k / (n * n), (k / n) % n, k % n};
                int x[3];
                for (int a = 0; a < 3; ++a) {
                    x[a] = 0;
                    for (int b = 0; b < 3; ++b) x[a] += R.m[a][b] * ik[b];
                    x[a] = ((x[a] % n) + n) % n;
                }
                rk[size_t(r) * h.nk + k] = (x[0] * n + x[1]) * n + x[2];
            }
            for (int i = 0; i < ni; ++i) {
                std::array<int, 3> y{};
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) y[a] += R.m[a][b] * g[i][b];
                rg[size_t(r) * ni + i] = index.at(y);
            }
        }
        for (int i = 0; i < ni; ++i) g2[i] = g[i][0] * g[i][0] + g[i][1] * g[i][1] + g[i][2] * g[i][2];
        MSGW_HIP(hipMemcpy(c->d.sym_rk, rk.data(), sizeof(int) * rk.size(), hipMemcpyHostToDevice));
        MSGW_HIP(hipMemcpy(c->d.sym_rg, rg.data(), sizeof(int) * rg.size(), hipMemcpyHostToDevice));
        MSGW_HIP(hipMemcpy(c->d.sym_g2, g2.data(), sizeof(int) * g2.size(), hipMemcpyHostToDevice));
        c->cubic_ni = ni;
        launch_synth_cubic(c->d, h, S(stream), seed, q0, nq, m_dtype, M, c->d.sym_rk, c->d.sym_rg, c->d.sym_g2);
    });
}

}  // extern "C"
