// G0, synthetic M, tau <-> i omega transforms, exchange self-energy, Dyson + chemical potential.
// All arithmetic here is FP64.
#include <mutex>

#include "internal.h"

// Scratch of msgw_dyson_noalloc (the E array and the mu search state) in a static device array, so
// that the call allocates nothing.  Each device the library runs on holds its own copy until the
// process ends; host code uses only the device address looked up per device by noalloc_scratch().
static __device__ __align__(256) char scratch[msgw::kNoAllocScratchBytes];

namespace msgw {

namespace {
std::mutex g_noalloc_mu;
std::vector<void*> g_noalloc_ptr;  // per device: the address of `scratch` there
}  // namespace

void* noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (int(g_noalloc_ptr.size()) <= device) g_noalloc_ptr.resize(device + 1, nullptr);
    if (!g_noalloc_ptr[device]) {
        int cur = 0;
        MSGW_HIP(hipGetDevice(&cur));
        MSGW_HIP(hipSetDevice(device));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        MSGW_HIP(hipSetDevice(cur));
        if (e != hipSuccess || p == nullptr)
            throw Error(MSGW_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_noalloc_ptr[device] = p;
    }
    return g_noalloc_ptr[device];
}

namespace {

constexpr double kPi = 3.14159265358979323846;

inline unsigned ceil_div(int64_t a, int64_t b) {
    const int64_t r = (a + b - 1) / b;
    if (r > int64_t(0xFFFFFFFFu)) throw Error(MSGW_ENOTSUP, "shape too large for one launch");
    return unsigned(r);
}

__device__ __forceinline__ double2 ld_c(const void* p, int64_t i, bool c64) {
    if (c64) {
        float2 f = reinterpret_cast<const float2*>(p)[i];
        return make_double2(f.x, f.y);
    }
    return reinterpret_cast<const double2*>(p)[i];
}

// 1 / (i w - E)
__device__ __forceinline__ double2 inv_iw_minus(double w, double E) {
    double den = E * E + w * w;
    return make_double2(-E / den, -w / den);
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    // a / b, scaled to avoid overflow for large |b|
    double s = fmax(fabs(b.x), fabs(b.y));
    double bx = b.x / s, by = b.y / s;
    double den = bx * bx + by * by;
    return make_double2((a.x * bx + a.y * by) / (den * s), (a.y * bx - a.x * by) / (den * s));
}

__device__ __forceinline__ double fermi(double E, double beta) {
    double x = beta * E;
    double ex = exp(-fabs(x));
    return x >= 0.0 ? ex / (1.0 + ex) : 1.0 / (1.0 + ex);
}

// ---------------------------------------------------------------------------------------------
// a1: G0
// ---------------------------------------------------------------------------------------------
__global__ void k_green0(const double* __restrict__ eps, double mu, const int* __restrict__ nb,
                         const double* __restrict__ tau, int nk, int nbmax, int ntau, double beta,
                         double* __restrict__ G) {
    int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t tot = int64_t(nk) * nbmax * ntau;
    if (e >= tot) return;
    int i = int(e % ntau);
    int64_t kn = e / ntau;
    int n = int(kn % nbmax), k = int(kn / nbmax);
    G[e] = (n < nb[k]) ? g0_tau(eps[kn] - mu, tau[i], beta) : 0.0;
}

// ---------------------------------------------------------------------------------------------
// synthetic M: Philox4x32-10 + Box-Muller, one draw per symmetry orbit
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = uint64_t(0xD2511F53u) * c[0];
        uint64_t p1 = uint64_t(0xCD9E8D57u) * c[2];
        uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
        uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
        uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return (double(a >> 5) * 67108864.0 + double(b >> 6) + 0.5) * (1.0 / 9007199254740992.0);
}

__global__ void k_synth(const int* __restrict__ kmq, const int* __restrict__ nb,
                        const int* __restrict__ ni, const int64_t* __restrict__ moff,
                        const int64_t* __restrict__ mpre, int nk, int nbmax, int q0, uint64_t seed,
                        int symmetric, int c64, void* __restrict__ M) {
    const int qk = blockIdx.y;
    const int q = q0 + qk / nk, k = qk % nk;
    const int kq = kmq[q * nk + k];
    const int nn = nb[k], nm = nb[kq], nI = ni[q];
    const int64_t blk = int64_t(nI) * nn * nm;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= blk) return;
    const int m = int(e % nm);
    const int n = int((e / nm) % nn);
    const int I = int(e / (int64_t(nn) * nm));
    auto lin = [&](int Q, int K, int N, int Mi) -> uint64_t {
        return ((uint64_t(Q) * nk + K) * nbmax + N) * uint64_t(nbmax) + Mi;
    };
    uint64_t xe = lin(q, k, n, m), canon = xe;
    bool conj = false, real = false;
    if (symmetric) {
        int mq = kmq[q * nk + 0];    // -q
        int mk = kmq[k * nk + 0];    // -k
        int qmk = kmq[k * nk + q];   // q - k
        uint64_t xa = lin(q, qmk, m, n);
        uint64_t xb = lin(mq, mk, n, m);
        uint64_t xab = lin(mq, kq, m, n);
        canon = min(min(xe, xa), min(xb, xab));
        conj = (canon != xe) && (canon != xa);
        real = (xb == xe) || (xab == xe);
    }
    uint32_t c[4] = {uint32_t(canon), uint32_t(canon >> 32), uint32_t(I), 0x4D475731u};
    philox10(c, uint32_t(seed), uint32_t(seed >> 32));
    double u1 = u53(c[0], c[1]), u2 = u53(c[2], c[3]);
    double rad = sqrt(-2.0 * log(u1));
    double ang = 2.0 * kPi * u2;
    double z0 = rad * cos(ang), z1 = rad * sin(ang);
    double var = 1.0 / (1.0 + double(I) / 16.0);
    double re, im;
    if (real) {
        re = sqrt(var) * z0;
        im = 0.0;
    } else {
        double sc = sqrt(var / 2.0);
        re = sc * z0;
        im = conj ? -(sc * z1) : sc * z1;
    }
    int64_t at = (mpre[q] - mpre[q0]) + moff[q * nk + k] + e;
    if (c64)
        reinterpret_cast<float2*>(M)[at] = make_float2(float(re), float(im));
    else
        reinterpret_cast<double2*>(M)[at] = make_double2(re, im);
}

// Cubic-symmetric M (harness-only input generation, the twin of the host generator): one draw per
// orbit of (k, q, G) under the 48 operations of O_h, keyed by the orbit's smallest (q' nk + k') NI + I'.
// rk: [48][nk] index of R k; rg: [48][NI] index of R G_I; g2: [NI] |G_I|^2.  One work-group per (q, k, I)
// row of nb x nb band pairs.
__global__ __launch_bounds__(256) void k_synth_cubic(const int* __restrict__ rk, const int* __restrict__ rg,
                                                     const int* __restrict__ g2, const int64_t* __restrict__ moff,
                                                     const int64_t* __restrict__ mpre, int nk, int nI, int nb,
                                                     int q0, uint64_t seed, int c64, void* __restrict__ M) {
    const int row = blockIdx.x;  // (qrel, k, I)
    const int I = row % nI, k = (row / nI) % nk, q = q0 + row / (nI * nk);
    uint64_t key = ~uint64_t(0);
    for (int r = 0; r < 48; ++r) {
        const uint64_t x = (uint64_t(rk[r * nk + q]) * nk + uint64_t(rk[r * nk + k])) * uint64_t(nI) + rg[r * nI + I];
        key = x < key ? x : key;
    }
    const double sc = sqrt(1.0 / (1.0 + double(g2[I]) / 4.0) / 2.0);
    const int64_t base = (mpre[q] - mpre[q0]) + moff[q * nk + k] + int64_t(I) * nb * nb;
    for (int e = threadIdx.x; e < nb * nb; e += 256) {
        uint32_t c[4] = {uint32_t(key), uint32_t(key >> 32), uint32_t(e), 0x4D435542u};
        philox10(c, uint32_t(seed), uint32_t(seed >> 32));
        const double u1 = u53(c[0], c[1]), u2 = u53(c[2], c[3]);
        const double rad = sqrt(-2.0 * log(u1)), ang = 2.0 * kPi * u2;
        const double re = sc * (rad * cos(ang)), im = sc * (rad * sin(ang));
        if (c64)
            reinterpret_cast<float2*>(M)[base + e] = make_float2(float(re), float(im));
        else
            reinterpret_cast<double2*>(M)[base + e] = make_double2(re, im);
    }
}

// Sigma[k] += sum over the star of q_ibz of C[R^-1 k] (kmap[q'][k] = R^-1 k for the operation R that
// maps q_ibz onto the star member q'), for Sigma^c (ntau values per state) and Sigma^x (one).
__global__ __launch_bounds__(256) void k_sigma_star(const int* __restrict__ kmap, const int* __restrict__ star,
                                                    int s0, int s1, int nk, int nbmax, int ntau,
                                                    const double* __restrict__ C, const double* __restrict__ Cx,
                                                    double* __restrict__ S, double* __restrict__ Sx) {
    const int64_t per = int64_t(nbmax) * ntau;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= int64_t(nk) * per) return;
    const int k = int(e / per);
    const int64_t rest = e - int64_t(k) * per;
    double acc = 0.0, accx = 0.0;
    for (int i = s0; i < s1; ++i) {
        const int kk = kmap[int64_t(star[i]) * nk + k];
        acc += C[int64_t(kk) * per + rest];
        if (Cx && rest % ntau == 0) accx += Cx[int64_t(kk) * nbmax + rest / ntau];
    }
    S[e] += acc;
    if (Sx && rest % ntau == 0) Sx[int64_t(k) * nbmax + rest / ntau] += accx;
}

// ---------------------------------------------------------------------------------------------
// forward transform: out[b][n][e] = sum_i W[n][i] (f[b][i][e] - G0(E, tau_i)) (+ 1/(i w_n - E))
// ---------------------------------------------------------------------------------------------
constexpr int FCH = 16;

template <bool CPLX>
__global__ void k_fwd(const double2* __restrict__ W, int niw, int ntau, int64_t nblk, int64_t len,
                      const void* __restrict__ f, const double* __restrict__ eref,
                      const double* __restrict__ tau, double beta, int fermion,
                      double2* __restrict__ out) {
    int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= nblk * len) return;
    int64_t b = idx / len, e = idx % len;
    int n0 = blockIdx.y * FCH;
    double E = eref ? eref[idx] : 0.0;
    double2 acc[FCH];
#pragma unroll
    for (int j = 0; j < FCH; ++j) acc[j] = make_double2(0.0, 0.0);
    auto load = [&](int i) {
        const int64_t at = (b * ntau + i) * len + e;
        return CPLX ? reinterpret_cast<const double2*>(f)[at]
                    : make_double2(reinterpret_cast<const double*>(f)[at], 0.0);
    };
    double2 fn = load(0);  // the next point's value is loaded while this one is accumulated
    for (int i = 0; i < ntau; ++i) {
        double2 fi = fn;
        if (i + 1 < ntau) fn = load(i + 1);
        if (eref) fi.x -= g0_tau(E, tau[i], beta);
#pragma unroll
        for (int j = 0; j < FCH; ++j) {
            int n = min(n0 + j, niw - 1);
            double2 w = W[int64_t(n) * ntau + i];
            acc[j].x += w.x * fi.x - w.y * fi.y;
            acc[j].y += w.x * fi.y + w.y * fi.x;
        }
    }
#pragma unroll
    for (int j = 0; j < FCH; ++j) {
        int n = n0 + j;
        if (n >= niw) break;
        double2 o = acc[j];
        if (eref) {
            double w = (fermion ? (2.0 * n + 1.0) : 2.0 * n) * kPi / beta;
            o = cadd(o, inv_iw_minus(w, E));
        }
        out[(b * niw + n) * len + e] = o;
    }
}

// ---------------------------------------------------------------------------------------------
// inverse fermionic transform (real output)
// ---------------------------------------------------------------------------------------------
constexpr int ICH = 16;

__global__ void k_inv_f(const double2* __restrict__ ef, int niw, int ntau, int64_t nblk,
                        int64_t len, const double2* __restrict__ F, const double* __restrict__ eref,
                        const double* __restrict__ tau, double beta, double* __restrict__ out) {
    int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= nblk * len) return;
    int64_t b = idx / len, e = idx % len;
    int i0 = blockIdx.y * ICH;
    double E = eref ? eref[idx] : 0.0;
    double acc[ICH];
#pragma unroll
    for (int j = 0; j < ICH; ++j) acc[j] = 0.0;
    for (int n = 0; n < niw; ++n) {
        double2 Fn = F[(b * niw + n) * len + e];
        if (eref) {
            double w = (2.0 * n + 1.0) * kPi / beta;
            double2 r = inv_iw_minus(w, E);
            Fn.x -= r.x;
            Fn.y -= r.y;
        }
#pragma unroll
        for (int j = 0; j < ICH; ++j) {
            int i = min(i0 + j, ntau - 1);
            double2 p = ef[int64_t(i) * niw + n];
            acc[j] += p.x * Fn.x - p.y * Fn.y;
        }
    }
#pragma unroll
    for (int j = 0; j < ICH; ++j) {
        int i = i0 + j;
        if (i >= ntau) break;
        double r = (2.0 / beta) * acc[j];
        if (eref) r += g0_tau(E, tau[i], beta);
        out[(b * ntau + i) * len + e] = r;
    }
}

// ---------------------------------------------------------------------------------------------
// inverse bosonic transform of Hermitian-pair matrices, with an optional exact-in-tau term
// add (scaled v_I add_IJ v_J when v is given)
// ---------------------------------------------------------------------------------------------
constexpr int BT = 16;    // matrix tile edge
constexpr int BTAU = 21;  // most tau points per work-group

// One work-group per (tile pair, tau chunk, block b): the tiles (ti, tj) and (tj, ti), ti <= tj, are
// produced together, so R(J, I) for the conjugate-pair term comes from the mirror tile through LDS and
// every element of R is read once per tau chunk.  With p = e^{-i nu tau}, S = R(I,J) + conj R(J,I)
// and D = R(I,J) - conj R(J,I), the pair p R(I,J) + conj(p) conj R(J,I) equals Re(p) S + i Im(p) D.
// The elements of the next frequency are loaded while the current one is combined, and the two tiles
// alternate between two LDS buffers, so one barrier per frequency suffices.
__global__ __launch_bounds__(256) void k_inv_b(const double2* __restrict__ eb, int niw, int ntau, int n,
                                               int nch, const double2* __restrict__ F,
                                               const double2* __restrict__ add, const double* __restrict__ v,
                                               double beta, double2* __restrict__ out) {
    __shared__ double2 ta[2][BT][BT + 1], tb[2][BT][BT + 1];
    extern __shared__ double2 ph[];  // [niw][BTAU] phases of this tau chunk
    const int nt = (n + BT - 1) / BT;
    int p = blockIdx.x, ti = 0;      // tile pair -> (ti, tj), rows of the upper triangle of tiles
    while (p >= nt - ti) {
        p -= nt - ti;
        ++ti;
    }
    const int tj = ti + p;
    const int c = blockIdx.y;
    const int i0 = int(int64_t(c) * ntau / nch), i1 = int(int64_t(c + 1) * ntau / nch);  // <= BTAU points
    const int64_t b = blockIdx.z, nn = int64_t(n) * n;
    const int tid = threadIdx.x, ty = tid / BT, tx = tid % BT;
    for (int e = tid; e < niw * BTAU; e += 256) {
        const int w = e / BTAU, j = e % BTAU;
        ph[e] = eb[int64_t(min(i0 + j, ntau - 1)) * niw + w];
    }
    const int IA = BT * ti + ty, JA = BT * tj + tx;  // element of tile A owned by this thread
    const int IB = BT * tj + ty, JB = BT * ti + tx;  // element of tile B
    const bool okA = IA < n && JA < n, okB = IB < n && JB < n;
    const bool two = ti != tj;
    const double2* Fb = F + b * niw * nn;
    const double2 z0 = make_double2(0.0, 0.0);
    double2 accA[BTAU], accB[BTAU];
    {
        const double2 a0 = okA ? Fb[int64_t(IA) * n + JA] : z0;
        const double2 b0 = okB && two ? Fb[int64_t(IB) * n + JB] : z0;
#pragma unroll
        for (int j = 0; j < BTAU; ++j) {
            accA[j] = a0;
            accB[j] = b0;
        }
    }
    __syncthreads();  // phases staged
    const int64_t offA = int64_t(IA) * n + JA, offB = int64_t(IB) * n + JB;
    double2 an = z0, bn = z0;  // the elements of frequency w + 1
    if (niw > 1) {
        an = okA ? Fb[nn + offA] : z0;
        bn = okB && two ? Fb[nn + offB] : z0;
    }
    for (int w = 1; w < niw; ++w) {
        const double2 a = an, bb = bn;
        if (w + 1 < niw) {
            const double2* Fn = Fb + int64_t(w + 1) * nn;
            an = okA ? Fn[offA] : z0;
            bn = okB && two ? Fn[offB] : z0;
        }
        const int buf = w & 1;  // written here, read after the barrier; rewritten two frequencies later
        ta[buf][ty][tx] = a;
        tb[buf][ty][tx] = bb;
        __syncthreads();
        const double2 tA = two ? tb[buf][tx][ty] : ta[buf][tx][ty];  // R(JA, IA)
        const double2 tB = ta[buf][tx][ty];                          // R(JB, IB)
        const double SAx = a.x + tA.x, SAy = a.y - tA.y, DAx = a.x - tA.x, DAy = a.y + tA.y;
        const double SBx = bb.x + tB.x, SBy = bb.y - tB.y, DBx = bb.x - tB.x, DBy = bb.y + tB.y;
        const double2* pw = ph + w * BTAU;
#pragma unroll
        for (int j = 0; j < BTAU; ++j) {
            const double2 q = pw[j];
            accA[j].x += q.x * SAx - q.y * DAy;
            accA[j].y += q.x * SAy + q.y * DAx;
            accB[j].x += q.x * SBx - q.y * DBy;
            accB[j].y += q.x * SBy + q.y * DBx;
        }
    }
    const double ib = 1.0 / beta;
    const double vA = okA && v ? v[IA] * v[JA] : 1.0, vB = okB && v ? v[IB] * v[JB] : 1.0;
#pragma unroll
    for (int j = 0; j < BTAU; ++j) {
        const int i = i0 + j;
        if (i >= i1) break;
        const int64_t base = (b * ntau + i) * nn;
        if (okA) {
            const int64_t at = base + int64_t(IA) * n + JA;
            double2 r = make_double2(accA[j].x * ib, accA[j].y * ib);
            if (add) {
                const double2 x = add[at];
                r.x += vA * x.x;
                r.y += vA * x.y;
            }
            out[at] = r;
        }
        if (okB && two) {
            const int64_t at = base + int64_t(IB) * n + JB;
            double2 r = make_double2(accB[j].x * ib, accB[j].y * ib);
            if (add) {
                const double2 x = add[at];
                r.x += vB * x.x;
                r.y += vB * x.y;
            }
            out[at] = r;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// exchange self-energy
// ---------------------------------------------------------------------------------------------
__device__ double block_sum(double x, double* red) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
    __syncthreads();
    if (l == 0) red[w] = x;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += red[i];
    return t;
}

// DIAG: block per (q, k, n); threads over m and slices of I
__global__ void k_sigx_diag(Dev d, int q0, const void* __restrict__ M, int c64,
                            const double* __restrict__ occ, const double* __restrict__ v,
                            double* __restrict__ out) {
    __shared__ double red[16];
    const int n = blockIdx.x;
    const int q = q0 + blockIdx.z, k = blockIdx.y;
    const int nk = d.nk;
    const int kq = d.kmq[q * nk + k];
    const int nn = d.nb[k], nm = d.nb[kq], nI = d.ni[q];
    if (n >= nn) return;
    const int64_t base = (d.mpre[q] - d.mpre[q0]) + d.moff[q * nk + k];
    const double* vq = v + (d.vpre[q] - d.vpre[q0]);
    // the threads cover mw >= nm columns m (whole waves, coalesced rows of M) times S slices of I
    const int mw = min(int(blockDim.x), (nm + 63) / 64 * 64), S = int(blockDim.x) / mw;
    const int sl = threadIdx.x / mw;
    double part = 0.0;
    if (sl < S) {
        for (int m = threadIdx.x % mw; m < nm; m += mw) {
            double s = 0.0;
#pragma unroll 4
            for (int I = sl; I < nI; I += S) {
                const double2 x = ld_c(M, base + (int64_t(I) * nn + n) * nm + m, c64);
                s += vq[I] * (x.x * x.x + x.y * x.y);
            }
            part += (-occ[(int64_t(kq) * d.nbmax + m) * d.ntau + d.ntau - 1]) * s;
        }
    }
    double tot = block_sum(part, red);
    if (threadIdx.x == 0) atomicAdd(&out[int64_t(k) * d.nbmax + n], d.scale * tot);
}

// FULL: block per (q, k, n); threads over n'
__global__ void k_sigx_full(Dev d, int q0, const void* __restrict__ M, int c64,
                            const double* __restrict__ occ, const double* __restrict__ v,
                            double2* __restrict__ out) {
    const int n = blockIdx.x;
    const int q = q0 + blockIdx.z, k = blockIdx.y;
    const int nk = d.nk;
    const int kq = d.kmq[q * nk + k];
    const int nn = d.nb[k], nm = d.nb[kq], nI = d.ni[q];
    if (n >= nn) return;
    const int64_t base = (d.mpre[q] - d.mpre[q0]) + d.moff[q * nk + k];
    const double* vq = v + (d.vpre[q] - d.vpre[q0]);
    for (int np = threadIdx.x; np < nn; np += blockDim.x) {
        double2 s = make_double2(0.0, 0.0);
        for (int m = 0; m < nm; ++m) {
            double f = (-occ[(int64_t(kq) * d.nbmax + m) * d.ntau + d.ntau - 1]);
            double2 t = make_double2(0.0, 0.0);
            for (int I = 0; I < nI; ++I) {
                double2 a = ld_c(M, base + (int64_t(I) * nn + n) * nm + m, c64);
                double2 b = ld_c(M, base + (int64_t(I) * nn + np) * nm + m, c64);
                // conj(a) b
                t.x += vq[I] * (a.x * b.x + a.y * b.y);
                t.y += vq[I] * (a.x * b.y - a.y * b.x);
            }
            s.x += f * t.x;
            s.y += f * t.y;
        }
        double2* o = &out[(int64_t(k) * d.nbmax + n) * d.nbmax + np];
        atomicAdd(&o->x, d.scale * s.x);
        atomicAdd(&o->y, d.scale * s.y);
    }
}

// ---------------------------------------------------------------------------------------------
// Dyson + chemical potential (one block) and G(i w), G(tau)
// ---------------------------------------------------------------------------------------------
struct DysonArgs {
    const double* eps;
    const double* sstat;
    const double2* sigc;
    const int* nb;
    int nk, nbmax, niw;
    double beta, n_target;
};

__device__ double number_partial(const DysonArgs& a, const double* E0, double mu) {
    double part = 0.0;
    const int64_t nstate = int64_t(a.nk) * a.nbmax;
    for (int64_t b = threadIdx.x; b < nstate; b += blockDim.x) {
        int k = int(b / a.nbmax), n = int(b % a.nbmax);
        if (n >= a.nb[k]) continue;
        double E = E0[b] - mu;
        double acc = 0.0;
        const double2* S = a.sigc + b * a.niw;
        for (int w = 0; w < a.niw; ++w) {
            double om = (2.0 * w + 1.0) * kPi / a.beta;
            double2 z = make_double2(-E, om);               // i w - E
            double2 s = S[w];
            double2 zs = make_double2(z.x - s.x, z.y - s.y);  // i w - E - Sigma
            // G - G_ref = Sigma / ((i w - E - Sigma)(i w - E))
            double2 d = cdiv(s, cmul(zs, z));
            acc += d.x;
        }
        part += fermi(E, a.beta) + (2.0 / a.beta) * acc;
    }
    return part;
}

// ---- chemical potential: multisection on N(mu) = n_target ------------------------------------------
// Each round evaluates N at MS_S + 2 equally spaced points of the bracket [lo, hi] (ends included), one
// work-group per point, and the next round (or the final kernel) narrows the bracket to the cell where
// N - n_target changes sign: a factor MS_S + 1 = 256 per round, 2^64 after MS_ROUNDS rounds.  The
// number of launches is fixed, so the search can be captured in a graph.  Search state in scratch
// (doubles): br[2][2] (bracket of the round, ping-pong), Nv[2][MS_S + 2], flags (as a double).
constexpr int MS_S = 255;
constexpr int MS_ROUNDS = 8;
constexpr int MS_NV = MS_S + 2;
__device__ __forceinline__ double* ms_br(double* st, int r) { return st + 2 * (r & 1); }
__device__ __forceinline__ double* ms_nv(double* st, int r) { return st + 4 + MS_NV * (r & 1); }
__device__ __forceinline__ double* ms_fl(double* st) { return st + 4 + 2 * MS_NV; }

// the bracket after round r: the cell [mu_j, mu_j+1] of round r's points that holds the sign change
// (the end of the old bracket where every point is on one side)
__device__ void ms_narrow(double* st, int r, double target, double& lo, double& hi) {
    const double* br = ms_br(st, r);
    const double* N = ms_nv(st, r);
    const double l0 = br[0], h0 = br[1];
    int jl = -1;
    for (int j = 0; j < MS_NV; ++j)
        if (N[j] < target) jl = j;
    auto at = [&](int j) { return l0 + (h0 - l0) * (double(j) / double(MS_S + 1)); };
    lo = jl >= 0 ? at(jl) : l0;
    hi = jl + 1 < MS_NV ? at(jl + 1) : h0;
}

// E0 = eps + Sigma_static (written to Eout), NaN check, initial bracket
__global__ __launch_bounds__(1024) void k_dyson_prep(DysonArgs a, double* Eout, double* st) {
    const int64_t nstate = int64_t(a.nk) * a.nbmax;
    double lo = 1e300, hi = -1e300;
    int bad = 0;
    for (int64_t b = threadIdx.x; b < nstate; b += blockDim.x) {
        int k = int(b / a.nbmax), n = int(b % a.nbmax);
        if (n >= a.nb[k]) {
            Eout[b] = 0.0;
            continue;
        }
        double e0 = a.eps[b] + a.sstat[b];
        Eout[b] = e0;
        if (!isfinite(e0)) bad = 1;
        lo = fmin(lo, e0);
        hi = fmax(hi, e0);
        for (int w = 0; w < a.niw; ++w) {
            double2 s = a.sigc[b * a.niw + w];
            if (!isfinite(s.x) || !isfinite(s.y)) bad = 1;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, o));
        hi = fmax(hi, __shfl_xor(hi, o));
        bad |= __shfl_xor(bad, o);
    }
    __shared__ double rlo[16], rhi[16];
    __shared__ int rbad[16];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
    if (l == 0) {
        rlo[w] = lo;
        rhi[w] = hi;
        rbad[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        lo = 1e300;
        hi = -1e300;
        bad = 0;
        for (int i = 0; i < nw; ++i) {
            lo = fmin(lo, rlo[i]);
            hi = fmax(hi, rhi[i]);
            bad |= rbad[i];
        }
        double* br = ms_br(st, 0);
        br[0] = lo - 50.0 / a.beta;
        br[1] = hi + 50.0 / a.beta;
        *ms_fl(st) = bad ? double(MSGW_FLAG_NAN) : 0.0;
    }
}

// round r: narrow the bracket of round r - 1 (r > 0), then N at point blockIdx.x of the new bracket
__global__ __launch_bounds__(1024) void k_dyson_round(DysonArgs a, const double* __restrict__ E, double* st,
                                                      int r) {
    __shared__ double red[16];
    double lo, hi;
    if (r == 0) {
        lo = ms_br(st, 0)[0];
        hi = ms_br(st, 0)[1];
    } else {
        ms_narrow(st, r - 1, a.n_target, lo, hi);
    }
    const int j = blockIdx.x;
    const double mu = lo + (hi - lo) * (double(j) / double(MS_S + 1));
    const double N = block_sum(number_partial(a, E, mu), red);
    if (threadIdx.x == 0) {
        ms_nv(st, r)[j] = N;
        if (j == 0) {
            ms_br(st, r)[0] = lo;
            ms_br(st, r)[1] = hi;
        }
        if (r == 1 && j == 0) {  // the ends of the first bracket were points 0 and MS_S + 1 of round 0
            const double* N0 = ms_nv(st, 0);
            if (!(N0[0] <= a.n_target && a.n_target <= N0[MS_NV - 1]))
                *ms_fl(st) = double(int(*ms_fl(st)) | MSGW_FLAG_NOBRACKET);
        }
    }
}

// final: mu (the middle of the last bracket, or the given one), N(mu), flags, E0 - mu
__global__ __launch_bounds__(1024) void k_dyson_mu(DysonArgs a, int search, double* mu_io, double* n_out,
                                                   int* flags, double* Eout, double* st) {
    __shared__ double red[16];
    const int64_t nstate = int64_t(a.nk) * a.nbmax;
    double mu;
    if (search) {
        double lo, hi;
        ms_narrow(st, MS_ROUNDS - 1, a.n_target, lo, hi);
        mu = 0.5 * (lo + hi);
    } else {
        mu = *mu_io;
    }
    int fl = int(*ms_fl(st));
    if (!search) fl &= ~MSGW_FLAG_NOBRACKET;
    double N = block_sum(number_partial(a, Eout, mu), red);
    if (!isfinite(N)) fl |= MSGW_FLAG_NAN;
    __syncthreads();
    for (int64_t b = threadIdx.x; b < nstate; b += blockDim.x) {
        int k = int(b / a.nbmax), n = int(b % a.nbmax);
        if (n < a.nb[k]) Eout[b] = Eout[b] - mu;
    }
    if (threadIdx.x == 0) {
        *mu_io = mu;
        *n_out = N;
        *flags = fl;
    }
}

__global__ void k_dyson_g(const double2* __restrict__ ef, const double* __restrict__ tau,
                          DysonArgs a, int ntau, const double* __restrict__ E_,
                          double2* __restrict__ G_iw, double* __restrict__ G_tau) {
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nstate = int64_t(a.nk) * a.nbmax;
    if (b >= nstate) return;
    const int k = int(b / a.nbmax), n = int(b % a.nbmax);
    const int i0 = blockIdx.y * ICH;
    if (n >= a.nb[k]) {
        if (G_iw && blockIdx.y == 0)
            for (int w = 0; w < a.niw; ++w) G_iw[b * a.niw + w] = make_double2(0.0, 0.0);
        for (int j = 0; j < ICH && i0 + j < ntau; ++j) G_tau[b * ntau + i0 + j] = 0.0;
        return;
    }
    const double E = E_[b];
    double acc[ICH];
#pragma unroll
    for (int j = 0; j < ICH; ++j) acc[j] = 0.0;
    for (int w = 0; w < a.niw; ++w) {
        double om = (2.0 * w + 1.0) * kPi / a.beta;
        double2 z = make_double2(-E, om);
        double2 s = a.sigc[b * a.niw + w];
        double2 zs = make_double2(z.x - s.x, z.y - s.y);
        if (G_iw && blockIdx.y == 0) G_iw[b * a.niw + w] = cdiv(make_double2(1.0, 0.0), zs);
        double2 d = cdiv(s, cmul(zs, z));
#pragma unroll
        for (int j = 0; j < ICH; ++j) {
            int i = min(i0 + j, ntau - 1);
            double2 p = ef[int64_t(i) * a.niw + w];
            acc[j] += p.x * d.x - p.y * d.y;
        }
    }
#pragma unroll
    for (int j = 0; j < ICH; ++j) {
        int i = i0 + j;
        if (i >= ntau) break;
        G_tau[b * ntau + i] = g0_tau(E, tau[i], a.beta) + (2.0 / a.beta) * acc[j];
    }
}

// ---------------------------------------------------------------------------------------------
// gap proxy: E_(N+1) - E_(N) of E^QP = eps + sstat + Re Sigma^c(i w_0) - mu (one block)
// ---------------------------------------------------------------------------------------------
__device__ double block_max(double x, double* red) {
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
    __syncthreads();
    if (l == 0) red[w] = x;
    __syncthreads();
    double t = -INFINITY;
    for (int i = 0; i < nw; ++i) t = fmax(t, red[i]);
    return t;
}

__device__ double eqp(const DysonArgs& a, double mu, int64_t b) {
    return a.eps[b] + a.sstat[b] + a.sigc[b * a.niw].x - mu;
}

// value of the N-th smallest energy (1-based) over the states n < Nb_k; energy(b) for state b
template <class EF>
__device__ double select_nth(EF energy, int nk, int nbmax, const int* nb, int N, double lo, double hi,
                             double* red) {
    const int64_t nstate = int64_t(nk) * nbmax;
    for (int s = 0; s < 200; ++s) {
        double mid = 0.5 * (lo + hi);
        double cnt = 0.0;
        for (int64_t b = threadIdx.x; b < nstate; b += blockDim.x) {
            int k = int(b / nbmax), n = int(b % nbmax);
            if (n < nb[k] && energy(b) <= mid) cnt += 1.0;
        }
        cnt = block_sum(cnt, red);
        if (cnt >= N)
            hi = mid;
        else
            lo = mid;
    }
    double best = -INFINITY;
    for (int64_t b = threadIdx.x; b < nstate; b += blockDim.x) {
        int k = int(b / nbmax), n = int(b % nbmax);
        if (n < nb[k]) {
            double e = energy(b);
            if (e <= hi) best = fmax(best, e);
        }
    }
    return block_max(best, red);
}

// gap E_(N+1) - E_(N) of the energies energy(b) over the states n < Nb_k
template <class EF>
__device__ void gap_of(EF energy, int nk, int nbmax, const int* nb, int N, double* gap) {
    __shared__ double red[16];
    const int64_t nstate = int64_t(nk) * nbmax;
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t b = threadIdx.x; b < nstate; b += blockDim.x) {
        int k = int(b / nbmax), n = int(b % nbmax);
        if (n >= nb[k]) continue;
        double e = energy(b);
        lo = fmin(lo, e);
        hi = fmax(hi, e);
    }
    hi = block_max(hi, red);
    lo = -block_max(-lo, red);
    const double start = lo - (1.0 + fabs(lo));
    const double eN = select_nth(energy, nk, nbmax, nb, N, start, hi, red);
    const double eN1 = select_nth(energy, nk, nbmax, nb, N + 1, start, hi, red);
    if (threadIdx.x == 0) *gap = eN1 - eN;
}

__global__ __launch_bounds__(1024) void k_gap(DysonArgs a, const double* mu_p, int N, double* gap) {
    const double mu = *mu_p;
    gap_of([&](int64_t b) { return eqp(a, mu, b); }, a.nk, a.nbmax, a.nb, N, gap);
}

// the same over given energies (quasiparticle energies of the continuation)
__global__ __launch_bounds__(1024) void k_gap_given(const double* __restrict__ E, int nk, int nbmax,
                                                    const int* __restrict__ nb, int N, double* gap) {
    gap_of([&](int64_t b) { return E[b]; }, nk, nbmax, nb, N, gap);
}

}  // namespace

void launch_synth_cubic(const Dev& d, const Host& h, hipStream_t s, uint64_t seed, int q0, int nq, int m_dtype,
                        void* M, const int* rk, const int* rg, const int* g2) {
    const int nI = h.ni[q0], nb = h.nb[0];
    const dim3 grid(unsigned(int64_t(nq) * h.nk * nI));
    MSGW_LAUNCH(k_synth_cubic, grid, dim3(256), 0, s, rk, rg, g2, d.moff, d.mpre, h.nk, nI, nb, q0, seed,
                m_dtype == MSGW_C64 ? 1 : 0, M);
    MSGW_HIP(hipGetLastError());
}

void launch_sigma_star(const Dev& d, const Host& h, hipStream_t s, const int* kmap, const int* star, int s0,
                       int s1, const double* C, const double* Cx, double* S, double* Sx) {
    const int64_t n = int64_t(h.nk) * h.nbmax * h.ntau;
    MSGW_LAUNCH(k_sigma_star, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, kmap, star, s0, s1, h.nk, h.nbmax,
                h.ntau, C, Cx, S, Sx);
    MSGW_HIP(hipGetLastError());
}

void launch_gap_given(const Dev& d, const Host& h, hipStream_t s, const double* E, int n_index, double* gap) {
    MSGW_LAUNCH(k_gap_given, dim3(1), dim3(1024), 0, s, E, h.nk, h.nbmax, d.nb, n_index, gap);
    MSGW_HIP(hipGetLastError());
}

void launch_gap(const Dev& d, const Host& h, hipStream_t s, const double* eps,
                const double* sstat, const void* sigc, const double* mu, int n_index, double* gap) {
    (void)h;
    DysonArgs a{eps, sstat, (const double2*)sigc, d.nb, d.nk, d.nbmax, d.niw_f, d.beta, 0.0};
    MSGW_LAUNCH(k_gap, dim3(1), dim3(1024), 0, s, a, mu, n_index, gap);
    MSGW_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------------
void launch_green0(const Dev& d, hipStream_t s, const double* eps, double mu, double* G) {
    int64_t tot = int64_t(d.nk) * d.nbmax * d.ntau;
    MSGW_LAUNCH(k_green0, dim3(ceil_div(tot, 256)), dim3(256), 0, s, eps, mu, d.nb, d.tau, d.nk,
                       d.nbmax, d.ntau, d.beta, G);
    MSGW_HIP(hipGetLastError());
}

void launch_synth_M(const Dev& d, const Host& h, hipStream_t s, uint64_t seed, int q0, int nq,
                    int symmetric, int m_dtype, void* M) {
    int64_t maxblk = 0;
    for (int q = q0; q < q0 + nq; ++q)
        for (int k = 0; k < h.nk; ++k)
            maxblk = std::max<int64_t>(maxblk, int64_t(h.ni[q]) * h.nb[k] * h.nb[h.kmq[size_t(q) * h.nk + k]]);
    if (int64_t(nq) * h.nk > 65535) throw Error(MSGW_ENOTSUP, "synth_M: nq * nk must be <= 65535");
    MSGW_LAUNCH(k_synth, dim3(ceil_div(maxblk, 256), nq * h.nk), dim3(256), 0, s, d.kmq, d.nb, d.ni,
                       d.moff, d.mpre, d.nk, d.nbmax, q0, seed, symmetric, m_dtype == MSGW_C64, M);
    MSGW_HIP(hipGetLastError());
}

void launch_fwd(const Dev& d, hipStream_t s, int stat, int64_t nblk, int64_t len, const void* f,
                int f_cplx, const double* eref, void* out) {
    const bool fer = stat == MSGW_FERMION;
    const int niw = fer ? d.niw_f : d.niw_b;
    const double2* W = fer ? d.wf : d.wb;
    dim3 grid(ceil_div(nblk * len, 256), ceil_div(niw, FCH));
    if (f_cplx)
        MSGW_LAUNCH(k_fwd<true>, grid, dim3(256), 0, s, W, niw, d.ntau, nblk, len, f, eref,
                           d.tau, d.beta, int(fer), (double2*)out);
    else
        MSGW_LAUNCH(k_fwd<false>, grid, dim3(256), 0, s, W, niw, d.ntau, nblk, len, f, eref,
                           d.tau, d.beta, int(fer), (double2*)out);
    MSGW_HIP(hipGetLastError());
}

void launch_inv_fermion(const Dev& d, hipStream_t s, int64_t nblk, int64_t len, const void* F,
                        const double* eref, double* out) {
    dim3 grid(ceil_div(nblk * len, 256), ceil_div(d.ntau, ICH));
    MSGW_LAUNCH(k_inv_f, grid, dim3(256), 0, s, d.ef, d.niw_f, d.ntau, nblk, len,
                       (const double2*)F, eref, d.tau, d.beta, out);
    MSGW_HIP(hipGetLastError());
}

void launch_inv_boson(const Dev& d, hipStream_t s, int64_t nblk, int mat_n, const void* F,
                      const void* add, const double* v, void* out) {
    const int64_t nt = ceil_div(mat_n, BT);
    const int nch = int(ceil_div(d.ntau, BTAU));
    const size_t lds = sizeof(double2) * size_t(d.niw_b) * BTAU;
    if (lds > 48 * 1024)
        throw Error(MSGW_ENOTSUP, "iw_to_tau: niw_b must be <= " + std::to_string(48 * 1024 / (16 * BTAU)) +
                                      " for BOSON matrices");
    if (nblk > 65535) throw Error(MSGW_ENOTSUP, "iw_to_tau: at most 65535 BOSON matrices per call");
    dim3 grid(ceil_div(nt * (nt + 1) / 2, 1), nch, unsigned(nblk));
    MSGW_LAUNCH(k_inv_b, grid, dim3(256), lds, s, d.eb, d.niw_b, d.ntau, mat_n, nch, (const double2*)F,
                (const double2*)add, v, d.beta, (double2*)out);
    MSGW_HIP(hipGetLastError());
}

void launch_sigma_x(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
                    int m_dtype, const double* occ, const double* v, void* out, int full) {
    dim3 grid(h.nbmax, h.nk, nq);
    if (full)
        MSGW_LAUNCH(k_sigx_full, grid, dim3(64), 0, s, d, q0, M, m_dtype == MSGW_C64, occ, v,
                           (double2*)out);
    else
        MSGW_LAUNCH(k_sigx_diag, grid, dim3(256), 0, s, d, q0, M, m_dtype == MSGW_C64, occ, v,
                           (double*)out);
    MSGW_HIP(hipGetLastError());
}

void launch_dyson(const Dev& d, const Host& h, hipStream_t s, const double* eps,
                  const double* sstat, const void* sigc, double n_target, int search, double* mu,
                  void* G_iw, double* G_tau, double* n_out, int* flags, double* E, double* st) {
    DysonArgs a{eps, sstat, (const double2*)sigc, d.nb, d.nk, d.nbmax, d.niw_f, d.beta, n_target};
    static_assert(sizeof(double) * (5 + 2 * MS_NV) <= kMuSearchBytes, "mu search state fits its scratch");
    MSGW_LAUNCH(k_dyson_prep, dim3(1), dim3(1024), 0, s, a, E, st);
    MSGW_HIP(hipGetLastError());
    for (int r = 0; search && r < MS_ROUNDS; ++r) {
        MSGW_LAUNCH(k_dyson_round, dim3(MS_NV), dim3(1024), 0, s, a, E, st, r);
        MSGW_HIP(hipGetLastError());
    }
    MSGW_LAUNCH(k_dyson_mu, dim3(1), dim3(1024), 0, s, a, search, mu, n_out, flags, E, st);
    MSGW_HIP(hipGetLastError());
    int64_t nstate = int64_t(h.nk) * h.nbmax;
    MSGW_LAUNCH(k_dyson_g, dim3(ceil_div(nstate, 128), ceil_div(h.ntau, ICH)), dim3(128), 0, s, d.ef,
                       d.tau, a, d.ntau, E, (double2*)G_iw, G_tau);
    MSGW_HIP(hipGetLastError());
}

}  // namespace msgw
