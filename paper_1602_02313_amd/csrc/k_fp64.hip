// FP64 contractions (the reference GPU path): polarization (eq. irpol) and the correlation
// self-energy (eq. sigc), as LDS-tiled complex GEMMs on the FP64 vector units.
#include "internal.h"

namespace msgw {
namespace {

constexpr int TT = 64;   // output tile (rows and columns)
constexpr int KC = 16;   // K chunk staged in LDS

inline unsigned ceil_div(int64_t a, int64_t b) {
    const int64_t r = (a + b - 1) / b;
    if (r > int64_t(0xFFFFFFFFu)) throw Error(MSGW_ENOTSUP, "shape too large for one launch");
    return unsigned(r);
}

// P_IJ(q,tau) = s sum_k sum_nm M^I_nm g_nm conj(M^J_nm),  g_nm = G_n(k,tau) G_m(k-q,beta-tau)
// grid: x = I-tile * nt + J-tile, y = tau, z = q - q0.  256 threads, 4x4 complex per thread.
__global__ __launch_bounds__(256) void k_pol_fp64(Dev d, int q0, const double2* __restrict__ M,
                                                  const double* __restrict__ G,
                                                  double2* __restrict__ P) {
    __shared__ double2 As[TT][KC + 1];
    __shared__ double2 Bs[TT][KC + 1];
    const int q = q0 + blockIdx.z, it = blockIdx.y;
    const int nk = d.nk, ntau = d.ntau, nbmax = d.nbmax;
    const int NI = d.ni[q];
    const int nt = (NI + TT - 1) / TT;
    if (int(blockIdx.x) >= nt * nt) return;
    const int i0 = (blockIdx.x / nt) * TT, j0 = (blockIdx.x % nt) * TT;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int itb = ntau - 1 - it;
    double2 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);
    const double2* Mq = M + (d.mpre[q] - d.mpre[q0]);
    for (int k = d.kb0; k < d.kb1; ++k) {  // all k unless a partial range is set
        const int kq = d.kmq[q * nk + k];
        const int nn = d.nb[k], nm = d.nb[kq];
        const int Kk = nn * nm;
        const double2* A = Mq + d.moff[q * nk + k];
        const double* Gk = G + int64_t(k) * nbmax * ntau;
        const double* Gq = G + int64_t(kq) * nbmax * ntau;
        for (int kc = 0; kc < Kk; kc += KC) {
#pragma unroll
            for (int l = 0; l < (TT * KC) / 256; ++l) {
                const int e = tid + 256 * l;
                const int r = e / KC, c = e % KC;
                const int kk = kc + c;
                double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
                if (kk < Kk) {
                    if (i0 + r < NI) a = A[int64_t(i0 + r) * Kk + kk];
                    if (j0 + r < NI) {
                        const int n = kk / nm, m = kk - n * nm;
                        const double g = Gk[n * ntau + it] * Gq[m * ntau + itb];
                        double2 x = A[int64_t(j0 + r) * Kk + kk];
                        b = make_double2(g * x.x, g * x.y);
                    }
                }
                As[r][c] = a;
                Bs[r][c] = b;
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                double2 av[4], bv[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) av[a] = As[ty + 16 * a][c];
#pragma unroll
                for (int b = 0; b < 4; ++b) bv[b] = Bs[tx + 16 * b][c];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        // av * conj(bv)
                        acc[a][b].x += av[a].x * bv[b].x + av[a].y * bv[b].y;
                        acc[a][b].y += av[a].y * bv[b].x - av[a].x * bv[b].y;
                    }
            }
            __syncthreads();
        }
    }
    double2* Pq = P + (d.ppre[q] - d.ppre[q0]) + int64_t(it) * NI * NI;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int I = i0 + ty + 16 * a, J = j0 + tx + 16 * b;
            if (I < NI && J < NI) {
                double2 v = make_double2(d.scale * acc[a][b].x, d.scale * acc[a][b].y);
                if (d.kb0 > 0) v = cadd(v, Pq[int64_t(I) * NI + J]);  // a range past k = 0 adds
                Pq[int64_t(I) * NI + J] = v;
            }
        }
}

// Sigma_n(k,tau) += s sum_m G_m(k-q,tau) Re sum_I conj(M^I_nm) Y^I_nm,  Y = W~(q,tau) M(q,k)
// grid: x = I-tile * ncol + col-tile, y = tau, z = (q - q0) * nk + k.
__global__ __launch_bounds__(256) void k_sig_fp64(Dev d, int q0, const double2* __restrict__ M,
                                                  const double* __restrict__ G,
                                                  const double2* __restrict__ W,
                                                  double* __restrict__ Sig) {
    __shared__ double2 As[TT][KC + 1];
    __shared__ double2 Bs[KC][TT + 1];
    __shared__ double red[16][TT];
    const int nk = d.nk, ntau = d.ntau, nbmax = d.nbmax;
    const int q = q0 + blockIdx.z / nk, k = blockIdx.z % nk, it = blockIdx.y;
    if (k < d.kb0 || k >= d.kb1) return;  // outside a partial k range
    const int kq = d.kmq[q * nk + k];
    const int nn = d.nb[k], nm = d.nb[kq], NI = d.ni[q];
    const int Kk = nn * nm;
    const int nti = (NI + TT - 1) / TT, ntc = (Kk + TT - 1) / TT;
    if (int(blockIdx.x) >= nti * ntc) return;
    const int i0 = (blockIdx.x / ntc) * TT, c0 = (blockIdx.x % ntc) * TT;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const double2* A = M + (d.mpre[q] - d.mpre[q0]) + d.moff[q * nk + k];
    const double2* Wq = W + (d.ppre[q] - d.ppre[q0]) + int64_t(it) * NI * NI;
    double2 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);
    for (int jc = 0; jc < NI; jc += KC) {
#pragma unroll
        for (int l = 0; l < (TT * KC) / 256; ++l) {
            const int e = tid + 256 * l;
            {
                const int r = e / KC, c = e % KC;
                As[r][c] = (i0 + r < NI && jc + c < NI) ? Wq[int64_t(i0 + r) * NI + jc + c]
                                                        : make_double2(0.0, 0.0);
            }
            {
                const int r = e / TT, c = e % TT;
                Bs[r][c] = (jc + r < NI && c0 + c < Kk) ? A[int64_t(jc + r) * Kk + c0 + c]
                                                        : make_double2(0.0, 0.0);
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            double2 av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = As[ty + 16 * a][c];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Bs[c][tx + 16 * b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    acc[a][b].x += av[a].x * bv[b].x - av[a].y * bv[b].y;
                    acc[a][b].y += av[a].x * bv[b].y + av[a].y * bv[b].x;
                }
        }
        __syncthreads();
    }
    // epilogue: Re(conj(M) Y) summed over this tile's rows
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int col = c0 + tx + 16 * b;
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int I = i0 + ty + 16 * a;
            if (I < NI && col < Kk) {
                const double2 m = A[int64_t(I) * Kk + col];
                s += m.x * acc[a][b].x + m.y * acc[a][b].y;
            }
        }
        red[ty][tx + 16 * b] = s;
    }
    __syncthreads();
    if (tid < TT) {
        const int col = c0 + tid;
        if (col < Kk) {
            double s = 0.0;
            for (int t = 0; t < 16; ++t) s += red[t][tid];
            const int n = col / nm, m = col - (col / nm) * nm;
            const double g = G[(int64_t(kq) * nbmax + m) * ntau + it];
            atomicAdd(&Sig[(int64_t(k) * nbmax + n) * ntau + it], d.scale * g * s);
        }
    }
}

// FULL mode: Sigma_nn'(k,tau) += s sum_m G_m sum_I conj(M^I_nm) [W~ M_{.,.,m}]^I_n'
// block per (m, tau, (q,k)); Z = W~ B_m staged in LDS (NI * Nb_k <= 4096).
__global__ __launch_bounds__(256) void k_sig_full_fp64(Dev d, int q0,
                                                       const double2* __restrict__ M,
                                                       const double* __restrict__ G,
                                                       const double2* __restrict__ W,
                                                       double2* __restrict__ Sig) {
    extern __shared__ double2 Z[];
    const int nk = d.nk, ntau = d.ntau, nbmax = d.nbmax;
    const int q = q0 + blockIdx.z / nk, k = blockIdx.z % nk, it = blockIdx.y, m = blockIdx.x;
    const int kq = d.kmq[q * nk + k];
    const int nn = d.nb[k], nm = d.nb[kq], NI = d.ni[q];
    if (m >= nm) return;
    const double2* A = M + (d.mpre[q] - d.mpre[q0]) + d.moff[q * nk + k];
    const double2* Wq = W + (d.ppre[q] - d.ppre[q0]) + int64_t(it) * NI * NI;
    for (int e = threadIdx.x; e < NI * nn; e += blockDim.x) {
        const int I = e / nn, np = e % nn;
        double2 s = make_double2(0.0, 0.0);
        for (int J = 0; J < NI; ++J) s = cadd(s, cmul(Wq[int64_t(I) * NI + J], A[(int64_t(J) * nn + np) * nm + m]));
        Z[e] = s;
    }
    __syncthreads();
    const double g = d.scale * G[(int64_t(kq) * nbmax + m) * ntau + it];
    for (int e = threadIdx.x; e < nn * nn; e += blockDim.x) {
        const int n = e / nn, np = e % nn;
        double2 s = make_double2(0.0, 0.0);
        for (int I = 0; I < NI; ++I) {
            const double2 a = A[(int64_t(I) * nn + n) * nm + m];
            const double2 z = Z[I * nn + np];
            s.x += a.x * z.x + a.y * z.y;
            s.y += a.x * z.y - a.y * z.x;
        }
        double2* o = &Sig[((int64_t(k) * nbmax + n) * nbmax + np) * ntau + it];
        atomicAdd(&o->x, g * s.x);
        atomicAdd(&o->y, g * s.y);
    }
}

}  // namespace

void launch_pol_fp64(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
                     const double* G, void* P) {
    int maxt = 0;
    for (int q = q0; q < q0 + nq; ++q) {
        int nt = (h.ni[q] + TT - 1) / TT;
        maxt = std::max(maxt, nt * nt);
    }
    record_kernel_event(d, MSGW_OP_POLARIZATION, false, s);
    MSGW_LAUNCH(k_pol_fp64, dim3(maxt, h.ntau, nq), dim3(256), 0, s, d, q0,
                       (const double2*)M, G, (double2*)P);
    MSGW_HIP(hipGetLastError());
    record_kernel_event(d, MSGW_OP_POLARIZATION, true, s);
}

void launch_sig_fp64(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
                     const double* G, const void* W, void* Sig) {
    int maxt = 0;
    for (int q = q0; q < q0 + nq; ++q)
        for (int k = 0; k < h.nk; ++k) {
            int Kk = h.nb[k] * h.nb[h.kmq[size_t(q) * h.nk + k]];
            maxt = std::max(maxt, int(ceil_div(h.ni[q], TT) * ceil_div(Kk, TT)));
        }
    if (int64_t(nq) * h.nk > 65535) throw Error(MSGW_ENOTSUP, "self_energy: nq * nk must be <= 65535");
    record_kernel_event(d, MSGW_OP_SELF_ENERGY, false, s);
    MSGW_LAUNCH(k_sig_fp64, dim3(maxt, h.ntau, nq * h.nk), dim3(256), 0, s, d, q0,
                       (const double2*)M, G, (const double2*)W, (double*)Sig);
    MSGW_HIP(hipGetLastError());
    record_kernel_event(d, MSGW_OP_SELF_ENERGY, true, s);
}

void launch_sig_full_fp64(const Dev& d, const Host& h, hipStream_t s, int q0, int nq,
                          const void* M, const double* G, const void* W, void* Sig) {
    size_t lds = sizeof(double2) * size_t(h.nimax) * h.nbmax;
    if (lds > 65536) throw Error(MSGW_ENOTSUP, "FULL self-energy needs NI * Nb <= 4096");
    if (int64_t(nq) * h.nk > 65535) throw Error(MSGW_ENOTSUP, "self_energy: nq * nk must be <= 65535");
    MSGW_LAUNCH(k_sig_full_fp64, dim3(h.nbmax, h.ntau, nq * h.nk), dim3(256), lds, s, d, q0,
                       (const double2*)M, G, (const double2*)W, (double2*)Sig);
    MSGW_HIP(hipGetLastError());
}

}  // namespace msgw
