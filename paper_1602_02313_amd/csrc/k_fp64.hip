// FP64 contractions (the reference GPU path): polarization (eq. irpol) and the correlation
// self-energy (eq. sigc), as LDS-tiled complex GEMMs on v_mfma_f64_16x16x4f64: 64 x 64 output tiles of
// four waves (each a 32 x 32 quarter of 2 x 2 blocks of 16 x 16), the reduction in chunks of 16 complex
// terms staged in LDS with (re, im) interleaved along it, so that a complex product takes two real
// MFMAs per 2 terms (one for the real part, one for the imaginary part, whose B column is built from the
// same LDS values with a swap and a sign).  Layouts of the 16x16x4 FP64 MFMA: A[i][k] in lane i + 16 k,
// B[k][j] in lane j + 16 k, D[i][j] in lane j + 16 (i % 4), element i / 4.
#include "internal.h"

namespace msgw {
namespace {

constexpr int TT = 64;   // output tile (rows and columns)
constexpr int KC = 16;   // K chunk staged in LDS (complex terms)
typedef double f64x4 __attribute__((ext_vector_type(4)));

inline unsigned ceil_div(int64_t a, int64_t b) {
    const int64_t r = (a + b - 1) / b;
    if (r > int64_t(0xFFFFFFFFu)) throw Error(MSGW_ENOTSUP, "shape too large for one launch");
    return unsigned(r);
}

// P_IJ(q,tau) = s sum_k sum_nm M^I_nm g_nm conj(M^J_nm),  g_nm = G_n(k,tau) G_m(k-q,beta-tau)
// grid: x = I-tile * nt + J-tile, y = tau, z = q - q0.  Row I holds (Re, Im) of M^I along the reduction,
// the column J for Re P (Re, Im) of g M^J and for Im P (-Im, Re).
__global__ __launch_bounds__(256) void k_pol_fp64(Dev d, int q0, const double2* __restrict__ M,
                                                  const double* __restrict__ G,
                                                  double2* __restrict__ P) {
    __shared__ double As[TT][2 * KC + 1];
    __shared__ double Bs[2 * KC][TT + 1];
    const int q = q0 + blockIdx.z, it = blockIdx.y;
    const int nk = d.nk, ntau = d.ntau, nbmax = d.nbmax;
    const int NI = d.ni[q];
    const int nt = (NI + TT - 1) / TT;
    if (int(blockIdx.x) >= nt * nt) return;
    const int i0 = (blockIdx.x / nt) * TT, j0 = (blockIdx.x % nt) * TT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32, r16 = lane & 15, k4 = lane >> 4;
    const int itb = ntau - 1 - it;
    f64x4 cre[2][2], cim[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            cre[bi][bj] = f64x4{0.0, 0.0, 0.0, 0.0};
            cim[bi][bj] = f64x4{0.0, 0.0, 0.0, 0.0};
        }
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
                As[r][2 * c] = a.x;
                As[r][2 * c + 1] = a.y;
                Bs[2 * c][r] = b.x;
                Bs[2 * c + 1][r] = b.y;
            }
            __syncthreads();
#pragma unroll
            for (int k0 = 0; k0 < 2 * KC; k0 += 4) {
                const int kx = k0 + k4;
                double av[2], br[2], bi_[2];
#pragma unroll
                for (int bi = 0; bi < 2; ++bi) av[bi] = As[wr + 16 * bi + r16][kx];
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    const int col = wc + 16 * bj + r16;
                    br[bj] = Bs[kx][col];
                    bi_[bj] = (kx & 1) ? Bs[kx - 1][col] : -Bs[kx + 1][col];
                }
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj) {
                        cre[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi], br[bj], cre[bi][bj], 0, 0, 0);
                        cim[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi], bi_[bj], cim[bi][bj], 0, 0, 0);
                    }
            }
            __syncthreads();
        }
    }
    double2* Pq = P + (d.ppre[q] - d.ppre[q0]) + int64_t(it) * NI * NI;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int I = i0 + wr + 16 * bi + 4 * r4 + k4, J = j0 + wc + 16 * bj + r16;
                if (I < NI && J < NI) {
                    double2 v = make_double2(d.scale * cre[bi][bj][r4], d.scale * cim[bi][bj][r4]);
                    if (d.kb0 > 0) v = cadd(v, Pq[int64_t(I) * NI + J]);  // a range past k = 0 adds
                    Pq[int64_t(I) * NI + J] = v;
                }
            }
}

// Sigma_n(k,tau) += s sum_m G_m(k-q,tau) Re sum_I conj(M^I_nm) Y^I_nm,  Y = W~(q,tau) M(q,k)
// grid: x = I-tile * ncol + col-tile, y = tau, z = (q - q0) * nk + k.  Row I holds (Re, Im) of W~_I.,
// the column c for Re Y (Re, -Im) of M_.c and for Im Y (Im, Re).
__global__ __launch_bounds__(256) void k_sig_fp64(Dev d, int q0, const double2* __restrict__ M,
                                                  const double* __restrict__ G,
                                                  const double2* __restrict__ W,
                                                  double* __restrict__ Sig) {
    __shared__ double As[TT][2 * KC + 1];
    __shared__ double Bs[2 * KC][TT + 1];
    __shared__ double red[2][TT];
    const int nk = d.nk, ntau = d.ntau, nbmax = d.nbmax;
    const int q = q0 + blockIdx.z / nk, k = blockIdx.z % nk, it = blockIdx.y;
    if (k < d.kb0 || k >= d.kb1) return;  // outside a partial k range
    const int kq = d.kmq[q * nk + k];
    const int nn = d.nb[k], nm = d.nb[kq], NI = d.ni[q];
    const int Kk = nn * nm;
    const int nti = (NI + TT - 1) / TT, ntc = (Kk + TT - 1) / TT;
    if (int(blockIdx.x) >= nti * ntc) return;
    const int i0 = (blockIdx.x / ntc) * TT, c0 = (blockIdx.x % ntc) * TT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32, r16 = lane & 15, k4 = lane >> 4;
    const double2* A = M + (d.mpre[q] - d.mpre[q0]) + d.moff[q * nk + k];
    const double2* Wq = W + (d.ppre[q] - d.ppre[q0]) + int64_t(it) * NI * NI;
    f64x4 cre[2][2], cim[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            cre[bi][bj] = f64x4{0.0, 0.0, 0.0, 0.0};
            cim[bi][bj] = f64x4{0.0, 0.0, 0.0, 0.0};
        }
    for (int jc = 0; jc < NI; jc += KC) {
#pragma unroll
        for (int l = 0; l < (TT * KC) / 256; ++l) {
            const int e = tid + 256 * l;
            {
                const int r = e / KC, c = e % KC;
                const double2 w = (i0 + r < NI && jc + c < NI) ? Wq[int64_t(i0 + r) * NI + jc + c]
                                                               : make_double2(0.0, 0.0);
                As[r][2 * c] = w.x;
                As[r][2 * c + 1] = w.y;
            }
            {
                const int r = e / TT, c = e % TT;
                const double2 m = (jc + r < NI && c0 + c < Kk) ? A[int64_t(jc + r) * Kk + c0 + c]
                                                               : make_double2(0.0, 0.0);
                Bs[2 * r][c] = m.x;
                Bs[2 * r + 1][c] = m.y;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k0 = 0; k0 < 2 * KC; k0 += 4) {
            const int kx = k0 + k4;
            double av[2], br[2], bi_[2];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi) av[bi] = As[wr + 16 * bi + r16][kx];
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                const int col = wc + 16 * bj + r16;
                br[bj] = (kx & 1) ? -Bs[kx][col] : Bs[kx][col];
                bi_[bj] = (kx & 1) ? Bs[kx - 1][col] : Bs[kx + 1][col];
            }
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    cre[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi], br[bj], cre[bi][bj], 0, 0, 0);
                    cim[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi], bi_[bj], cim[bi][bj], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    // epilogue: Re(conj(M) Y) summed over this tile's rows: per lane its 8 rows of each column, then
    // over the four lanes of a column (k4) and the two waves that share the columns
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        const int col = c0 + wc + 16 * bj + r16;
        double s = 0.0;
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int I = i0 + wr + 16 * bi + 4 * r4 + k4;
                if (I < NI && col < Kk) {
                    const double2 m = A[int64_t(I) * Kk + col];
                    s += m.x * cre[bi][bj][r4] + m.y * cim[bi][bj][r4];
                }
            }
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        if (k4 == 0) red[wr / 32][wc + 16 * bj + r16] = s;
    }
    __syncthreads();
    if (tid < TT) {
        const int col = c0 + tid;
        if (col < Kk) {
            const double s = red[0][tid] + red[1][tid];
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
