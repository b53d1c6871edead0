// The FULL band-matrix self-energy in split precision (MSGW_F16X3):
//     Sigma_nn'(k, tau) += s sum_q sum_m G_m(k - q, tau) sum_IJ conj(M^I_nm) W~_IJ(q, tau) M^J_n'm
// (eq. sigc for every pair of bands n, n' instead of n = n' only), as two contractions per (q, k) and
// chunk of tau points:
//   k_sf_ywm      Y(tau) = W~(q, tau) M(q, k): NI x NI times NI x K (K = Nb_k Nb_{k-q} columns (n', m)),
//                 F16X3 on v_mfma_f32_32x32x16_f16 with FP32 accumulation, written to the scratch in FP32;
//   k_sf_contract Sigma_nn' += s sum_I sum_m conj(M^I_nm) G_m(tau) Y^I_n'm: an Nb x Nb product with the
//                 reduction over (I, m), on v_mfma_f64_16x16x4f64 in FP64, split over 16-row groups of I
//                 with FP64 atomics into Sigma.
// The second contraction costs Nb_k / NI of the first (18% at 128 bands and NI = 700).
// F16X3 operands: each element x of W~(q, tau) and of M(q) is scaled by a power of two that puts the
// largest |Re|, |Im| below 2^14, then split into hi = f16(x) and lo = f16(x - hi); the products hi hi,
// hi lo and lo hi are summed in FP32 (the dropped lo lo is ~2^-22 relative) and the scales are undone
// when Y is written.  The complex product runs on real MFMAs with K interleaving (re, im): a row of W~
// holds (Re W, Im W) per J, the column for Re Y holds (Re M, -Im M) and the one for Im Y (Im M, Re M).
#include "internal.h"

namespace msgw {
namespace {

typedef _Float16 sf_f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 sf_f16x2 __attribute__((ext_vector_type(2)));
typedef float sf_floatx16 __attribute__((ext_vector_type(16)));
typedef uint32_t sf_u32x4 __attribute__((ext_vector_type(4)));
typedef double sf_dbl4 __attribute__((ext_vector_type(4)));

constexpr int SF_TC = 8;    // tau points per chunk at most (the scratch holds Y of one (q, k) and chunk)
constexpr int SF_KS = 16;   // J per stage of k_sf_ywm
constexpr int SF_RS = 20;   // LDS row stride in u32 (80 B)
constexpr int SF_IG = 16;   // rows I per work-group of k_sf_contract (its split of the reduction)

__device__ __forceinline__ uint32_t sf_pk(float a, float b) {
    sf_f16x2 v = {(_Float16)a, (_Float16)b};
    return __builtin_bit_cast(uint32_t, v);
}
// (a, b) -> packed hi = f16 (a, b) and lo = f16 (a - hi_a, b - hi_b); a - hi is exact in FP32
__device__ __forceinline__ void sf_split(float a, float b, uint32_t& h, uint32_t& l) {
    h = sf_pk(a, b);
    const sf_f16x2 hh = __builtin_bit_cast(sf_f16x2, h);
    l = sf_pk(a - float(hh.x), b - float(hh.y));
}
__device__ __forceinline__ uint32_t sf_conj(uint32_t p) { return p ^ 0x80000000u; }      // (re, -im)
__device__ __forceinline__ uint32_t sf_swap(uint32_t p) { return __builtin_amdgcn_alignbit(p, p, 16); }
__device__ __forceinline__ sf_floatx16 sf_mfma(sf_u32x4 a, sf_u32x4 b, sf_floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(sf_f16x8, a), __builtin_bit_cast(sf_f16x8, b),
                                                  c, 0, 0, 0);
}
// x with m < 2^x (m > 0)
__device__ __forceinline__ int sf_exp_above(double m) {
    int x;
    frexp(m, &x);
    return x;
}
// the scale exponent that puts m = max |Re|, |Im| below 2^14 (0 for an all-zero operand)
__device__ __forceinline__ int sf_scale_exp(unsigned long long bits) {
    const double m = __longlong_as_double(static_cast<long long>(bits));
    return m > 0.0 ? min(max(14 - sf_exp_above(m), -200), 200) : 0;
}

__global__ void k_sf_zero(unsigned long long* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}
// max |Re|, |Im| of n complex floats into *out (bits of a non-negative double: ordered as integers)
__global__ __launch_bounds__(256) void k_sf_max_c64(const float2* __restrict__ x, int64_t n,
                                                    unsigned long long* __restrict__ out) {
    double m = 0.0;
    for (int64_t i = blockIdx.x * int64_t(256) + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        const float2 v = x[i];
        m = fmax(m, fmax(fabs(double(v.x)), fabs(double(v.y))));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) atomicMax(out, static_cast<unsigned long long>(__double_as_longlong(m)));
}
// the same for W~(q, tau), one y-row of the grid per tau
__global__ __launch_bounds__(256) void k_sf_max_w(const double2* __restrict__ W, int64_t nn,
                                                  unsigned long long* __restrict__ out) {
    const double2* w = W + int64_t(blockIdx.y) * nn;
    double m = 0.0;
    for (int64_t i = blockIdx.x * int64_t(256) + threadIdx.x; i < nn; i += int64_t(gridDim.x) * 256) {
        const double2 v = w[i];
        m = fmax(m, fmax(fabs(v.x), fabs(v.y)));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0)
        atomicMax(out + blockIdx.y, static_cast<unsigned long long>(__double_as_longlong(m)));
}

// Y(tau) = W~(q, tau) A for the tau points t0 .. t0 + nt - 1, A = M(q, k) (NI x K, row stride K).
// Work-group: 4 waves over 64 rows I and 128 columns c, wave (wi, wc) a 32 x 64 quarter (two 32 x 32
// blocks); stages of 16 J staged through LDS (converted, scaled and split on the way), the next stage
// fetched into registers while the current one is multiplied.  Grid: (row tiles x column tiles, nt).
__global__ __launch_bounds__(256) void k_sf_ywm(const double2* __restrict__ Wq, const float2* __restrict__ A,
                                                float2* __restrict__ Y, int NI, int K, int t0, int tiles_i,
                                                const unsigned long long* __restrict__ mxw,
                                                const unsigned long long* __restrict__ mxm) {
    __shared__ uint32_t As[2][2][64][SF_RS];   // [buffer][hi, lo][row I][J]: packed (Re W, Im W)
    __shared__ uint32_t Bs[2][2][128][SF_RS];  // [buffer][hi, lo][column c][J]: packed (Re M, Im M)
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r32 = lane & 31, h2 = lane >> 5;
    const int wi = wave & 1, wc = wave >> 1;
    const int t = t0 + int(blockIdx.y);
    const int i0 = int(blockIdx.x % tiles_i) * 64, c0 = int(blockIdx.x / tiles_i) * 128;
    const int ew = sf_scale_exp(mxw[t]), em = sf_scale_exp(*mxm);
    const double fw = ldexp(1.0, ew);
    const float fmv = ldexpf(1.f, em);
    const double2* W = Wq + int64_t(t) * NI * NI;

    double2 ra[4];
    float2 rb[8];
    auto gload = [&](int J0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u, row = e >> 4, j = e & 15, I = i0 + row, J = J0 + j;
            ra[u] = (I < NI && J < NI) ? W[int64_t(I) * NI + J] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u, j = e >> 7, col = e & 127, J = J0 + j, c = c0 + col;
            rb[u] = (J < NI && c < K) ? A[int64_t(J) * K + c] : make_float2(0.f, 0.f);
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u, row = e >> 4, j = e & 15;
            uint32_t h, l;
            sf_split(float(ra[u].x * fw), float(ra[u].y * fw), h, l);
            As[buf][0][row][j] = h;
            As[buf][1][row][j] = l;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u, j = e >> 7, col = e & 127;
            uint32_t h, l;
            sf_split(rb[u].x * fmv, rb[u].y * fmv, h, l);
            Bs[buf][0][col][j] = h;
            Bs[buf][1][col][j] = l;
        }
    };

    sf_floatx16 acc[2][2];  // [column block][re, im]
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int x = 0; x < 16; ++x) acc[b][p][x] = 0.f;

    const int ns = (NI + SF_KS - 1) / SF_KS;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int s = 0; s < ns; ++s) {
        const int buf = s & 1;
        if (s + 1 < ns) gload((s + 1) * SF_KS);
#pragma unroll
        for (int kk = 0; kk < SF_KS / 8; ++kk) {
            // lane (r32, h2): row / column r32 of its block, J = 8 kk + 4 h2 .. + 3
            const int jo = 8 * kk + 4 * h2;
            const sf_u32x4 ah = *reinterpret_cast<const sf_u32x4*>(&As[buf][0][32 * wi + r32][jo]);
            const sf_u32x4 al = *reinterpret_cast<const sf_u32x4*>(&As[buf][1][32 * wi + r32][jo]);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int col = 64 * wc + 32 * b + r32;
                const sf_u32x4 bh = *reinterpret_cast<const sf_u32x4*>(&Bs[buf][0][col][jo]);
                const sf_u32x4 bl = *reinterpret_cast<const sf_u32x4*>(&Bs[buf][1][col][jo]);
                sf_u32x4 brh, brl, bih, bil;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    brh[e] = sf_conj(bh[e]);
                    brl[e] = sf_conj(bl[e]);
                    bih[e] = sf_swap(bh[e]);
                    bil[e] = sf_swap(bl[e]);
                }
                acc[b][0] = sf_mfma(ah, brh, acc[b][0]);
                acc[b][1] = sf_mfma(ah, bih, acc[b][1]);
                acc[b][0] = sf_mfma(ah, brl, acc[b][0]);
                acc[b][1] = sf_mfma(ah, bil, acc[b][1]);
                acc[b][0] = sf_mfma(al, brh, acc[b][0]);
                acc[b][1] = sf_mfma(al, bih, acc[b][1]);
            }
        }
        if (s + 1 < ns) lstore(buf ^ 1);
        __syncthreads();
    }
    // the 16 accumulators of lane l hold rows 8 g + 4 (l / 32) + r (index 4 g + r) of column l % 32
    const float sc = ldexpf(1.f, -(ew + em));
    float2* Yt = Y + int64_t(blockIdx.y) * NI * K;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int c = c0 + 64 * wc + 32 * b + r32;
        if (c >= K) continue;
#pragma unroll
        for (int x = 0; x < 16; ++x) {
            const int I = i0 + 32 * wi + 8 * (x >> 2) + 4 * h2 + (x & 3);
            if (I < NI) Yt[int64_t(I) * K + c] = make_float2(acc[b][0][x] * sc, acc[b][1][x] * sc);
        }
    }
}

// Sigma_nn'(k, t) += s sum_{I in the group} sum_m conj(M^I_nm) G_m(k - q, t) Y^I_n'm(t), for a 64 x 64
// tile (n, n'), one group of SF_IG rows I and one tau point per work-group, FP64.  The reduction index
// runs over (I, m) in chunks of 16 m; the complex product on real MFMAs with K interleaving (re, im):
// the row n holds (Re M, Im M), the column n' for Re Sigma (Re Y, Im Y), for Im Sigma (Im Y, -Re Y).
// Grid: (tiles_n * tiles_n * groups of I, nt).
__global__ __launch_bounds__(256) void k_sf_contract(const float2* __restrict__ A, const float2* __restrict__ Y,
                                                     const double* __restrict__ Gkq, double2* __restrict__ Sig,
                                                     int NI, int nn, int nm, int nbmax, int ntau, int t0,
                                                     int tiles_n, double s) {
    __shared__ double Xs[64][33];  // [row n][2 j + (re, im)]
    __shared__ double Ys[32][65];  // [2 j + (re, im)][column n']
    const int K = nn * nm;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int t = t0 + int(blockIdx.y);
    const int tile = int(blockIdx.x) % (tiles_n * tiles_n), grp = int(blockIdx.x) / (tiles_n * tiles_n);
    const int n0 = (tile % tiles_n) * 64, p0 = (tile / tiles_n) * 64;
    const int I0 = grp * SF_IG, I1 = min(I0 + SF_IG, NI);
    const float2* Yt = Y + int64_t(blockIdx.y) * NI * K;
    const int wr = (wave >> 1) * 32, wcl = (wave & 1) * 32;
    const int r16 = lane & 15, k4 = lane >> 4;
    sf_dbl4 cre[2][2], cim[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            cre[bi][bj] = sf_dbl4{0.0, 0.0, 0.0, 0.0};
            cim[bi][bj] = sf_dbl4{0.0, 0.0, 0.0, 0.0};
        }
    for (int I = I0; I < I1; ++I) {
        for (int m0 = 0; m0 < nm; m0 += 16) {
            // rows n: M^I_n,m0..m0+15; columns n': G_m Y^I_n',m for the same m
            for (int e = tid; e < 64 * 16; e += 256) {
                const int r = e >> 4, j = e & 15, n = n0 + r, m = m0 + j;
                float2 v = make_float2(0.f, 0.f);
                if (n < nn && m < nm) v = A[int64_t(I) * K + n * nm + m];
                Xs[r][2 * j] = v.x;
                Xs[r][2 * j + 1] = v.y;
            }
            for (int e = tid; e < 16 * 64; e += 256) {
                const int col = e >> 4, j = e & 15, np = p0 + col, m = m0 + j;
                double yr = 0.0, yi = 0.0;
                if (np < nn && m < nm) {
                    const float2 y = Yt[int64_t(I) * K + np * nm + m];
                    const double g = Gkq[int64_t(m) * ntau + t];
                    yr = g * y.x;
                    yi = g * y.y;
                }
                Ys[2 * j][col] = yr;
                Ys[2 * j + 1][col] = yi;
            }
            __syncthreads();
#pragma unroll
            for (int k0 = 0; k0 < 32; k0 += 4) {
                // lane (r16, k4): A row r16 and B column r16 of its 16 x 16 block, K index k0 + k4
                const int kx = k0 + k4;
                double av[2], br[2], bim[2];
#pragma unroll
                for (int bi = 0; bi < 2; ++bi) av[bi] = Xs[wr + 16 * bi + r16][kx];
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    const int col = wcl + 16 * bj + r16;
                    br[bj] = Ys[kx][col];
                    bim[bj] = (kx & 1) ? -Ys[kx - 1][col] : Ys[kx + 1][col];
                }
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj) {
                        cre[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi], br[bj], cre[bi][bj], 0, 0, 0);
                        cim[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi], bim[bj], cim[bi][bj], 0, 0, 0);
                    }
            }
            __syncthreads();
        }
    }
    // D[i][j] of a 16 x 16 block sits in lane j + 16 (i % 4), element i / 4
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int n = n0 + wr + 16 * bi + 4 * r4 + k4, np = p0 + wcl + 16 * bj + r16;
                if (n < nn && np < nn) {
                    double2* o = &Sig[(int64_t(n) * nbmax + np) * ntau + t];
                    atomicAdd(&o->x, s * cre[bi][bj][r4]);
                    atomicAdd(&o->y, s * cim[bi][bj][r4]);
                }
            }
}

}  // namespace

namespace {
// bytes of Y for one tau point at the largest (q, k) block
size_t sf_plane_bytes(const Host& h) {
    int64_t kmax = 0;
    for (int k = 0; k < h.nk; ++k)
        for (int q = 0; q < h.nk; ++q) kmax = std::max<int64_t>(kmax, int64_t(h.nb[k]) * h.nb[h.kmq[size_t(q) * h.nk + k]]);
    return size_t(h.nimax) * size_t(kmax) * sizeof(float2);
}
// tau points per chunk: up to SF_TC while Y stays within 1 GiB, at least one
int sf_tau_chunk(const Host& h) {
    const size_t plane = sf_plane_bytes(h);
    const int64_t fit = int64_t((size_t(1) << 30) / std::max<size_t>(plane, 1));
    return int(std::max<int64_t>(1, std::min<int64_t>({int64_t(SF_TC), int64_t(h.ntau), fit})));
}
size_t sf_maxima_bytes(const Host& h) { return (size_t(h.nk) * (1 + h.ntau) * 8 + 255) / 256 * 256; }
}  // namespace

size_t sigfull_split_scratch_bytes(const Host& h) {
    if (h.sigma_mode != MSGW_SIGMA_FULL) return 0;
    return sf_maxima_bytes(h) + sf_plane_bytes(h) * size_t(sf_tau_chunk(h));
}

void launch_sig_full_split(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
                           const double* G, const void* W, void* Sig, char* scratch, size_t scratch_bytes) {
    if (scratch_bytes < sigfull_split_scratch_bytes(h))
        throw Error(MSGW_ENOMEM, "workspace too small for the split FULL self-energy");
    const int nk = h.nk, ntau = h.ntau, nbmax = h.nbmax;
    auto* mxm = reinterpret_cast<unsigned long long*>(scratch);       // [nk]        max |Re|, |Im| of M(q)
    auto* mxw = mxm + nk;                                             // [nk][ntau]  the same of W~(q, tau)
    float2* Y = reinterpret_cast<float2*>(scratch + sf_maxima_bytes(h));
    const int tc = sf_tau_chunk(h);
    MSGW_LAUNCH(k_sf_zero, dim3((nk * (1 + ntau) + 255) / 256), dim3(256), 0, s, mxm, nk * (1 + ntau));
    for (int q = q0; q < q0 + nq; ++q) {
        const int64_t msz = h.mpre[q + 1] - h.mpre[q], nn = int64_t(h.ni[q]) * h.ni[q];
        if (msz > 0)
            MSGW_LAUNCH(k_sf_max_c64, dim3(unsigned(std::min<int64_t>((msz + 255) / 256, 2048))), dim3(256), 0, s,
                        (const float2*)M + (h.mpre[q] - h.mpre[q0]), msz, mxm + q);
        if (nn > 0)
            MSGW_LAUNCH(k_sf_max_w, dim3(unsigned(std::min<int64_t>((nn + 255) / 256, 64)), ntau), dim3(256), 0, s,
                        (const double2*)W + (h.ppre[q] - h.ppre[q0]), nn, mxw + int64_t(q) * ntau);
    }
    for (int q = q0; q < q0 + nq; ++q) {
        const int NI = h.ni[q];
        const double2* Wq = (const double2*)W + (h.ppre[q] - h.ppre[q0]);
        for (int k = 0; k < nk; ++k) {
            const int kq = h.kmq[size_t(q) * nk + k];
            const int nn = h.nb[k], nm = h.nb[kq], K = nn * nm;
            if (K == 0 || NI == 0) continue;
            const float2* A = (const float2*)M + (h.mpre[q] - h.mpre[q0]) + h.moff[size_t(q) * nk + k];
            const int tiles_i = (NI + 63) / 64, tiles_c = (K + 127) / 128, tiles_n = (nn + 63) / 64;
            const int groups = (NI + SF_IG - 1) / SF_IG;
            for (int t0 = 0; t0 < ntau; t0 += tc) {
                const int nt = std::min(tc, ntau - t0);
                MSGW_LAUNCH(k_sf_ywm, dim3(tiles_i * tiles_c, nt), dim3(256), 0, s, Wq, A, Y, NI, K, t0, tiles_i,
                            mxw + int64_t(q) * ntau, mxm + q);
                MSGW_LAUNCH(k_sf_contract, dim3(tiles_n * tiles_n * groups, nt), dim3(256), 0, s, A, Y,
                            G + int64_t(kq) * nbmax * ntau, (double2*)Sig + int64_t(k) * nbmax * nbmax * ntau, NI, nn,
                            nm, nbmax, ntau, t0, tiles_n, h.scale);
            }
        }
    }
    MSGW_HIP(hipGetLastError());
}

}  // namespace msgw
