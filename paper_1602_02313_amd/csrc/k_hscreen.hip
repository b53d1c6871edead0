// The screen's Hermitian path: when P(q, i nu) is Hermitian, A = 1 - v^1/2 P v^1/2 is Hermitian and, for
// a polarization with P <= 0 (which the physics gives), positive definite; it is then inverted by the
// blocked sweep on its upper triangle without pivoting, half the flops of the pivoting Gauss-Jordan and
// no row swaps.  The sweep of a block J of indices, with R the others and A^(J) the state it leaves,
//     A_JJ <- -A_JJ^-1,  A_JR <- A_JJ^-1 A_JR,  A_RR <- A_RR - A_JR^H A_JJ^-1 A_JR,
// keeps the state Hermitian, so the upper triangle holds all of it; sweeping every block leaves -A^-1.
//   k_hp_check   per matrix max |A_ij - conj A_ji| and max |A_ij - delta_ij| (32 x 32 tile pairs);
//   k_hp_decide  Hermitian when the first is at most 1e-6 of the second (the Hermitian part is used);
//   k_hp_sym     the upper triangle <- the Hermitian part;
//   per 64-column block J:
//     k_hp_diag    one work-group per matrix sweeps A_JJ in LDS (every pivot must be positive, else the
//                  matrix is marked failed and left to the pivoting elimination), keeps X = A_JJ^-1;
//     k_hp_u       U = X A_JR for the columns outside J (FP64 MFMA tiles);
//     k_hp_update  A_RR -= A_JR^H U on the upper 64 x 64 tiles outside J (FP64 MFMA, XCD-aware grid);
//     k_hp_write   A_JR <- U;
//   k_hp_fin     W~ = v^1/2 (-S - 1) v^1/2 from the upper triangle S = -A^-1 (mirrored) and R = W~ - vPv.
// A matrix that is not Hermitian, or whose sweep met a non-positive pivot, goes through the pivoting
// Gauss-Jordan (k_gj.hip); the failed ones are rebuilt from P first.
#include "internal.h"

namespace msgw {
namespace {

typedef double hp_dbl4 __attribute__((ext_vector_type(4)));
constexpr int HP_W = 64;   // sweep block
constexpr int HP_T = 32;   // tile of the check, symmetrization and finish kernels
constexpr double HP_HERM_TOL = 1e-6;

__device__ __forceinline__ double2 hp_conj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double hp_abs1(double2 a) { return fmax(fabs(a.x), fabs(a.y)); }
__device__ __forceinline__ double2 hp_mul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// pair index u -> (ti, tj), ti <= tj, of a T x T upper triangle of tiles (row-major)
__device__ __forceinline__ void hp_pair(int u, int T, int& ti, int& tj) {
    ti = 0;
    while (u >= T - ti) {
        u -= T - ti;
        ++ti;
    }
    tj = ti + u;
}

struct HpState {
    unsigned long long *asym, *amax;  // [batch]
    int *flag, *fail, *skip_gj, *skip_rb;
    double2* X;  // [batch][64][64]  A_JJ^-1 of the current block
    double2* U;  // [batch][64][nimax]
    int nimax;
};

__global__ void k_hp_zero(unsigned long long* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__device__ __forceinline__ double hp_block_max(double m) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    return m;
}

// loads the tile (ti, tj) and its mirror (tj, ti) of a matrix into LDS (zeros outside the order)
__device__ __forceinline__ void hp_load_pair(const double2* A, int n, int ld, int i0, int j0,
                                             double2 (&t1)[HP_T][HP_T + 1], double2 (&t2)[HP_T][HP_T + 1]) {
    for (int e = threadIdx.x; e < HP_T * HP_T; e += 256) {
        const int r = e / HP_T, c = e % HP_T;
        t1[r][c] = (i0 + r < n && j0 + c < n) ? A[int64_t(i0 + r) * ld + j0 + c] : make_double2(0.0, 0.0);
        t2[r][c] = (j0 + r < n && i0 + c < n) ? A[int64_t(j0 + r) * ld + i0 + c] : make_double2(0.0, 0.0);
    }
}

__global__ __launch_bounds__(256) void k_hp_check(GjArgs g, int T, HpState st) {
    __shared__ double2 t1[HP_T][HP_T + 1], t2[HP_T][HP_T + 1];
    const int b = blockIdx.y;
    int n, ld;
    int64_t off;
    gj_item(g, b, n, ld, off);
    int ti, tj;
    hp_pair(blockIdx.x, T, ti, tj);
    const int i0 = ti * HP_T, j0 = tj * HP_T;
    if (i0 >= n || j0 >= n) return;
    hp_load_pair(g.A + off, n, ld, i0, j0, t1, t2);
    __syncthreads();
    double as = 0.0, am = 0.0;
    for (int e = threadIdx.x; e < HP_T * HP_T; e += 256) {
        const int r = e / HP_T, c = e % HP_T, i = i0 + r, j = j0 + c;
        if (i < n && j < n) {
            const double2 a = t1[r][c], m = t2[c][r];  // A_ij and A_ji
            as = fmax(as, hp_abs1(make_double2(a.x - m.x, a.y + m.y)));
            const double dg = i == j ? 1.0 : 0.0;
            am = fmax(am, fmax(hp_abs1(make_double2(a.x - dg, a.y)), hp_abs1(make_double2(m.x - dg, m.y))));
        }
    }
    as = hp_block_max(as);
    am = hp_block_max(am);
    if ((threadIdx.x & 63) == 0) {
        atomicMax(st.asym + b, static_cast<unsigned long long>(__double_as_longlong(as)));
        atomicMax(st.amax + b, static_cast<unsigned long long>(__double_as_longlong(am)));
    }
}

__global__ void k_hp_decide(int batch, HpState st) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const double as = __longlong_as_double(static_cast<long long>(st.asym[b]));
    const double am = __longlong_as_double(static_cast<long long>(st.amax[b]));
    st.flag[b] = as <= HP_HERM_TOL * am ? 1 : 0;
    st.fail[b] = 0;
}

__global__ __launch_bounds__(256) void k_hp_sym(GjArgs g, int T, HpState st) {
    __shared__ double2 t1[HP_T][HP_T + 1], t2[HP_T][HP_T + 1];
    const int b = blockIdx.y;
    if (!st.flag[b]) return;
    int n, ld;
    int64_t off;
    gj_item(g, b, n, ld, off);
    int ti, tj;
    hp_pair(blockIdx.x, T, ti, tj);
    const int i0 = ti * HP_T, j0 = tj * HP_T;
    if (i0 >= n || j0 >= n) return;
    double2* A = g.A + off;
    hp_load_pair(A, n, ld, i0, j0, t1, t2);
    __syncthreads();
    for (int e = threadIdx.x; e < HP_T * HP_T; e += 256) {
        const int r = e / HP_T, c = e % HP_T, i = i0 + r, j = j0 + c;
        if (i < n && j < n && i <= j) {
            const double2 a = t1[r][c], m = t2[c][r];
            A[int64_t(i) * ld + j] = make_double2(0.5 * (a.x + m.x), 0.5 * (a.y - m.y));
        }
    }
}

// sweep of the diagonal block J = [P, P + w) of each Hermitian matrix, in LDS
__global__ __launch_bounds__(256) void k_hp_diag(GjArgs g, int P, HpState st) {
    __shared__ double2 S[HP_W][HP_W + 1];
    const int b = blockIdx.x;
    if (!st.flag[b] || st.fail[b]) return;
    int n, ld;
    int64_t off;
    gj_item(g, b, n, ld, off);
    if (P >= n) return;
    const int w = min(HP_W, n - P);
    double2* A = g.A + off;
    const int tid = threadIdx.x;
    for (int e = tid; e < w * w; e += 256) {
        const int a = e / w, c = e % w;
        S[a][c] = a <= c ? A[int64_t(P + a) * ld + P + c] : hp_conj(A[int64_t(P + c) * ld + P + a]);
    }
    __syncthreads();
    for (int k = 0; k < w; ++k) {
        const double d = S[k][k].x;  // the same value in every thread: a uniform branch
        if (!(d > 0.0)) {
            if (tid == 0) st.fail[b] = 1;
            return;
        }
        const double rd = 1.0 / d;
        for (int e = tid; e < w * w; e += 256) {
            const int a = e / w, c = e % w;
            if (a != k && c != k) {
                const double2 t = hp_mul(S[a][k], S[k][c]);
                S[a][c].x -= t.x * rd;
                S[a][c].y -= t.y * rd;
            }
        }
        __syncthreads();
        for (int e = tid; e < w; e += 256) {
            if (e != k) {
                S[e][k].x *= rd;
                S[e][k].y *= rd;
                S[k][e].x *= rd;
                S[k][e].y *= rd;
            }
        }
        if (tid == 0) S[k][k] = make_double2(-rd, 0.0);
        __syncthreads();
    }
    // S = -A_JJ^-1: the new diagonal block (upper) and X = A_JJ^-1
    double2* X = st.X + int64_t(b) * HP_W * HP_W;
    for (int e = tid; e < w * w; e += 256) {
        const int a = e / w, c = e % w;
        X[a * HP_W + c] = make_double2(-S[a][c].x, -S[a][c].y);
        if (a <= c) A[int64_t(P + a) * ld + P + c] = S[a][c];
    }
}

// 64 x 64 complex tile C (+)= sum_k opA(r, k) opB(k, c) on FP64 MFMA (four waves, 32 x 32 each), the
// reduction in chunks of 16 staged through LDS.  AR / BT: the loaders' fastest index (rows of A / the
// reduction index of B) for coalesced reads.
template <class FA, class FB>
__device__ __forceinline__ void hp_mma(int K, bool AR, bool BT, FA fa, FB fb, hp_dbl4 (&cre)[2][2],
                                       hp_dbl4 (&cim)[2][2], double2 (&As)[64][17], double2 (&Bs)[16][65]) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32, r16 = lane & 15, k4 = lane >> 4;
    // each chunk is fetched into registers while the previous one is multiplied
    double2 pa[4], pb[4];
    auto fetch = [&](int t0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u;
            const int r = AR ? (e & 63) : (e >> 4), t = AR ? (e >> 6) : (e & 15);
            pa[u] = t0 + t < K ? fa(r, t0 + t) : make_double2(0.0, 0.0);
            const int tb = BT ? (e & 15) : (e >> 6), c = BT ? (e >> 4) : (e & 63);
            pb[u] = t0 + tb < K ? fb(t0 + tb, c) : make_double2(0.0, 0.0);
        }
    };
    fetch(0);
    for (int t0 = 0; t0 < K; t0 += 16) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u;
            As[AR ? (e & 63) : (e >> 4)][AR ? (e >> 6) : (e & 15)] = pa[u];
            Bs[BT ? (e & 15) : (e >> 6)][BT ? (e >> 4) : (e & 63)] = pb[u];
        }
        __syncthreads();
        if (t0 + 16 < K) fetch(t0 + 16);
#pragma unroll
        for (int k0 = 0; k0 < 16; k0 += 4) {
            double2 av[2], bv[2];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi) av[bi] = As[wr + bi * 16 + r16][k0 + k4];
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) bv[bj] = Bs[k0 + k4][wc + bj * 16 + r16];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    cre[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi].x, bv[bj].x, cre[bi][bj], 0, 0, 0);
                    cre[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[bi].y, bv[bj].y, cre[bi][bj], 0, 0, 0);
                    cim[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi].x, bv[bj].y, cim[bi][bj], 0, 0, 0);
                    cim[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi].y, bv[bj].x, cim[bi][bj], 0, 0, 0);
                }
        }
        __syncthreads();
    }
}

// the element (lane, acc index r4) of a 64 x 64 tile: D[i][j] of a 16 x 16 block sits in lane
// j + 16 (i % 4), element i / 4
__device__ __forceinline__ void hp_rc(int bi, int bj, int r4, int& r, int& c) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    r = (wv >> 1) * 32 + bi * 16 + 4 * r4 + (lane >> 4);
    c = (wv & 1) * 32 + bj * 16 + (lane & 15);
}

// U = X A_J,c for the column tile c0 (outside J); A_s,c from the upper triangle
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_hp_u(GjArgs g, int P,
                                                                                       HpState st) {
    __shared__ double2 As[64][17];
    __shared__ double2 Bs[16][65];
    const int b = blockIdx.y;
    if (!st.flag[b] || st.fail[b]) return;
    int n, ld;
    int64_t off;
    gj_item(g, b, n, ld, off);
    const int c0 = int(blockIdx.x) * 64;
    if (P >= n || c0 >= n || c0 == P) return;
    const int w = min(HP_W, n - P);
    const double2* A = g.A + off;
    const double2* X = st.X + int64_t(b) * HP_W * HP_W;
    double2* U = st.U + int64_t(b) * HP_W * st.nimax;
    hp_dbl4 cre[2][2], cim[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) cre[bi][bj] = cim[bi][bj] = hp_dbl4{0.0, 0.0, 0.0, 0.0};
    auto fa = [&](int r, int s) { return (r < w && s < w) ? X[r * HP_W + s] : make_double2(0.0, 0.0); };
    if (c0 > P) {  // right of J: rows P + s of the upper triangle
        auto fb = [&](int s, int c) {
            return (s < w && c0 + c < n) ? A[int64_t(P + s) * ld + c0 + c] : make_double2(0.0, 0.0);
        };
        hp_mma(w, false, false, fa, fb, cre, cim, As, Bs);
    } else {  // left of J: A_s,c = conj A_c,s, rows c of the upper triangle
        auto fb = [&](int s, int c) {
            return (s < w && c0 + c < n) ? hp_conj(A[int64_t(c0 + c) * ld + P + s]) : make_double2(0.0, 0.0);
        };
        hp_mma(w, false, true, fa, fb, cre, cim, As, Bs);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                int r, c;
                hp_rc(bi, bj, r4, r, c);
                if (r < w && c0 + c < n) U[int64_t(r) * st.nimax + c0 + c] = make_double2(cre[bi][bj][r4], cim[bi][bj][r4]);
            }
}

// A_ij -= sum_t conj(A_{P+t, i}) U_tj on the upper tiles (ti <= tj) outside J.  1-D XCD-aware grid:
// work-group L = 8 k + x takes tile k mod nu of matrix x + 8 (k / nu).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_hp_update(GjArgs g, int P, int T,
                                                                                            int nu, int batch,
                                                                                            HpState st) {
    __shared__ double2 As[64][17];
    __shared__ double2 Bs[16][65];
    const int xcd = int(blockIdx.x & 7), kx = int(blockIdx.x >> 3);
    const int b = xcd + 8 * (kx / nu);
    if (b >= batch || !st.flag[b] || st.fail[b]) return;
    int n, ld;
    int64_t off;
    gj_item(g, b, n, ld, off);
    int ti, tj;
    hp_pair(kx % nu, T, ti, tj);
    const int i0 = ti * 64, j0 = tj * 64;
    if (P >= n || i0 >= n || j0 >= n || i0 == P || j0 == P) return;
    const int w = min(HP_W, n - P);
    double2* A = g.A + off;
    const double2* U = st.U + int64_t(b) * HP_W * st.nimax;
    hp_dbl4 cre[2][2], cim[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                int r, c;
                hp_rc(bi, bj, r4, r, c);
                const double2 y = (i0 + r < n && j0 + c < n) ? A[int64_t(i0 + r) * ld + j0 + c] : make_double2(0.0, 0.0);
                cre[bi][bj][r4] = y.x;
                cim[bi][bj][r4] = y.y;
            }
    auto fb = [&](int t, int c) {
        return (t < w && j0 + c < n) ? U[int64_t(t) * st.nimax + j0 + c] : make_double2(0.0, 0.0);
    };
    // -conj(A_{P+t, i}): left of J it is -A_{i, P+t} (row i of the upper triangle), right of J the
    // conjugate of row P + t
    const bool left = i0 < P;
    auto fa = [&](int r, int t) {
        if (t >= w || i0 + r >= n) return make_double2(0.0, 0.0);
        const double2 a = left ? A[int64_t(i0 + r) * ld + P + t] : A[int64_t(P + t) * ld + i0 + r];
        return make_double2(-a.x, left ? -a.y : a.y);
    };
    hp_mma(w, !left, false, fa, fb, cre, cim, As, Bs);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                int r, c;
                hp_rc(bi, bj, r4, r, c);
                if (i0 + r < n && j0 + c < n)
                    A[int64_t(i0 + r) * ld + j0 + c] = make_double2(cre[bi][bj][r4], cim[bi][bj][r4]);
            }
}

// A_J,c <- U for the columns outside J (stored at (P + t, c) right of J, conjugated at (c, P + t) left of it)
__global__ __launch_bounds__(256) void k_hp_write(GjArgs g, int P, HpState st) {
    const int b = blockIdx.y;
    if (!st.flag[b] || st.fail[b]) return;
    int n, ld;
    int64_t off;
    gj_item(g, b, n, ld, off);
    const int c0 = int(blockIdx.x) * 64;
    if (P >= n || c0 >= n || c0 == P) return;
    const int w = min(HP_W, n - P);
    double2* A = g.A + off;
    const double2* U = st.U + int64_t(b) * HP_W * st.nimax;
    for (int e = threadIdx.x; e < 64 * HP_W; e += 256) {
        if (c0 > P) {
            const int t = e >> 6, c = c0 + (e & 63);
            if (t < w && c < n) A[int64_t(P + t) * ld + c] = U[int64_t(t) * st.nimax + c];
        } else {
            const int t = e & 63, c = c0 + (e >> 6);
            if (t < w && c < n) A[int64_t(c) * ld + P + t] = hp_conj(U[int64_t(t) * st.nimax + c]);
        }
    }
}

__global__ void k_hp_masks(int batch, HpState st) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const int f = st.flag[b], bad = st.fail[b];
    st.skip_gj[b] = (f && !bad) ? 1 : 0;
    st.skip_rb[b] = (f && bad) ? 0 : 1;
}

// W~ and R of the swept matrices from the upper triangle S = -A^-1: W~_ij = s_i s_j (-S_ij - delta_ij) for
// i <= j and W~_ji = conj W~_ij (s = v^1/2); R = W~ - v_i v_j P_ij
__global__ __launch_bounds__(256) void k_hp_fin(GjArgs g, int T, HpState st, const double2* __restrict__ Piw,
                                                const double* __restrict__ v, const int64_t* vpre,
                                                double2* __restrict__ R) {
    __shared__ double2 t1[HP_T][HP_T + 1];
    const int b = blockIdx.y;
    if (!st.skip_gj[b]) return;
    GjArgs ga = g;
    ga.skip = nullptr;
    int n, ld;
    int64_t off;
    gj_item(ga, b, n, ld, off);
    int ti, tj;
    hp_pair(blockIdx.x, T, ti, tj);
    const int i0 = ti * HP_T, j0 = tj * HP_T;
    if (i0 >= n || j0 >= n) return;
    const int q = g.q0 + b / g.niw_b;
    const double* vq = v + (vpre[q] - vpre[g.q0]);
    double2* A = g.A + off;
    const double2* Pm = Piw + off;
    double2* Rq = R ? R + off : nullptr;
    for (int e = threadIdx.x; e < HP_T * HP_T; e += 256) {
        const int r = e / HP_T, c = e % HP_T, i = i0 + r, j = j0 + c;
        t1[r][c] = (i < n && j < n && i <= j) ? A[int64_t(i) * ld + j] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < HP_T * HP_T; e += 256) {
        const int r = e / HP_T, c = e % HP_T, i = i0 + r, j = j0 + c;
        if (i >= n || j >= n || i > j) continue;
        const double f = sqrt(vq[i]) * sqrt(vq[j]);
        const double2 s = t1[r][c];
        const double2 wv = make_double2(f * (-s.x - (i == j ? 1.0 : 0.0)), -f * s.y);
        A[int64_t(i) * ld + j] = wv;
        if (i != j) A[int64_t(j) * ld + i] = hp_conj(wv);
        if (Rq) {
            const double vv = vq[i] * vq[j];
            const double2 p = Pm[int64_t(i) * ld + j];
            Rq[int64_t(i) * ld + j] = make_double2(wv.x - vv * p.x, wv.y - vv * p.y);
            if (i != j) {
                const double2 pm = Pm[int64_t(j) * ld + i];
                Rq[int64_t(j) * ld + i] = make_double2(wv.x - vv * pm.x, -wv.y - vv * pm.y);
            }
        }
    }
}

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

HpState hp_carve(char* p, int batch, int nimax) {
    HpState st;
    st.asym = reinterpret_cast<unsigned long long*>(p);
    p += al256(8 * size_t(batch));
    st.amax = reinterpret_cast<unsigned long long*>(p);
    p += al256(8 * size_t(batch));
    st.flag = reinterpret_cast<int*>(p);
    p += al256(4 * size_t(batch));
    st.fail = reinterpret_cast<int*>(p);
    p += al256(4 * size_t(batch));
    st.skip_gj = reinterpret_cast<int*>(p);
    p += al256(4 * size_t(batch));
    st.skip_rb = reinterpret_cast<int*>(p);
    p += al256(4 * size_t(batch));
    st.X = reinterpret_cast<double2*>(p);
    p += al256(sizeof(double2) * size_t(batch) * HP_W * HP_W);
    st.U = reinterpret_cast<double2*>(p);
    st.nimax = nimax;
    return st;
}

}  // namespace

size_t hp_scratch_bytes(int batch, int nimax) {
    return 2 * al256(8 * size_t(batch)) + 4 * al256(4 * size_t(batch)) +
           al256(sizeof(double2) * size_t(batch) * HP_W * HP_W) + al256(sizeof(double2) * size_t(batch) * HP_W * nimax);
}

void hp_run(const GjArgs& g, int batch, int nmax, int nimax, char* scratch, hipStream_t s, const int** skip_gj,
            const int** skip_rb) {
    if (batch > 65535) throw Error(MSGW_ENOTSUP, "screen: more than 65535 matrices in one call");
    HpState st = hp_carve(scratch, batch, nimax);
    *skip_gj = st.skip_gj;
    *skip_rb = st.skip_rb;
    MSGW_LAUNCH(k_hp_zero, dim3((batch + 255) / 256), dim3(256), 0, s, st.asym, batch);
    MSGW_LAUNCH(k_hp_zero, dim3((batch + 255) / 256), dim3(256), 0, s, st.amax, batch);
    const int T32 = (nmax + HP_T - 1) / HP_T, np32 = T32 * (T32 + 1) / 2;
    MSGW_LAUNCH(k_hp_check, dim3(np32, batch), dim3(256), 0, s, g, T32, st);
    MSGW_LAUNCH(k_hp_decide, dim3((batch + 255) / 256), dim3(256), 0, s, batch, st);
    MSGW_LAUNCH(k_hp_sym, dim3(np32, batch), dim3(256), 0, s, g, T32, st);
    const int T = (nmax + 63) / 64, nu = T * (T + 1) / 2;
    const unsigned groups = unsigned(batch + 7) / 8;
    for (int P = 0; P < nmax; P += HP_W) {
        MSGW_LAUNCH(k_hp_diag, dim3(batch), dim3(256), 0, s, g, P, st);
        MSGW_LAUNCH(k_hp_u, dim3(T, batch), dim3(256), 0, s, g, P, st);
        MSGW_LAUNCH(k_hp_update, dim3(8u * groups * unsigned(nu)), dim3(256), 0, s, g, P, T, nu, batch, st);
        MSGW_LAUNCH(k_hp_write, dim3(T, batch), dim3(256), 0, s, g, P, st);
    }
    MSGW_LAUNCH(k_hp_masks, dim3((batch + 255) / 256), dim3(256), 0, s, batch, st);
    MSGW_HIP(hipGetLastError());
}

void hp_finish(const GjArgs& g, int batch, int nmax, int nimax, char* scratch, const double2* Piw, const double* v,
               const int64_t* vpre, double2* R, hipStream_t s) {
    HpState st = hp_carve(scratch, batch, nimax);
    const int T32 = (nmax + HP_T - 1) / HP_T, np32 = T32 * (T32 + 1) / 2;
    MSGW_LAUNCH(k_hp_fin, dim3(np32, batch), dim3(256), 0, s, g, T32, st, Piw, v, vpre, R);
    MSGW_HIP(hipGetLastError());
}

}  // namespace msgw
