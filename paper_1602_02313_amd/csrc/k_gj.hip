// Batched blocked Gauss-Jordan elimination with partial pivoting, FP64 complex.
//
// Two forms (GjArgs::mode):
//   GJ_INVERT  A (n x n, row stride n) is replaced by A^-1 with its columns permuted by the pivot
//              swaps; the pivot row of every column is recorded so the caller can undo them;
//   GJ_SOLVE   [A | B] (n x (ld - n) right-hand sides, row stride ld) is reduced until B holds A^-1 B.
// A step eliminates a panel of columns J = [a, a + w) within a window of columns [lo, hi):
//   k_gj_panel   one work-group per matrix, a 16 (or 8, 4) column panel in registers (row i in thread
//                i mod NT, slot i / NT): per column it picks the pivot (largest |re| + |im| at or below
//                the diagonal, the smallest row on ties), swaps the whole rows (every column), scales the
//                pivot row and eliminates the column from every other row.  The panel columns then hold
//                T[:, J], the columns of the product of the panel's elementary eliminations.
//   k_gj_update  C <- C + T[:, J] C_J on the window's columns outside the panel, for the rows outside
//                J, on 16x16x4 FP64 MFMA tiles of 64 x 64 (K = w in chunks of 16).
//   k_gj_update<FIN>  C_J <- T_JJ C_J on the same columns: the pivot rows need the old C_J that the
//                update tiles read, so they are finished after it, by a second launch of the same tiles.
// Matrices of order <= 1024 run two levels: 16-column panels update only the 64-column outer panel
// they belong to (window [P, P + 64)); the outer panel then holds T[:, J64] of its 64 eliminations and
// one K = 64 update (window: every column) applies them to the rest, so the whole matrix is read and
// written once per 64 columns instead of once per 16.  Larger orders run one level with 8- or
// 4-column panels.  A zero pivot sets info = its column + 1 (the first one) and the elimination runs on
// with IEEE infinities / NaN, as in the single-matrix form.
#include "internal.h"

namespace msgw {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 gj_recip(double2 a) {
    const double s = fmax(fabs(a.x), fabs(a.y));
    const double ax = a.x / s, ay = a.y / s;
    const double den = (ax * ax + ay * ay) * s;
    return make_double2(ax / den, -ay / den);
}

// row[jj] for a run-time jj without indexing the register array by it (bitwise select: a select of
// array elements would be folded back into an indexed load, which moves the array to scratch)
template <int NB>
__device__ __forceinline__ double2 pick(const double2 (&row)[NB], int jj) {
    unsigned long long rx = 0, ry = 0;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const unsigned long long m = 0ull - (unsigned long long)(c == jj);
        rx |= __double_as_longlong(row[c].x) & m;
        ry |= __double_as_longlong(row[c].y) & m;
    }
    return make_double2(__longlong_as_double(rx), __longlong_as_double(ry));
}

// A step's columns: the window [lo, hi) (clipped to the matrix's columns) without the panel
// [a, a + jb) when the panel lies inside it.  ov is the panel's overlap with the clipped window.
struct GjCols {
    int lo, hiC, a, ov;
    __device__ int count() const { return max(0, hiC - lo - ov); }
    __device__ int col(int cc) const {
        const int c = lo + cc;
        return (ov > 0 && c >= a) ? c + ov : c;
    }
};
__device__ __forceinline__ GjCols gj_cols(int lo, int hi, int ncol, int a, int jb) {
    GjCols w;
    w.lo = lo;
    w.hiC = min(hi, ncol);
    w.a = a;
    w.ov = max(0, min(w.hiC, a + jb) - max(lo, a));
    return w;
}

// swap_lo: the first column whose rows are swapped (0 when inverting; the outer panel's first column
// when solving, since the columns left of it are no longer read)
template <int NT, int RPT, int NB>
__global__ __launch_bounds__(NT) void k_gj_panel(GjArgs g, int j0, int swap_lo) {
    __shared__ double rv[NT / 64];
    __shared__ int ri[NT / 64];
    __shared__ double2 srow[2][NB];
    __shared__ double2 prow[NB];

    const int b = blockIdx.x;
    int n, ld;
    int64_t off;
    gj_item(g, b, n, ld, off);
    double2* A = g.A + off;
    if (j0 >= n) return;
    const int jb = min(NB, n - j0);
    const int tid = threadIdx.x;
    const int cend = g.mode == GJ_INVERT ? n : ld;

    double2 x[RPT][NB];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int i = u * NT + tid;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            x[u][c] = (i < n && c < jb) ? A[int64_t(i) * ld + j0 + c] : make_double2(0.0, 0.0);
    }

    // the column loop stays rolled; x is only indexed by unrolled (compile-time) c, with c == jj
    // selecting the current column, so the panel stays in registers
#pragma unroll 1
    for (int jj = 0; jj < jb; ++jj) {
        {
            const int j = j0 + jj;
            // ---- pivot: largest |re| + |im| in column j at rows >= j (smallest row on ties)
            double best = -1.0;
            int bi = n;
#pragma unroll
            for (int u = 0; u < RPT; ++u) {
                const int i = u * NT + tid;
                if (i >= j && i < n) {
                    const double2 xj = pick(x[u], jj);
                    const double m = fabs(xj.x) + fabs(xj.y);
                    if (m > best) {
                        best = m;
                        bi = i;
                    }
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
            if ((tid & 63) == 0) {
                rv[tid >> 6] = best;
                ri[tid >> 6] = bi;
            }
            __syncthreads();
            best = -1.0;
            bi = n;
            for (int w = 0; w < NT / 64; ++w)
                if (rv[w] > best || (rv[w] == best && ri[w] < bi)) {
                    best = rv[w];
                    bi = ri[w];
                }
            const int p = bi < n ? bi : j;  // an all-NaN column keeps its row
            if (tid == 0) g.perm[int64_t(b) * g.pmax + j] = p;
            const int oj = j % NT, uj = j / NT, opv = p % NT, upv = p / NT;
            if (p != j) {
                // the panel part of rows j and p through LDS, the rest in memory (each thread always
                // swaps the same columns, so successive swaps of a column stay in order)
                if (tid == oj) {
#pragma unroll
                    for (int u = 0; u < RPT; ++u)
                        if (u == uj)
#pragma unroll
                            for (int c = 0; c < NB; ++c) srow[0][c] = x[u][c];
                }
                if (tid == opv) {
#pragma unroll
                    for (int u = 0; u < RPT; ++u)
                        if (u == upv)
#pragma unroll
                            for (int c = 0; c < NB; ++c) srow[1][c] = x[u][c];
                }
                // four columns per round: their loads are all issued before the stores
                double2* rj = A + int64_t(j) * ld;
                double2* rp = A + int64_t(p) * ld;
                for (int c0 = swap_lo + tid; c0 < cend; c0 += 4 * NT) {
                    double2 tj[4], tp[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int c = c0 + u * NT;
                        const bool ok = c < cend && (c < j0 || c >= j0 + jb);
                        tj[u] = ok ? rj[c] : make_double2(0.0, 0.0);
                        tp[u] = ok ? rp[c] : make_double2(0.0, 0.0);
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int c = c0 + u * NT;
                        if (c < cend && (c < j0 || c >= j0 + jb)) {
                            rj[c] = tp[u];
                            rp[c] = tj[u];
                        }
                    }
                }
                __syncthreads();
                if (tid == oj) {
#pragma unroll
                    for (int u = 0; u < RPT; ++u)
                        if (u == uj)
#pragma unroll
                            for (int c = 0; c < NB; ++c) x[u][c] = srow[1][c];
                }
                if (tid == opv) {
#pragma unroll
                    for (int u = 0; u < RPT; ++u)
                        if (u == upv)
#pragma unroll
                            for (int c = 0; c < NB; ++c) x[u][c] = srow[0][c];
                }
            }
            // ---- scale the pivot row
            if (tid == oj) {
#pragma unroll
                for (int u = 0; u < RPT; ++u)
                    if (u == uj) {
                        const double2 piv = pick(x[u], jj);
                        if (piv.x == 0.0 && piv.y == 0.0 && g.info[b] == 0) g.info[b] = j + 1;
                        const double2 inv = gj_recip(piv);
#pragma unroll
                        for (int c = 0; c < NB; ++c) {
                            const double2 val = (c == jj) ? inv : cmul(x[u][c], inv);
                            x[u][c] = val;
                            prow[c] = val;
                        }
                    }
            }
            __syncthreads();
            // ---- eliminate column j from the other rows of the panel
            const double2 inv = prow[jj];
#pragma unroll
            for (int u = 0; u < RPT; ++u) {
                const int i = u * NT + tid;
                if (i < n && i != j) {
                    const double2 f = pick(x[u], jj);
                    const double2 w = cmul(f, inv);
#pragma unroll
                    for (int c = 0; c < NB; ++c) {
                        const double2 r = prow[c];
                        double2 y = x[u][c];
                        y.x -= f.x * r.x - f.y * r.y;
                        y.y -= f.x * r.y + f.y * r.x;
                        x[u][c] = (c == jj) ? make_double2(-w.x, -w.y) : y;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int i = u * NT + tid;
        if (i < n)
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c < jb) A[int64_t(i) * ld + j0 + c] = x[u][c];
    }
}

// C <- C + T[:, J] C_J for the rows outside J = [a, a + w) on the step's columns (window [lo, hi)
// without the panel), K = w in chunks of 16, 64 x 64 tiles of four waves.  FIN: the pivot rows'
// C_J <- T_JJ C_J instead (one row tile; a work-group reads all of its columns' C_J before it writes
// them, and no other work-group touches those columns).
// The grid is 1-D and XCD-aware: work-group L runs on XCD L mod 8 (round-robin dispatch), and the
// tiles of matrix b all run on XCD b mod 8 (as its panel kernel does), so a matrix's T and C_J tiles are
// fetched into one L2 instead of eight: L = 8 k + x takes tile k mod ntiles of matrix x + 8 (k / ntiles).
// Three waves per SIMD: the accumulators then live in VGPRs.
template <int W, bool FIN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_gj_update(
    GjArgs g, int a, int lo, int hi, int tiles_m, int ntiles, int batch) {
    constexpr int KC = W < 16 ? W : 16;
    __shared__ double2 As[64][KC + 1];
    __shared__ double2 Bs[KC][64];

    const int xcd = int(blockIdx.x & 7), kx = int(blockIdx.x >> 3);
    const int b = xcd + 8 * (kx / ntiles), tile = kx % ntiles;
    if (b >= batch) return;
    int n, ld;
    int64_t off;
    gj_item(g, b, n, ld, off);
    if (a >= n) return;
    const int jb = min(W, n - a);
    const GjCols cols = gj_cols(lo, hi, g.mode == GJ_INVERT ? n : ld, a, jb);
    const int ncols = cols.count();
    const int row0 = FIN ? a : (tile % tiles_m) * 64;
    const int col0 = (FIN ? tile : tile / tiles_m) * 64;
    const int rend = FIN ? a + jb : n;
    if (row0 >= rend || col0 >= ncols) return;
    double2* A = g.A + off;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const int r16 = lane & 15, k4 = lane >> 4;
    auto row_ok = [&](int i) { return i < rend && (FIN || i < a || i >= a + jb); };
    // the accumulators start from C (the update) or from zero (FIN): the tile's C is fetched once, while
    // the first chunk is staged, and written once at the end
    dbl4 cre[2][2], cim[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int i = row0 + wr + bi * 16 + 4 * r4 + k4;
                const int cc = col0 + wc + bj * 16 + r16;
                double2 y = make_double2(0.0, 0.0);
                if (!FIN && row_ok(i) && cc < ncols) y = A[int64_t(i) * ld + cols.col(cc)];
                cre[bi][bj][r4] = y.x;
                cim[bi][bj][r4] = y.y;
            }
    // T[rows, J] (the update: zero on the pivot rows) and C_J[:, cols] of a K chunk, fetched into
    // registers one chunk ahead of the MFMAs
    constexpr int NE = 64 * KC / 256;
    double2 pa[NE], pb[NE];
    auto fetch = [&](int t0) {
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int e = tid + u * 256;
            const int r = e / KC, t = e % KC, i = row0 + r;
            pa[u] = (t0 + t < jb && row_ok(i)) ? A[int64_t(i) * ld + a + t0 + t] : make_double2(0.0, 0.0);
            const int tb = e / 64, cc = col0 + (e % 64);
            pb[u] = (t0 + tb < jb && cc < ncols) ? A[int64_t(a + t0 + tb) * ld + cols.col(cc)]
                                                 : make_double2(0.0, 0.0);
        }
    };
    fetch(0);
    for (int t0 = 0; t0 < jb; t0 += KC) {
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int e = tid + u * 256;
            As[e / KC][e % KC] = pa[u];
            Bs[e / 64][e % 64] = pb[u];
        }
        __syncthreads();
        if (t0 + KC < jb) fetch(t0 + KC);
#pragma unroll
        for (int k0 = 0; k0 < KC; k0 += 4) {
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
    // D[i][j] of a 16 x 16 block sits in lane j + 16 (i % 4), element i / 4 (A[i][k] in lane i + 16 k,
    // B[k][j] in lane j + 16 k)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int i = row0 + wr + bi * 16 + 4 * r4 + k4;
                const int cc = col0 + wc + bj * 16 + r16;
                if (row_ok(i) && cc < ncols)
                    A[int64_t(i) * ld + cols.col(cc)] = make_double2(cre[bi][bj][r4], cim[bi][bj][r4]);
            }
}

__global__ void k_gj_zero(int* p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// one elimination step's update and finish on the window [lo, hi) without the panel [a, a + W)
template <int W>
void gj_apply(const GjArgs& g, int batch, int nmax, int cmax, int a, int lo, int hi, hipStream_t s) {
    const int tiles_m = (nmax + 63) / 64, span = std::max(0, std::min(hi, cmax) - lo);
    const int tiles_n = (span + 63) / 64;
    if (tiles_n == 0) return;
    const unsigned groups = unsigned(batch + 7) / 8;
    MSGW_LAUNCH((k_gj_update<W, false>), dim3(8u * groups * unsigned(tiles_m * tiles_n)), dim3(256), 0, s, g, a, lo,
                hi, tiles_m, tiles_m * tiles_n, batch);
    MSGW_LAUNCH((k_gj_update<W, true>), dim3(8u * groups * unsigned(tiles_n)), dim3(256), 0, s, g, a, lo, hi, 1,
                tiles_n, batch);
}

// one level: panels of NB columns, each applied to every column of its step
template <int NT, int RPT, int NB>
void gj_one_level(const GjArgs& g, int batch, int nmax, int cmax, hipStream_t s) {
    for (int j0 = 0; j0 < nmax; j0 += NB) {
        MSGW_LAUNCH((k_gj_panel<NT, RPT, NB>), dim3(batch), dim3(NT), 0, s, g, j0, g.mode == GJ_INVERT ? 0 : j0);
        // solving: from the panel on (a matrix whose order ends inside the panel has right-hand sides there)
        gj_apply<NB>(g, batch, nmax, cmax, j0, g.mode == GJ_INVERT ? 0 : j0, cmax, s);
    }
}

// two levels: 16-column panels within 64-column outer panels (orders <= 1024, every matrix's panels
// at the same columns; a matrix whose order ends inside a panel sees a narrower one)
void gj_two_level(const GjArgs& g, int batch, int nmax, int cmax, hipStream_t s) {
    constexpr int NB = 16, NBO = 64;
    for (int P = 0; P < nmax; P += NBO) {
        for (int j0 = P; j0 < std::min(P + NBO, nmax); j0 += NB) {
            MSGW_LAUNCH((k_gj_panel<512, 2, NB>), dim3(batch), dim3(512), 0, s, g, j0, g.mode == GJ_INVERT ? 0 : P);
            gj_apply<NB>(g, batch, nmax, cmax, j0, P, P + NBO, s);  // within the outer panel only
        }
        if (g.mode == GJ_INVERT)
            gj_apply<NBO>(g, batch, nmax, cmax, P, 0, cmax, s);
        else
            gj_apply<NBO>(g, batch, nmax, cmax, P, P + NBO, cmax, s);
    }
}

}  // namespace

void gj_run(const GjArgs& g, int batch, int nmax, int ldmax, hipStream_t s) {
    if (batch <= 0 || nmax <= 0) return;
    if (nmax > kGjMaxN) throw Error(MSGW_ENOTSUP, "Gauss-Jordan: order above 4096");
    if (batch > 65535) throw Error(MSGW_ENOTSUP, "Gauss-Jordan: more than 65535 matrices in one call");
    const int cmax = g.mode == GJ_INVERT ? nmax : ldmax;
    // the update's 1-D grid holds at most 2^32 - 1 threads
    if (8.0 * ((batch + 7) / 8) * ((nmax + 63) / 64) * ((cmax + 63) / 64) * 256.0 > 4294967295.0)
        throw Error(MSGW_ENOTSUP, "Gauss-Jordan: too many update tiles for one launch (split the call)");
    MSGW_LAUNCH(k_gj_zero, dim3((batch + 255) / 256), dim3(256), 0, s, g.info, batch);
    // the panel stays in registers: RPT rows of NB complex columns per thread
    if (nmax <= 1024)
        gj_two_level(g, batch, nmax, cmax, s);
    else if (nmax <= 2048)
        gj_one_level<512, 4, 8>(g, batch, nmax, cmax, s);
    else
        gj_one_level<512, 8, 4>(g, batch, nmax, cmax, s);
    MSGW_HIP(hipGetLastError());
}

}  // namespace msgw
