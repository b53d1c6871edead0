// Batched blocked Gauss-Jordan elimination with partial pivoting, FP64 complex.
//
// Two forms (GjArgs::mode):
//   GJ_INVERT  A (n x n, row stride n) is replaced by A^-1 with its columns permuted by the pivot
//              swaps; the pivot row of every column is recorded so the caller can undo them;
//   GJ_SOLVE   [A | B] (n x (ld - n) right-hand sides, row stride ld) is reduced until B holds A^-1 B.
// A step handles a panel of NB columns [j0, j0 + jb) in two launches:
//   k_gj_panel   one work-group per matrix, the panel in registers (row i in thread i mod NT, slot
//                i / NT): per column it picks the pivot (largest |re| + |im| at or below the diagonal,
//                the smallest row on ties), swaps the whole rows, scales the pivot row and eliminates
//                the column from every other row.  The panel columns then hold T[:, J], the columns of
//                the product of the step's elementary eliminations.
//   k_gj_update  C <- C + T[:, J] C_J on every column outside the panel, for the rows outside J, on
//                16x16x4 FP64 MFMA tiles of 64 x 64 (the rows J of T - I vanish outside J's rows).
// The pivot rows themselves, C_J <- T_JJ C_J, need the old C_J that every update tile reads, so they
// are finished at the start of the next step's panel kernel (or by k_gj_tail after the last step).
// A zero pivot sets info = its column + 1 (the first one) and the elimination runs on with IEEE
// infinities / NaN, as in the single-matrix form.
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

// The columns a step with panel [j0, j0 + jb) updates.
__device__ __forceinline__ bool gj_outside(int mode, int c, int n, int ld, int j0, int jb) {
    return mode == GJ_INVERT ? (c < n && (c < j0 || c >= j0 + jb)) : (c >= j0 + jb && c < ld);
}

// C_J <- T_JJ C_J for the pivot rows of the panel at P0 (every column that step updated).
template <int NT, int NB>
__device__ void gj_finish_rows(const GjArgs& g, double2* A, int n, int ld, int P0, double2 (*tjj)[NB]) {
    const int jbp = min(NB, n - P0);
    for (int e = threadIdx.x; e < NB * NB; e += NT) {
        const int i = e / NB, t = e % NB;
        tjj[i][t] = (i < jbp && t < jbp) ? A[int64_t(P0 + i) * ld + P0 + t] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int cend = g.mode == GJ_INVERT ? n : ld;
    for (int c = threadIdx.x; c < cend; c += NT) {
        if (!gj_outside(g.mode, c, n, ld, P0, jbp)) continue;
        double2 old[NB];
#pragma unroll
        for (int t = 0; t < NB; ++t)
            old[t] = t < jbp ? A[int64_t(P0 + t) * ld + c] : make_double2(0.0, 0.0);
        // one row of T_JJ at a time (its LDS reads stay inside the column loop)
#pragma unroll 1
        for (int i = 0; i < jbp; ++i) {
            double2 s = make_double2(0.0, 0.0);
#pragma unroll
            for (int t = 0; t < NB; ++t) {
                const double2 a = tjj[i][t];
                s.x += a.x * old[t].x - a.y * old[t].y;
                s.y += a.x * old[t].y + a.y * old[t].x;
            }
            A[int64_t(P0 + i) * ld + c] = s;
        }
    }
    __syncthreads();
}

template <int NT, int RPT, int NB>
__global__ __launch_bounds__(NT) void k_gj_panel(GjArgs g, int j0) {
    __shared__ double2 tjj[NB][NB];
    __shared__ double rv[NT / 64];
    __shared__ int ri[NT / 64];
    __shared__ double2 srow[2][NB];
    __shared__ double2 prow[NB];

    const int b = blockIdx.x;
    int n, ld;
    int64_t off;
    gj_item(g, b, n, ld, off);
    double2* A = g.A + off;
    if (j0 > 0 && j0 - NB < n) gj_finish_rows<NT, NB>(g, A, n, ld, j0 - NB, tjj);
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
                for (int c = tid; c < cend; c += NT) {
                    if (!gj_outside(g.mode, c, n, ld, j0, jb)) continue;
                    const double2 t = A[int64_t(j) * ld + c];
                    A[int64_t(j) * ld + c] = A[int64_t(p) * ld + c];
                    A[int64_t(p) * ld + c] = t;
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

template <int NB>
__global__ __launch_bounds__(256) void k_gj_update(GjArgs g, int j0, int tiles_m) {
    __shared__ double2 As[64][NB + 1];
    __shared__ double2 Bs[NB][64];

    const int b = blockIdx.y;
    int n, ld;
    int64_t off;
    gj_item(g, b, n, ld, off);
    if (j0 >= n) return;
    const int jb = min(NB, n - j0);
    const int row0 = (blockIdx.x % tiles_m) * 64, col0 = (blockIdx.x / tiles_m) * 64;
    const int ncols = g.mode == GJ_INVERT ? n - jb : ld - j0 - jb;
    if (row0 >= n || col0 >= ncols) return;
    double2* A = g.A + off;
    const bool inv_mode = g.mode == GJ_INVERT;
    auto colmap = [&](int cc) { return inv_mode ? (cc < j0 ? cc : cc + jb) : j0 + jb + cc; };
    const int tid = threadIdx.x;

    // T[rows, J] (zero on the pivot rows, which the next panel kernel finishes) and C_J[:, cols]
    for (int e = tid; e < 64 * NB; e += 256) {
        const int r = e / NB, t = e % NB, i = row0 + r;
        double2 a = make_double2(0.0, 0.0);
        if (i < n && t < jb && (i < j0 || i >= j0 + jb)) a = A[int64_t(i) * ld + j0 + t];
        As[r][t] = a;
    }
    for (int e = tid; e < NB * 64; e += 256) {
        const int t = e / 64, cc = col0 + (e % 64);
        double2 v = make_double2(0.0, 0.0);
        if (t < jb && cc < ncols) v = A[int64_t(j0 + t) * ld + colmap(cc)];
        Bs[t][e % 64] = v;
    }
    __syncthreads();

    // each wave a 32 x 32 quarter of the tile: 2 x 2 blocks of 16 x 16, real and imaginary parts
    const int lane = tid & 63, w = tid >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    dbl4 cre[2][2], cim[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            cre[bi][bj] = dbl4{0.0, 0.0, 0.0, 0.0};
            cim[bi][bj] = dbl4{0.0, 0.0, 0.0, 0.0};
        }
    const int r16 = lane & 15, k4 = lane >> 4;
#pragma unroll
    for (int k0 = 0; k0 < NB; k0 += 4) {
        double2 a[2], v[2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) a[bi] = As[wr + bi * 16 + r16][k0 + k4];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) v[bj] = Bs[k0 + k4][wc + bj * 16 + r16];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                cre[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi].x, v[bj].x, cre[bi][bj], 0, 0, 0);
                cre[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[bi].y, v[bj].y, cre[bi][bj], 0, 0, 0);
                cim[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi].x, v[bj].y, cim[bi][bj], 0, 0, 0);
                cim[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi].y, v[bj].x, cim[bi][bj], 0, 0, 0);
            }
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
                if (i < n && (i < j0 || i >= j0 + jb) && cc < ncols) {
                    double2* p = &A[int64_t(i) * ld + colmap(cc)];
                    double2 y = *p;
                    y.x += cre[bi][bj][r4];
                    y.y += cim[bi][bj][r4];
                    *p = y;
                }
            }
}

// the pivot rows of the last panel of every matrix whose last panel started at j0 - NB
template <int NT, int NB>
__global__ __launch_bounds__(NT) void k_gj_tail(GjArgs g, int j0) {
    __shared__ double2 tjj[NB][NB];
    int n, ld;
    int64_t off;
    gj_item(g, blockIdx.x, n, ld, off);
    if (j0 - NB >= 0 && j0 - NB < n) gj_finish_rows<NT, NB>(g, g.A + off, n, ld, j0 - NB, tjj);
}

__global__ void k_gj_zero(int* p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

template <int NT, int RPT, int NB>
void gj_steps(const GjArgs& g, int batch, int nmax, int cmax, hipStream_t s) {
    const int tiles_m = (nmax + 63) / 64, tiles_n = (cmax + 63) / 64;
    int j0 = 0;
    for (; j0 < nmax; j0 += NB) {
        MSGW_LAUNCH((k_gj_panel<NT, RPT, NB>), dim3(batch), dim3(NT), 0, s, g, j0);
        MSGW_LAUNCH((k_gj_update<NB>), dim3(tiles_m * tiles_n, batch), dim3(256), 0, s, g, j0, tiles_m);
    }
    MSGW_LAUNCH((k_gj_tail<NT, NB>), dim3(batch), dim3(NT), 0, s, g, j0);
}

}  // namespace

void gj_run(const GjArgs& g, int batch, int nmax, int ldmax, hipStream_t s) {
    if (batch <= 0 || nmax <= 0) return;
    if (nmax > kGjMaxN) throw Error(MSGW_ENOTSUP, "Gauss-Jordan: order above 4096");
    if (batch > 65535) throw Error(MSGW_ENOTSUP, "Gauss-Jordan: more than 65535 matrices in one call");
    MSGW_LAUNCH(k_gj_zero, dim3((batch + 255) / 256), dim3(256), 0, s, g.info, batch);
    const int cmax = g.mode == GJ_INVERT ? nmax : ldmax;
    // the panel stays in registers: RPT rows of NB complex columns per thread
    if (nmax <= 1024)
        gj_steps<512, 2, 16>(g, batch, nmax, cmax, s);
    else if (nmax <= 2048)
        gj_steps<512, 4, 8>(g, batch, nmax, cmax, s);
    else
        gj_steps<512, 8, 4>(g, batch, nmax, cmax, s);
    MSGW_HIP(hipGetLastError());
}

}  // namespace msgw
