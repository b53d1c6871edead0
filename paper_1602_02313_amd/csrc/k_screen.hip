// Screened interaction on the bosonic Matsubara axis, FP64.
//
// For each (q, nu):  A = 1 - v^1/2 P v^1/2 is inverted in place by blocked Gauss-Jordan with
// partial (row) pivoting, then W~ = v^1/2 (A^-1 - 1) v^1/2 and R = W~ - v P v.  This is the
// W~ Dyson equation W~ = v P v + v P W~ after the tau convolution becomes a product on i nu.
//
// One work-group of NT = 1024 threads owns one matrix (n <= 1024).  Panel of SB = 16 columns:
//   1. for each panel column j: pick the pivot row (max |re| + |im| over rows >= j), swap the
//      full rows, scale the pivot row and eliminate column j from every other row -- on the
//      panel columns only.  The panel then holds the columns J of T = E_last ... E_first.
//   2. every column c outside the panel (thread c) gets c <- T c = c + (T[:,J] - I[:,J]) c[J].
// At the end the in-place result is A^-1 with permuted columns; the swaps are undone in
// reverse order while writing W~ and R.
#include "internal.h"

namespace msgw {
namespace {

constexpr int RCH = 64;     // rows of the panel staged in LDS per chunk of the update
constexpr int UR = 3;       // rows of a column updated per group of loads

__device__ __forceinline__ double2 cmuls(double2 a, double2 b) { return cmul(a, b); }

__device__ __forceinline__ double2 crecip(double2 a) {
    double s = fmax(fabs(a.x), fabs(a.y));
    double ax = a.x / s, ay = a.y / s;
    double den = (ax * ax + ay * ay) * s;
    return make_double2(ax / den, -ay / den);
}

template <int NT, int SB>
__global__ __launch_bounds__(NT) void k_screen(Dev d, int q0, const double2* __restrict__ Piw,
                                               const double* __restrict__ v,
                                               double2* __restrict__ Wt, double2* __restrict__ R,
                                               int* __restrict__ info, int* __restrict__ flags) {
    __shared__ double sv[MSGW_MAX_NI];
    __shared__ int perm[MSGW_MAX_NI];
    __shared__ int idx[MSGW_MAX_NI];
    __shared__ double2 buf[MSGW_MAX_NI];        // pivot column multipliers / row buffer
    __shared__ double2 tch[RCH][SB];
    __shared__ double2 prow[SB];               // the scaled pivot row within the panel
    __shared__ double rv[NT / 64];
    __shared__ int ri[NT / 64];
    __shared__ int s_info;

    const int mi = blockIdx.x;
    const int q = q0 + mi / d.niw_b, nu = mi % d.niw_b;
    const int n = d.ni[q];
    const int tid = threadIdx.x;
    const int64_t off = (d.wpre[q] - d.wpre[q0]) + int64_t(nu) * n * n;
    double2* A = Wt + off;
    const double2* P = Piw + off;
    double2* Rq = R ? R + off : nullptr;
    const double* vq = v + (d.vpre[q] - d.vpre[q0]);

    for (int i = tid; i < n; i += NT) sv[i] = sqrt(vq[i]);
    if (tid == 0) s_info = 0;
    __syncthreads();
    for (int64_t e = tid; e < int64_t(n) * n; e += NT) {
        int i = int(e / n), j = int(e % n);
        double2 p = P[e];
        double f = -sv[i] * sv[j];
        double2 a = make_double2(f * p.x, f * p.y);
        if (i == j) a.x += 1.0;
        A[e] = a;
    }
    __syncthreads();

    for (int j0 = 0; j0 < n; j0 += SB) {
        const int jb = min(SB, n - j0);
        for (int jj = 0; jj < jb; ++jj) {
            const int j = j0 + jj;
            // ---- pivot search: max |re| + |im| in column j, rows >= j (smallest index on ties)
            double best = -1.0;
            int bi = n;
            for (int i = j + tid; i < n; i += NT) {
                double2 x = A[int64_t(i) * n + j];
                double m = fabs(x.x) + fabs(x.y);
                if (m > best) {
                    best = m;
                    bi = i;
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                double ob = __shfl_xor(best, o);
                int oi = __shfl_xor(bi, o);
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
            const int p = (bi < n) ? bi : j;  // all-NaN column: keep the row
            if (tid == 0) perm[j] = p;
            if (p != j)
                for (int c = tid; c < n; c += NT) {
                    double2 t = A[int64_t(j) * n + c];
                    A[int64_t(j) * n + c] = A[int64_t(p) * n + c];
                    A[int64_t(p) * n + c] = t;
                }
            __syncthreads();
            const double2 piv = A[int64_t(j) * n + j];
            if (tid == 0 && piv.x == 0.0 && piv.y == 0.0 && s_info == 0) s_info = j + 1;
            const double2 inv = crecip(piv);
            for (int i = tid; i < n; i += NT) buf[i] = A[int64_t(i) * n + j];
            __syncthreads();
            if (tid < jb) {
                const int c = j0 + tid;
                double2* a = &A[int64_t(j) * n + c];
                const double2 val = (c == j) ? inv : cmuls(*a, inv);
                *a = val;
                prow[tid] = val;
            }
            __syncthreads();
            // eliminate column j from the other rows of the panel: each thread loads its EB elements
            // together (one memory round trip), then updates them
            constexpr int EB = 8;
            for (int e0 = tid; e0 < n * jb; e0 += NT * EB) {
                double2 x[EB];
#pragma unroll
                for (int u = 0; u < EB; ++u) {
                    const int e = e0 + u * NT;
                    const int i = e / jb, c = j0 + e % jb;
                    x[u] = (e < n * jb && i != j && c != j) ? A[int64_t(i) * n + c] : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int u = 0; u < EB; ++u) {
                    const int e = e0 + u * NT;
                    const int i = e / jb, t = e % jb, c = j0 + t;
                    if (e >= n * jb || i == j) continue;
                    const double2 f = buf[i];
                    if (c == j) {
                        const double2 w = cmuls(f, inv);
                        A[int64_t(i) * n + c] = make_double2(-w.x, -w.y);
                    } else {
                        const double2 r = prow[t];
                        double2 y = x[u];
                        y.x -= f.x * r.x - f.y * r.y;
                        y.y -= f.x * r.y + f.y * r.x;
                        A[int64_t(i) * n + c] = y;
                    }
                }
            }
            __syncthreads();
        }
        // ---- update of the columns outside the panel: c <- c + (T[:,J] - I[:,J]) c[J]; NT / n threads
        // share a column, each taking every tpc-th group of UR rows
        const int tpc = NT / n, c = tid % n, sub = tid / n;
        const bool own = sub < tpc && (c < j0 || c >= j0 + jb);
        double2 cj[SB];
#pragma unroll
        for (int t = 0; t < SB; ++t)
            cj[t] = (own && t < jb) ? A[int64_t(j0 + t) * n + c] : make_double2(0.0, 0.0);
        for (int i0 = 0; i0 < n; i0 += RCH) {
            __syncthreads();
            for (int e = tid; e < RCH * SB; e += NT) {
                const int r = e / SB, t = e % SB;
                tch[r][t] = (i0 + r < n && t < jb) ? A[int64_t(i0 + r) * n + j0 + t]
                                                   : make_double2(0.0, 0.0);
            }
            __syncthreads();
            if (own) {
                const int rmax = min(RCH, n - i0);
                // UR rows at a time: their loads are in flight together
                for (int r0 = sub * UR; r0 < rmax; r0 += tpc * UR) {
                    double2 sr[UR];
#pragma unroll
                    for (int u = 0; u < UR; ++u) {
                        const int i = i0 + r0 + u;
                        sr[u] = (r0 + u >= rmax || (i >= j0 && i < j0 + jb)) ? make_double2(0.0, 0.0)
                                                                             : A[int64_t(i) * n + c];
                    }
#pragma unroll
                    for (int u = 0; u < UR; ++u) {
                        if (r0 + u >= rmax) break;
                        double2 s = sr[u];
#pragma unroll
                        for (int t = 0; t < SB; ++t) {
                            const double2 tv = tch[r0 + u][t];
                            s.x += tv.x * cj[t].x - tv.y * cj[t].y;
                            s.y += tv.x * cj[t].y + tv.y * cj[t].x;
                        }
                        A[int64_t(i0 + r0 + u) * n + c] = s;
                    }
                }
            }
        }
        __syncthreads();
    }

    // ---- undo the column permutation, form W~ and R
    if (tid == 0) {
        for (int c = 0; c < n; ++c) idx[c] = c;
        for (int j = n - 1; j >= 0; --j) {
            int t = idx[j];
            idx[j] = idx[perm[j]];
            idx[perm[j]] = t;
        }
    }
    __syncthreads();
    for (int i = 0; i < n; ++i) {
        for (int c = tid; c < n; c += NT) buf[c] = A[int64_t(i) * n + c];
        __syncthreads();
        for (int c = tid; c < n; c += NT) {
            double2 x = buf[idx[c]];
            if (c == i) x.x -= 1.0;
            const double f = sv[i] * sv[c];
            double2 w = make_double2(f * x.x, f * x.y);
            A[int64_t(i) * n + c] = w;
            if (Rq) {
                const double vv = vq[i] * vq[c];
                double2 p = P[int64_t(i) * n + c];
                Rq[int64_t(i) * n + c] = make_double2(w.x - vv * p.x, w.y - vv * p.y);
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        info[mi] = s_info;
        if (flags && s_info) atomicOr(flags, MSGW_FLAG_SINGULAR);
    }
}

}  // namespace

void launch_screen(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* P_iw,
                   const double* v, void* Wt_iw, void* R_iw, int* info, int* flags) {
    MSGW_LAUNCH((k_screen<1024, 16>), dim3(nq * h.niw_b), dim3(1024), 0, s, d, q0, (const double2*)P_iw, v,
                (double2*)Wt_iw, (double2*)R_iw, info, flags);
    MSGW_HIP(hipGetLastError());
}

}  // namespace msgw
