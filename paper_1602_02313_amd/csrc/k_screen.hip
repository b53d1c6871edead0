// Screened interaction on the bosonic Matsubara axis, FP64.
//
// For each (q, nu):  A = 1 - v^1/2 P v^1/2 is inverted in place, then W~ = v^1/2 (A^-1 - 1) v^1/2 and
// R = W~ - v P v.  This is the W~ Dyson equation W~ = v P v + v P W~ after the tau convolution becomes a
// product on i nu.
//
//   k_screen_build   A = 1 - v^1/2 P v^1/2 into the W~ buffer (16 rows per work-group);
//   hp_run           the Hermitian matrices by the blocked sweep (k_hscreen.hip), which marks them done;
//   k_screen_build   again for the matrices whose sweep met a non-positive pivot;
//   gj_run           A <- A^-1 with permuted columns for the rest (k_gj.hip, partial row pivoting);
//   k_screen_finish  undoes their column permutation (the pivot swaps in reverse), forms W~ and R and
//                    raises the singular flag of a matrix with a zero pivot;
//   hp_finish        W~ and R of the swept matrices.
#include "internal.h"

namespace msgw {
namespace {

constexpr int SROWS = 16;  // rows per work-group of the build and finish kernels

__global__ __launch_bounds__(256) void k_screen_build(GjArgs g, const double2* __restrict__ Piw,
                                                      const double* __restrict__ v, const int64_t* vpre) {
    const int b = blockIdx.y;
    int n, ld;
    int64_t off;
    gj_item(g, b, n, ld, off);
    const int r0 = blockIdx.x * SROWS;
    if (r0 >= n) return;
    const int q = g.q0 + b / g.niw_b;
    const double* vq = v + (vpre[q] - vpre[g.q0]);
    const int rows = min(SROWS, n - r0);
    for (int e = threadIdx.x; e < rows * n; e += 256) {
        const int i = r0 + e / n, j = e % n;
        const double2 p = Piw[off + int64_t(i) * n + j];
        const double f = -sqrt(vq[i]) * sqrt(vq[j]);
        double2 a = make_double2(f * p.x, f * p.y);
        if (i == j) a.x += 1.0;
        g.A[off + int64_t(i) * n + j] = a;
    }
}

__global__ __launch_bounds__(256) void k_screen_finish(GjArgs g, const double2* __restrict__ Piw,
                                                       const double* __restrict__ v, const int64_t* vpre,
                                                       double2* __restrict__ R, int* __restrict__ flags) {
    __shared__ int idx[MSGW_MAX_NI];
    __shared__ double2 buf[MSGW_MAX_NI];
    const int b = blockIdx.y;
    int n, ld;
    int64_t off;
    gj_item(g, b, n, ld, off);
    const int r0 = blockIdx.x * SROWS;
    if (r0 >= n) return;
    const int tid = threadIdx.x;
    const int q = g.q0 + b / g.niw_b;
    const double* vq = v + (vpre[q] - vpre[g.q0]);
    const int* perm = g.perm + int64_t(b) * g.pmax;
    // column c of A^-1 sits at column idx[c]: the pivot swaps applied in reverse order
    if (tid == 0) {
        for (int c = 0; c < n; ++c) idx[c] = c;
        for (int j = n - 1; j >= 0; --j) {
            const int t = idx[j];
            idx[j] = idx[perm[j]];
            idx[perm[j]] = t;
        }
        if (r0 == 0 && flags && g.info[b]) atomicOr(flags, MSGW_FLAG_SINGULAR);
    }
    double2* A = g.A + off;
    const double2* P = Piw + off;
    double2* Rq = R ? R + off : nullptr;
    const int rend = min(n, r0 + SROWS);
    for (int i = r0; i < rend; ++i) {
        __syncthreads();
        for (int c = tid; c < n; c += 256) buf[c] = A[int64_t(i) * n + c];
        __syncthreads();
        const double si = sqrt(vq[i]);
        for (int c = tid; c < n; c += 256) {
            double2 x = buf[idx[c]];
            if (c == i) x.x -= 1.0;
            const double f = si * sqrt(vq[c]);
            const double2 w = make_double2(f * x.x, f * x.y);
            A[int64_t(i) * n + c] = w;
            if (Rq) {
                const double vv = vq[i] * vq[c];
                const double2 p = P[int64_t(i) * n + c];
                Rq[int64_t(i) * n + c] = make_double2(w.x - vv * p.x, w.y - vv * p.y);
            }
        }
    }
}

}  // namespace

size_t screen_scratch_bytes(const Host& h, int nq) {
    const size_t perm = (sizeof(int) * size_t(nq) * h.niw_b * h.nimax + 255) / 256 * 256;
    return perm + hp_scratch_bytes(nq * h.niw_b, h.nimax);
}

void screen_validate(const Host& h, int q0, int nq) {
    int nmax = 0;
    for (int q = q0; q < q0 + nq; ++q) nmax = std::max(nmax, h.ni[q]);
    const int64_t batch = int64_t(nq) * h.niw_b;
    if (nmax > kGjMaxN) throw Error(MSGW_ENOTSUP, "screen: NI above 4096");
    if (batch > 65535)
        throw Error(MSGW_ENOTSUP, "screen: nq * niw_b above 65535 matrices in one call (split the q range)");
    // the 1-D grids of the two eliminations' updates hold at most 2^32 - 1 threads (the Gauss-Jordan's,
    // all 64 x 64 tiles of every matrix, is the larger)
    const double tiles = 8.0 * double((batch + 7) / 8) * ((nmax + 63) / 64) * ((nmax + 63) / 64);
    if (tiles * 256.0 > 4294967295.0)
        throw Error(MSGW_ENOTSUP, "screen: too many update tiles for one launch (split the q range)");
}

void launch_screen(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* P_iw,
                   const double* v, void* Wt_iw, void* R_iw, int* info, int* flags, int* perm) {
    int nmax = 0;
    for (int q = q0; q < q0 + nq; ++q) nmax = std::max(nmax, h.ni[q]);
    const int batch = nq * h.niw_b;
    GjArgs g;
    g.A = (double2*)Wt_iw;
    g.mode = GJ_INVERT;
    g.ni = d.ni;
    g.wpre = d.wpre;
    g.q0 = q0;
    g.niw_b = h.niw_b;
    g.perm = perm;
    g.pmax = h.nimax;
    g.info = info;
    const dim3 grid((nmax + SROWS - 1) / SROWS, batch);
    MSGW_LAUNCH(k_screen_build, grid, dim3(256), 0, s, g, (const double2*)P_iw, v, d.vpre);
    // the Hermitian matrices by the blocked sweep; the rest (and those whose sweep failed, rebuilt) by
    // the pivoting Gauss-Jordan
    char* hp = reinterpret_cast<char*>(perm) + (sizeof(int) * size_t(batch) * h.nimax + 255) / 256 * 256;
    const int *skip_gj = nullptr, *skip_rb = nullptr;
    hp_run(g, batch, nmax, h.nimax, hp, s, &skip_gj, &skip_rb);
    GjArgs grb = g;
    grb.skip = skip_rb;
    MSGW_LAUNCH(k_screen_build, grid, dim3(256), 0, s, grb, (const double2*)P_iw, v, d.vpre);
    GjArgs gg = g;
    gg.skip = skip_gj;
    gj_run(gg, batch, nmax, nmax, s);
    MSGW_LAUNCH(k_screen_finish, grid, dim3(256), 0, s, gg, (const double2*)P_iw, v, d.vpre, (double2*)R_iw,
                flags);
    hp_finish(g, batch, nmax, h.nimax, hp, (const double2*)P_iw, v, d.vpre, (double2*)R_iw, s);
    MSGW_HIP(hipGetLastError());
}

}  // namespace msgw
