// Mixed-precision contractions on the CDNA4 matrix cores.
//
// Polarization (eq. irpol):  P_IJ(q,tau) = s sum_k sum_{nm} M^I_nm g_nm(tau) conj(M^J_nm),
//   g_nm(tau) = G_n(k,tau) G_m(k-q,beta-tau).
// Correlation self-energy (eq. sigc, diagonal): Y(tau) = W~(q,tau) M(q,k),
//   Sigma_n(k,tau) += s sum_m G_m(k-q,tau) Re sum_I conj(M^I_nm) Y^I_nm.
//
// Complex products use the interleaved real embedding: with K' = (K, re/im),
//   Re(x conj(y)) = [xr, xi].[yr, yi],  Im(x conj(y)) = [xi, -xr].[yr, yi]
//   Re(w m) = [wr, wi].[mr, -mi],       Im(w m) = [wr, wi].[mi, mr]
// so every complex contraction is two real MFMA chains sharing one operand.
//
// Precisions
//   FP32:   v_mfma_f32_16x16x4_f32, FP32 operands and accumulation.
//   BF16X3: each FP32 operand x is split into hi = bf16(x) and lo = bf16(x - hi) (round to nearest
//           even), and x.y ~ hi.hi + hi.lo + lo.hi on bf16 MFMA with FP32 accumulation; the dropped
//           lo.lo term is ~2^-16 relative.
//   F16X3:  the same split into f16 halves (11 significant bits, so the dropped lo.lo is ~2^-22
//           relative), with every operand scaled by a power of two that keeps it inside the f16 range
//           (M per q, the weights per (q, tau)); the scales are undone in FP64.
// The FP32 accumulators of the polarization are flushed into the FP64 output every FLUSH_STEPS
// K-steps, so an FP32 sum never runs over more than 4096 complex terms (the pair-space polarization:
// GZ_FLUSH terms).
//
// The split-precision defaults are the pair-space kernels (32x32x16 MFMA, operands staged through LDS
// by 8-wave work-groups; see their sections below): the polarization in its persistent form
// (k_polz_queue: one work-group per CU taking items from per-XCD queues that k_polz_qbuild lists on
// the device), the self-energy k_sigz.  The tile forms: polarization, one wave (64 lanes) per
// work-group owning a (16 WI) x (16 WJ) x T output tile and streaming its operands from global memory
// (reuse between waves served by L2); self-energy, one-wave variants of the same kind and a 4-wave
// variant (v7) that stages its operands through LDS and runs on v_mfma_f32_32x32x16_bf16.  To make the
// reuse happen, the static grids are ordered XCD-aware: the hardware deals consecutive work-group ids
// round-robin to the 8 XCDs, so id b is mapped to item b / 8 of the slice of XCD b % 8 -- each XCD
// walks a contiguous slice of the work -- and the work space (rows x columns) is cut into super-tiles
// of SR x SC items (about the number of waves resident on one XCD), so the waves running together on
// an XCD share SR row panels and SC column panels in its L2.  Where only part of the item space holds
// work (the upper triangle of the Hermitian polarization), the slices are cut so that every XCD gets
// the same number of working items, not the same number of indices.
#include "internal.h"

namespace msgw {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int PREC_FP32 = MSGW_FP32;
constexpr int PREC_BF16X3 = MSGW_BF16X3;
constexpr int PREC_F16X3 = MSGW_F16X3;
constexpr int NB_LDS = 256;       // band limit of the MFMA path (G slices staged in LDS)
constexpr int FLUSH_STEPS = 256;  // K-steps of 16 complex between FP64 flushes
constexpr int PAD = 64;           // W~ planes are zero-padded to a multiple of PAD

inline unsigned ceil_div(int64_t a, int64_t b) {
    const int64_t r = (a + b - 1) / b;
    if (r > int64_t(0xFFFFFFFFu)) throw Error(MSGW_ENOTSUP, "shape too large for one launch");
    return unsigned(r);
}
inline int round_up(int a, int b) { return (a + b - 1) / b * b; }

// ---- bf16 helpers -------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
    bf16x2 v = {(__bf16)a, (__bf16)b};  // v_cvt_pk_bf16_f32, round to nearest even
    return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ float bf_lo(uint32_t p) { return __uint_as_float(p << 16); }
// the same by one byte permute (bytes 1:0 of p to 3:2, zeros below): where the compiler would rewrite
// the shift of a fresh conversion into a second conversion of the low element
__device__ __forceinline__ float bf_lo_perm(uint32_t p) {
    return __uint_as_float(__builtin_amdgcn_perm(0u, p, 0x01000c0cu));
}
__device__ __forceinline__ float bf_hi(uint32_t p) { return __uint_as_float(p & 0xffff0000u); }
// split a complex pair (re, im) into packed hi and lo bf16 pairs
__device__ __forceinline__ void split2(float re, float im, uint32_t& h, uint32_t& l) {
    h = pk_bf16(re, im);
    l = pk_bf16(re - bf_lo(h), im - bf_hi(h));
}
// (re, im) -> (im, -re): rotate by 16 bits, flip the sign of the new high half
__device__ __forceinline__ uint32_t rot_neg(uint32_t p) {
    return __builtin_amdgcn_alignbit(p, p, 16) ^ 0x80000000u;
}
// (re, im) -> (-im, re): rotate by 16 bits, flip the sign of the new low half
__device__ __forceinline__ uint32_t rot_pos(uint32_t p) {
    return __builtin_amdgcn_alignbit(p, p, 16) ^ 0x00008000u;
}
// (re, im) -> (re, -im)
__device__ __forceinline__ uint32_t conj_pk(uint32_t p) { return p ^ 0x80000000u; }
// (re, im) -> (im, re)
__device__ __forceinline__ uint32_t swap_pk(uint32_t p) { return __builtin_amdgcn_alignbit(p, p, 16); }

// ---- f16 helpers (MSGW_F16X3) --------------------------------------------------------------------
__device__ __forceinline__ uint32_t pk_f16(float a, float b) {
    f16x2 v = {(_Float16)a, (_Float16)b};  // v_cvt_pk_f16_f32, round to nearest even
    return __builtin_bit_cast(uint32_t, v);
}
// hi = f16(a), lo = f16(a - hi) for both halves of a pair; a - hi is exact in FP32.  The packed hi is
// made opaque so that its halves are read from the register rather than converted a second time, and
// a - hi is written as fma(hi, m1, a) with an opaque m1 = -1, which becomes one v_fma_mix_f32 that reads
// the f16 half directly (four instructions per pair instead of six).
__device__ __forceinline__ void split_f16(float a, float b, uint32_t& h, uint32_t& l) {
    h = pk_f16(a, b);
    uint32_t hv = h;
    asm("" : "+v"(hv));
    float m1 = -1.f;
    asm("" : "+s"(m1));
    const f16x2 hh = __builtin_bit_cast(f16x2, hv);
    l = pk_f16(__builtin_fmaf(float(hh.x), m1, a), __builtin_fmaf(float(hh.y), m1, b));
}
// the split of the pair (a, b) into packed hi and lo halves in the element type of precision PR
template <int PR>
__device__ __forceinline__ void split_pair(float a, float b, uint32_t& h, uint32_t& l) {
    if constexpr (PR == PREC_F16X3) {
        split_f16(a, b, h, l);
    } else {
        h = pk_bf16(a, b);
        l = pk_bf16(a - bf_lo(h), b - bf_hi(h));
    }
}

// Operand scales of MSGW_F16X3.  f16 holds 11 significant bits but overflows at 65504 (~2^16) and
// loses relative precision below 2^-14, so each operand is scaled by a power of two that puts its
// largest element in [2^13, 2^14]: M by 2^e_m per q (the pair products Z = M^I conj(M^J) then have
// |Re Z|, |Im Z| <= max |M|^2 2^(2 e_m) <= 2^14), the real weights per (q, tau) column.  Elements
// 2^-38 times the largest still keep f16 subnormal precision; the scales are undone in FP64.
__device__ __forceinline__ int exp_above(double mx) {  // x with mx < 2^x, for mx > 0
    int x;
    frexp(mx, &x);
    return x;
}
__device__ __forceinline__ int f16_exp_m(unsigned long long bits) {  // bits of max |M|^2
    const double mx = __longlong_as_double(static_cast<long long>(bits));
    if (!(mx > 0.0)) return 0;
    const int t = 14 - exp_above(mx);           // 2 e_m <= t
    const int e = t >= 0 ? t / 2 : -((1 - t) / 2);  // floor(t / 2)
    return min(max(e, -100), 100);              // 2^e_m stays a normal float
}
__device__ __forceinline__ int f16_exp_w(unsigned long long bits) {  // bits of max |Re|, |Im| of W~
    const double mx = __longlong_as_double(static_cast<long long>(bits));
    // the weights c H_IJ = (c / 2)(W_IJ + conj W_JI), c <= 2, are bounded by 2 mx
    return mx > 0.0 ? 14 - exp_above(2.0 * mx) : 0;
}

__device__ __forceinline__ floatx4 mfma_bf16(u32x4 a, u32x4 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma_f32(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Complex elements a lane holds per 16-element K step:
//   BF16X3: K = 4*(lane/16) + e, e < 4 (the 8 consecutive bf16 of the 16x16x32 operand)
//   FP32:   K = 2*e + (lane/16)/2, e < 8, component (lane/16)%2 (one 16x16x4 slice per e)
template <int PREC>
struct Lay {
    static constexpr int NE = PREC == PREC_BF16X3 ? 4 : 8;
    __device__ static int koff(int g4, int e) { return PREC == PREC_BF16X3 ? 4 * g4 + e : 2 * e + (g4 >> 1); }
};

// ---- XCD-aware ordering ---------------------------------------------------------------------------
struct Order {
    int R, C;      // work rows and columns per q
    int SR, SC;    // super-tile
    int nSC;       // super-tiles per row of super-tiles
    int per_q;     // padded items per q
    int total;     // nq * per_q
    int off, n;    // items [off, off + n) belong to this launch
    int xs[9];     // XCD x takes the launch's items [xs[x], xs[x + 1]) (offsets from off)
};

// item counts of an order; the work-items of one call must be countable in an int
inline void order_sizes(Order& o, int nq) {
    const int64_t per = int64_t((o.R + o.SR - 1) / o.SR) * o.nSC * o.SR * o.SC;
    if (per * nq >= (int64_t(1) << 31)) throw Error(MSGW_ENOTSUP, "too many work items in one call");
    o.per_q = int(per);
    o.total = int(per * nq);
    o.off = 0;
    o.n = o.total;
}

// window: work items resident at once on one XCD (waves or work-groups); window <= 0 gives plain
// row-major order (each row of C items consecutive)
Order make_order(int R, int C, int nq, int window = 128) {
    Order o;
    o.R = R;
    o.C = C;
    if (window <= 0) {
        o.SC = C;
        o.SR = 1;
    } else {
        o.SC = C <= 32 ? std::min(C, window) : std::min(16, window);
        o.SR = std::max(1, window / o.SC);
    }
    o.nSC = (C + o.SC - 1) / o.SC;
    order_sizes(o, nq);
    return o;
}

// explicit super-tile of SR x SC items (rows x columns)
Order make_order_st(int R, int C, int nq, int SR, int SC) {
    Order o;
    o.R = R;
    o.C = C;
    o.SR = std::max(1, std::min(SR, R));
    o.SC = std::max(1, std::min(SC, C));
    o.nSC = (C + o.SC - 1) / o.SC;
    order_sizes(o, nq);
    return o;
}

// the item at index w of an order (q relative to the call, row, column; r, c may lie in the padding)
inline void order_item(const Order& o, int w, int& qrel, int& r, int& c) {
    qrel = w / o.per_q;
    w -= qrel * o.per_q;
    const int sts = o.SR * o.SC;
    const int st = w / sts, in = w - st * sts;
    const int sr = st / o.nSC, sc = st - sr * o.nSC;
    r = sr * o.SR + in / o.SC;
    c = sc * o.SC + in % o.SC;
}

// Working items among [w0, w1) of an order whose row r of q holds work in the columns [lo, hi) that
// rows(qrel, r, lo, hi) returns.  Whole super-tiles are counted row by row, partial ones item by item.
template <class RR>
int64_t order_count(const Order& o, int64_t w0, int64_t w1, RR&& rows) {
    const int sts = o.SR * o.SC;
    int64_t n = 0;
    int64_t w = w0;
    while (w < w1) {
        const int64_t st0 = w / sts * sts;
        if (w == st0 && st0 + sts <= w1) {  // a whole super-tile
            int qrel, r, c;
            order_item(o, int(w), qrel, r, c);
            for (int rr = r; rr < std::min(r + o.SR, o.R); ++rr) {
                int lo, hi;
                rows(qrel, rr, lo, hi);
                lo = std::max(lo, c);
                hi = std::min({hi, c + o.SC, o.C});
                n += std::max(0, hi - lo);
            }
            w += sts;
        } else {
            int qrel, r, c;
            order_item(o, int(w), qrel, r, c);
            if (r < o.R && c < o.C) {
                int lo, hi;
                rows(qrel, r, lo, hi);
                n += (c >= lo && c < hi) ? 1 : 0;
            }
            ++w;
        }
    }
    return n;
}

// launch(grid, order) once per slice of at most 2^32 - 1 work-items, the most one grid dimension
// holds.  Each XCD takes a contiguous part of the slice: of equal length, or, given rows (see
// order_count), holding equal numbers of working items; the grid is 8 times the longest part.
template <class F, class RR = std::nullptr_t>
void launch_order(Order o, unsigned threads, F&& launch, RR&& rows = nullptr) {
    const int64_t cap = (int64_t(0xFFFFFFFFu) / threads) & ~int64_t(7);
    const int total = o.total;
    for (int64_t s0 = 0; s0 < total; s0 += cap) {
        o.off = int(s0);
        o.n = int(std::min<int64_t>(cap, total - s0));
        const int per = (o.n + 7) / 8;
        for (int x = 0; x <= 8; ++x) o.xs[x] = std::min(x * per, o.n);
        if constexpr (!std::is_same_v<std::decay_t<RR>, std::nullptr_t>) {
            // cut where the running count of working items reaches x/8 of them
            const int64_t nw = order_count(o, o.off, int64_t(o.off) + o.n, rows);
            int64_t w = o.off, seen = 0;
            const int sts = o.SR * o.SC;
            for (int x = 1; x < 8; ++x) {
                const int64_t want = nw * x / 8;
                while (seen < want) {  // whole super-tiles while they fit, then single items
                    const int64_t st_end = std::min<int64_t>((w / sts + 1) * sts, int64_t(o.off) + o.n);
                    const int64_t m = order_count(o, w, st_end, rows);
                    if (seen + m <= want && w % sts == 0) {
                        seen += m;
                        w = st_end;
                    } else {
                        seen += order_count(o, w, w + 1, rows);
                        ++w;
                    }
                }
                o.xs[x] = int(w - o.off);
            }
            o.xs[8] = o.n;
        }
        int longest = 0;
        for (int x = 0; x < 8; ++x) longest = std::max(longest, o.xs[x + 1] - o.xs[x]);
        launch(dim3(unsigned(8 * std::max(longest, 1))), o);
        MSGW_HIP(hipGetLastError());
    }
}

// the hardware deals work-group ids round-robin to the 8 XCDs: XCD b % 8 takes item xs[b % 8] + b / 8
// of its part; returns false past the part and for padding items
__device__ __forceinline__ bool work_item(const Order& o, int& qrel, int& r, int& c) {
    const int x = int(blockIdx.x & 7);
    int w = o.xs[x] + int(blockIdx.x >> 3);
    if (w >= o.xs[x + 1]) return false;
    w += o.off;
    qrel = w / o.per_q;
    w -= qrel * o.per_q;
    const int sts = o.SR * o.SC;
    const int st = w / sts, in = w - st * sts;
    const int sr = st / o.nSC, sc = st - sr * o.nSC;
    r = sr * o.SR + in / o.SC;
    c = sc * o.SC + in % o.SC;
    return r < o.R && c < o.C;
}

// =================================================================================================
// polarization
// =================================================================================================
template <int WI, int WJ, int T, int PREC, bool PF>
__global__ __launch_bounds__(64) void k_pol(Dev d, int q0, const float2* __restrict__ M,
                                            const double* __restrict__ G,
                                            double2* __restrict__ P, Order od, int ntI) {
    using LY = Lay<PREC>;
    constexpr int NE = LY::NE;
    __shared__ float Ga[NB_LDS * T];
    __shared__ float Gb[NB_LDS * T];
    int qrel, r, c;
    if (!work_item(od, qrel, r, c)) return;
    const int lane = threadIdx.x, r16 = lane & 15, g4 = lane >> 4;
    const int q = q0 + qrel;
    const int nk = d.nk, ntau = d.ntau, nbmax = d.nbmax;
    const int NI = d.ni[q];
    const int tg = r / ntI, ti = r - tg * ntI, tj = c;
    const int i0 = ti * 16 * WI, j0 = tj * 16 * WJ, t0 = tg * T;
    if (i0 >= NI || j0 >= NI || j0 + 16 * WJ <= i0) return;  // below the diagonal: mirrored later

    floatx4 acc[WI][WJ][T][2];
#pragma unroll
    for (int a = 0; a < WI; ++a)
#pragma unroll
        for (int b = 0; b < WJ; ++b)
#pragma unroll
            for (int t = 0; t < T; ++t) acc[a][b][t][0] = acc[a][b][t][1] = floatx4{0, 0, 0, 0};

    const float2* Mq = M + (d.mpre[q] - d.mpre[q0]);
    double2* Pq = P + (d.ppre[q] - d.ppre[q0]);
    const double sc = d.scale;
    bool first = true;
    int since = 0;

    auto flush = [&]() {
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int it = t0 + t;
#pragma unroll
            for (int a = 0; a < WI; ++a)
#pragma unroll
                for (int b = 0; b < WJ; ++b) {
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const int I = i0 + 16 * a + 4 * g4 + rr, J = j0 + 16 * b + r16;
                        if (it < ntau && I < NI && J < NI) {
                            double2* p = &Pq[int64_t(it) * NI * NI + int64_t(I) * NI + J];
                            double re = sc * double(acc[a][b][t][0][rr]);
                            double im = sc * double(acc[a][b][t][1][rr]);
                            if (!first) {
                                double2 o = *p;
                                re += o.x;
                                im += o.y;
                            }
                            *p = make_double2(re, im);
                        }
                    }
                    acc[a][b][t][0] = acc[a][b][t][1] = floatx4{0, 0, 0, 0};
                }
        }
        first = false;
        since = 0;
    };

    // rows used by this lane (clamped into range; out-of-range rows are zeroed by `keep`)
    int rowI[WI], rowJ[WJ];
    float keepI[WI], keepJ[WJ];
#pragma unroll
    for (int a = 0; a < WI; ++a) {
        const int I = i0 + 16 * a + r16;
        rowI[a] = min(I, NI - 1);
        keepI[a] = I < NI ? 1.f : 0.f;
    }
#pragma unroll
    for (int b = 0; b < WJ; ++b) {
        const int J = j0 + 16 * b + r16;
        rowJ[b] = min(J, NI - 1);
        keepJ[b] = J < NI ? 1.f : 0.f;
    }

    for (int k = 0; k < nk; ++k) {
        const int kq = d.kmq[q * nk + k];
        const int nn = d.nb[k], nm = d.nb[kq];
        const int Kk = nn * nm;
        const float2* A = Mq + d.moff[q * nk + k];
        // 16-byte vector loads of 4 consecutive complex values when every row start is aligned
        const bool vec = PREC == PREC_BF16X3 && (Kk & 3) == 0 &&
                         (reinterpret_cast<uintptr_t>(A) & 31) == 0;
        __syncthreads();
        for (int e = lane; e < nn * T; e += 64) {
            const int n = e / T, t = e - n * T;
            const int it = min(t0 + t, ntau - 1);
            Ga[e] = float(G[(int64_t(k) * nbmax + n) * ntau + it]);
        }
        for (int e = lane; e < nm * T; e += 64) {
            const int m = e / T, t = e - m * T;
            const int it = min(t0 + t, ntau - 1);
            Gb[e] = float(G[(int64_t(kq) * nbmax + m) * ntau + (ntau - 1 - it)]);
        }
        __syncthreads();
        int n0 = 0, m0 = 0;  // (n, m) of the first K of the current step
        const int nsteps = (Kk + 15) / 16;
        // raw FP32 operands of step s: rows I of this lane (xa) and rows J (yb)
        auto load_raw = [&](int s, float2 (&xa)[WI][NE], float2 (&yb)[WJ][NE]) {
            const int kb = s * 16;
            if (vec && kb + 16 <= Kk) {
#pragma unroll
                for (int a = 0; a < WI; ++a) {
                    const float4* p = reinterpret_cast<const float4*>(A + int64_t(rowI[a]) * Kk + kb + 4 * g4);
                    const float4 u = p[0], v = p[1];
                    xa[a][0] = make_float2(keepI[a] * u.x, keepI[a] * u.y);
                    xa[a][1] = make_float2(keepI[a] * u.z, keepI[a] * u.w);
                    xa[a][2] = make_float2(keepI[a] * v.x, keepI[a] * v.y);
                    xa[a][3] = make_float2(keepI[a] * v.z, keepI[a] * v.w);
                }
#pragma unroll
                for (int b = 0; b < WJ; ++b) {
                    const float4* p = reinterpret_cast<const float4*>(A + int64_t(rowJ[b]) * Kk + kb + 4 * g4);
                    const float4 u = p[0], v = p[1];
                    yb[b][0] = make_float2(keepJ[b] * u.x, keepJ[b] * u.y);
                    yb[b][1] = make_float2(keepJ[b] * u.z, keepJ[b] * u.w);
                    yb[b][2] = make_float2(keepJ[b] * v.x, keepJ[b] * v.y);
                    yb[b][3] = make_float2(keepJ[b] * v.z, keepJ[b] * v.w);
                }
            } else {
#pragma unroll
                for (int a = 0; a < WI; ++a)
#pragma unroll
                    for (int e = 0; e < NE; ++e)
                        xa[a][e] = (kb + LY::koff(g4, e) < Kk && keepI[a] != 0.f)
                                       ? A[int64_t(rowI[a]) * Kk + kb + LY::koff(g4, e)]
                                       : make_float2(0.f, 0.f);
#pragma unroll
                for (int b = 0; b < WJ; ++b)
#pragma unroll
                    for (int e = 0; e < NE; ++e)
                        yb[b][e] = (kb + LY::koff(g4, e) < Kk && keepJ[b] != 0.f)
                                       ? A[int64_t(rowJ[b]) * Kk + kb + LY::koff(g4, e)]
                                       : make_float2(0.f, 0.f);
            }
        };
        float2 xa[WI][NE], yb[WJ][NE];
        if (PF) load_raw(0, xa, yb);
        for (int s = 0; s < nsteps; ++s) {
            // PF: the next step's loads are issued before this step's arithmetic (register
            // double-buffering), so their latency overlaps the split and the MFMAs
            float2 xn[WI][NE], yn[WJ][NE];
            if (PF) {
                if (s + 1 < nsteps) load_raw(s + 1, xn, yn);
            } else {
                load_raw(s, xa, yb);
            }
            int gi[NE];   // n index * T into Ga
            int gj[NE];   // m index * T into Gb
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const int ko = LY::koff(g4, e);
                int mm = m0 + ko, nx = n0;
                while (mm >= nm) {
                    mm -= nm;
                    ++nx;
                }
                gi[e] = min(nx, nn - 1) * T;
                gj[e] = mm * T;
            }
            if constexpr (PREC == PREC_BF16X3) {
                u32x4 xh[WI], xl[WI], xh2[WI], xl2[WI];
#pragma unroll
                for (int a = 0; a < WI; ++a)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        uint32_t h, l;
                        split2(xa[a][e].x, xa[a][e].y, h, l);
                        xh[a][e] = h;
                        xl[a][e] = l;
                        xh2[a][e] = rot_neg(h);
                        xl2[a][e] = rot_neg(l);
                    }
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    float g[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) g[e] = Ga[gi[e] + t] * Gb[gj[e] + t];
#pragma unroll
                    for (int b = 0; b < WJ; ++b) {
                        u32x4 yh, yl;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            uint32_t h, l;
                            split2(g[e] * yb[b][e].x, g[e] * yb[b][e].y, h, l);
                            yh[e] = h;
                            yl[e] = l;
                        }
#pragma unroll
                        for (int a = 0; a < WI; ++a) {
                            acc[a][b][t][0] = mfma_bf16(xh[a], yh, acc[a][b][t][0]);
                            acc[a][b][t][1] = mfma_bf16(xh2[a], yh, acc[a][b][t][1]);
                        }
#pragma unroll
                        for (int a = 0; a < WI; ++a) {
                            acc[a][b][t][0] = mfma_bf16(xh[a], yl, acc[a][b][t][0]);
                            acc[a][b][t][1] = mfma_bf16(xh2[a], yl, acc[a][b][t][1]);
                        }
#pragma unroll
                        for (int a = 0; a < WI; ++a) {
                            acc[a][b][t][0] = mfma_bf16(xl[a], yh, acc[a][b][t][0]);
                            acc[a][b][t][1] = mfma_bf16(xl2[a], yh, acc[a][b][t][1]);
                        }
                    }
                }
            } else {
                const bool imc = g4 & 1;  // this lane holds the imaginary component
#pragma unroll
                for (int t = 0; t < T; ++t) {
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const float g = Ga[gi[e] + t] * Gb[gj[e] + t];
#pragma unroll
                        for (int b = 0; b < WJ; ++b) {
                            const float y = g * (imc ? yb[b][e].y : yb[b][e].x);
#pragma unroll
                            for (int a = 0; a < WI; ++a) {
                                const float x1 = imc ? xa[a][e].y : xa[a][e].x;
                                const float x2 = imc ? -xa[a][e].x : xa[a][e].y;
                                acc[a][b][t][0] = mfma_f32(x1, y, acc[a][b][t][0]);
                                acc[a][b][t][1] = mfma_f32(x2, y, acc[a][b][t][1]);
                            }
                        }
                    }
                }
            }
            if (PF) {
#pragma unroll
                for (int a = 0; a < WI; ++a)
#pragma unroll
                    for (int e = 0; e < NE; ++e) xa[a][e] = xn[a][e];
#pragma unroll
                for (int b = 0; b < WJ; ++b)
#pragma unroll
                    for (int e = 0; e < NE; ++e) yb[b][e] = yn[b][e];
            }
            m0 += 16;
            while (m0 >= nm) {
                m0 -= nm;
                ++n0;
            }
            if (++since == FLUSH_STEPS) flush();
        }
    }
    if (since > 0 || first) flush();
}

// =================================================================================================
// self-energy
// =================================================================================================
// W~(q,tau) converted once per call into zero-padded planes [ntau][NIp][NIp], NIp = NI rounded up
// to PAD: FP32 -> one complex64 plane; BF16X3 -> hi and lo planes of packed (re, im) bf16 pairs.
// q blocks are packed over the call's q range (wq[q] = offset in elements of each plane).
//
// The diagonal self-energy needs only Re sum_IJ conj(a_I) W_IJ a_J for the columns a of M.  The
// anti-Hermitian part of W contributes a purely imaginary amount to that sum, and the Hermitian part
// H = (W + W^H) / 2 splits into its diagonal and two mirrored triangles, so
//     Re sum_IJ conj(a_I) W_IJ a_J = 2 Re sum_{I <= J} conj(a_I) U_IJ a_J,
// with U_IJ = H_IJ above the diagonal, H_II / 2 on it and 0 below.  The planes hold U; the kernels
// start each row tile's reduction at its diagonal and double the result.  This holds for any W~,
// Hermitian or not.
constexpr int CW_TILE = 32;
__global__ __launch_bounds__(256) void k_convert_w(const double2* __restrict__ W, int NI, int NIp,
                                                   int prec, float2* __restrict__ w32,
                                                   uint32_t* __restrict__ whi,
                                                   uint32_t* __restrict__ wlo) {
    __shared__ double2 tt[CW_TILE][CW_TILE + 1];  // W^T tile: tt[j][i] = W[J0 + i][I0 + j]
    const int nt = NIp / CW_TILE;
    const int bi = blockIdx.x / nt, bj = blockIdx.x - bi * nt, it = blockIdx.y;
    const int I0 = bi * CW_TILE, J0 = bj * CW_TILE;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const double2* Wt = W + int64_t(it) * NI * NI;
    const bool upper = bj >= bi;
    if (upper) {
        for (int r = ty; r < CW_TILE; r += 8) {
            const int I = J0 + r, J = I0 + tx;  // coalesced read of the mirrored tile
            tt[tx][r] = (I < NI && J < NI) ? Wt[int64_t(I) * NI + J] : make_double2(0.0, 0.0);
        }
    }
    __syncthreads();
    for (int r = ty; r < CW_TILE; r += 8) {
        const int I = I0 + r, J = J0 + tx;
        double re = 0.0, im = 0.0;
        if (upper && I < NI && J < NI && J >= I) {
            const double2 w = Wt[int64_t(I) * NI + J];
            const double2 m = tt[r][tx];  // W[J][I]
            re = 0.5 * (w.x + m.x);
            im = 0.5 * (w.y - m.y);
            if (J == I) {
                re *= 0.5;
                im = 0.0;
            }
        }
        const int64_t o = (int64_t(it) * NIp + I) * NIp + J;
        if (prec == PREC_FP32) {
            w32[o] = make_float2(float(re), float(im));
        } else {
            uint32_t h, l;
            split2(float(re), float(im), h, l);
            whi[o] = h;
            wlo[o] = l;
        }
    }
}

// Polarization is Hermitian in (I, J): the contraction kernels skip tiles that lie wholly below the
// diagonal, and this kernel then sets every entry below the diagonal to the conjugate of its mirror.
__global__ __launch_bounds__(256) void k_herm_fill(double2* __restrict__ P, int NI) {
    __shared__ double2 tt[CW_TILE][CW_TILE + 1];
    const int nt = (NI + CW_TILE - 1) / CW_TILE;
    const int bi = blockIdx.x / nt, bj = blockIdx.x - bi * nt;  // target tile: rows bi, cols bj
    if (bj > bi) return;
    const int I0 = bi * CW_TILE, J0 = bj * CW_TILE;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    double2* Pt = P + int64_t(blockIdx.y) * NI * NI;
    for (int r = ty; r < CW_TILE; r += 8) {
        const int I = J0 + r, J = I0 + tx;  // source: the mirrored tile (rows J0.., cols I0..)
        if (I < NI && J < NI) tt[tx][r] = Pt[int64_t(I) * NI + J];
    }
    __syncthreads();
    for (int r = ty; r < CW_TILE; r += 8) {
        const int I = I0 + r, J = J0 + tx;
        if (I < NI && J < I) {
            const double2 v = tt[r][tx];
            Pt[int64_t(I) * NI + J] = make_double2(v.x, -v.y);
        }
    }
}

template <int WI, int WJ, int T, int PREC>
__global__ __launch_bounds__(64) void k_sig(Dev d, int q0, const float2* __restrict__ M,
                                            const double* __restrict__ G,
                                            const char* __restrict__ wsc, int64_t plane,
                                            double* __restrict__ Sig, Order od, int ntI, int ntC) {
    using LY = Lay<PREC>;
    constexpr int NE = LY::NE;
    int qrel, r, c;
    if (!work_item(od, qrel, r, c)) return;
    const int lane = threadIdx.x, r16 = lane & 15, g4 = lane >> 4;
    const int nk = d.nk, ntau = d.ntau, nbmax = d.nbmax;
    const int q = q0 + qrel;
    const int tg = r / ntI, ti = r - tg * ntI;
    const int k = c / ntC, tc = c - k * ntC;
    const int kq = d.kmq[q * nk + k];
    const int nm = d.nb[kq], NI = d.ni[q];
    const int Kk = d.nb[k] * nm;
    const int i0 = ti * 16 * WI, c0 = tc * 16 * WJ, t0 = tg * T;
    if (i0 >= NI || c0 >= Kk) return;
    const int NIp = (NI + PAD - 1) / PAD * PAD;
    int64_t wq = 0;  // offset of q's planes
    for (int qq = q0; qq < q; ++qq) {
        const int np = (d.ni[qq] + PAD - 1) / PAD * PAD;
        wq += int64_t(ntau) * np * np;
    }
    const float2* w32 = reinterpret_cast<const float2*>(wsc) + wq;
    const uint32_t* whi = reinterpret_cast<const uint32_t*>(wsc) + wq;
    const uint32_t* wlo = reinterpret_cast<const uint32_t*>(wsc) + plane + wq;

    const float2* A = M + (d.mpre[q] - d.mpre[q0]) + d.moff[q * nk + k];

    floatx4 acc[WI][WJ][T][2];
#pragma unroll
    for (int a = 0; a < WI; ++a)
#pragma unroll
        for (int b = 0; b < WJ; ++b)
#pragma unroll
            for (int t = 0; t < T; ++t) acc[a][b][t][0] = acc[a][b][t][1] = floatx4{0, 0, 0, 0};

    int tau_[T];
#pragma unroll
    for (int t = 0; t < T; ++t) tau_[t] = min(t0 + t, ntau - 1);

    const int nsteps = (NI + 15) / 16;
    for (int s = i0 / 16; s < nsteps; ++s) {
        const int jb = s * 16;
        float2 mb[WJ][NE];
#pragma unroll
        for (int b = 0; b < WJ; ++b) {
            const int col = c0 + 16 * b + r16;
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const int J = jb + LY::koff(g4, e);
                mb[b][e] = (J < NI && col < Kk) ? A[int64_t(J) * Kk + col] : make_float2(0.f, 0.f);
            }
        }
        if constexpr (PREC == PREC_BF16X3) {
            u32x4 bh_re[WJ], bl_re[WJ], bh_im[WJ], bl_im[WJ];
#pragma unroll
            for (int b = 0; b < WJ; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    uint32_t h, l;
                    split2(mb[b][e].x, mb[b][e].y, h, l);
                    bh_re[b][e] = conj_pk(h);
                    bl_re[b][e] = conj_pk(l);
                    bh_im[b][e] = swap_pk(h);
                    bl_im[b][e] = swap_pk(l);
                }
#pragma unroll
            for (int t = 0; t < T; ++t) {
#pragma unroll
                for (int a = 0; a < WI; ++a) {
                    const int64_t at = (int64_t(tau_[t]) * NIp + i0 + 16 * a + r16) * NIp + jb + 4 * g4;
                    const u32x4 ah = *reinterpret_cast<const u32x4*>(whi + at);
                    const u32x4 al = *reinterpret_cast<const u32x4*>(wlo + at);
#pragma unroll
                    for (int b = 0; b < WJ; ++b) {
                        acc[a][b][t][0] = mfma_bf16(ah, bh_re[b], acc[a][b][t][0]);
                        acc[a][b][t][1] = mfma_bf16(ah, bh_im[b], acc[a][b][t][1]);
                    }
#pragma unroll
                    for (int b = 0; b < WJ; ++b) {
                        acc[a][b][t][0] = mfma_bf16(ah, bl_re[b], acc[a][b][t][0]);
                        acc[a][b][t][1] = mfma_bf16(ah, bl_im[b], acc[a][b][t][1]);
                    }
#pragma unroll
                    for (int b = 0; b < WJ; ++b) {
                        acc[a][b][t][0] = mfma_bf16(al, bh_re[b], acc[a][b][t][0]);
                        acc[a][b][t][1] = mfma_bf16(al, bh_im[b], acc[a][b][t][1]);
                    }
                }
            }
        } else {
            const bool imc = g4 & 1;
#pragma unroll
            for (int t = 0; t < T; ++t) {
#pragma unroll
                for (int a = 0; a < WI; ++a) {
                    const int64_t row = (int64_t(tau_[t]) * NIp + i0 + 16 * a + r16) * NIp + jb;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const float2 w = w32[row + LY::koff(g4, e)];
                        const float x = imc ? w.y : w.x;
#pragma unroll
                        for (int b = 0; b < WJ; ++b) {
                            const float bre = imc ? -mb[b][e].y : mb[b][e].x;
                            const float bim = imc ? mb[b][e].x : mb[b][e].y;
                            acc[a][b][t][0] = mfma_f32(x, bre, acc[a][b][t][0]);
                            acc[a][b][t][1] = mfma_f32(x, bim, acc[a][b][t][1]);
                        }
                    }
                }
            }
        }
    }

    // epilogue: Re(conj(M) Y) over this tile's rows, weighted by G_m, summed per band n
    const double sc = 2.0 * d.scale;  // both triangles of U
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int it = t0 + t;
        if (it >= ntau) break;
        double part[WJ];
#pragma unroll
        for (int b = 0; b < WJ; ++b) {
            const int col = c0 + 16 * b + r16;
            float s = 0.f;
            if (col < Kk) {
#pragma unroll
                for (int a = 0; a < WI; ++a)
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const int I = i0 + 16 * a + 4 * g4 + rr;
                        if (I < NI) {
                            const float2 m = A[int64_t(I) * Kk + col];
                            s += m.x * acc[a][b][t][0][rr] + m.y * acc[a][b][t][1][rr];
                        }
                    }
            }
            double v = s;
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (col < Kk) {
                const int m = col - (col / nm) * nm;
                v *= G[(int64_t(kq) * nbmax + m) * ntau + it];
            }
            part[b] = v;
        }
        // sum the tile's columns band by band (columns are consecutive (n, m) pairs)
        const int cl = min(c0 + 16 * WJ, Kk) - 1;
        const int nlo = c0 / nm, nhi = cl / nm;
        for (int nx = nlo; nx <= nhi; ++nx) {
            double v = 0.0;
#pragma unroll
            for (int b = 0; b < WJ; ++b) {
                const int col = c0 + 16 * b + r16;
                if (col < Kk && col / nm == nx) v += part[b];
            }
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0) atomicAdd(&Sig[(int64_t(k) * nbmax + nx) * ntau + it], sc * v);
        }
    }
}

// =================================================================================================
// self-energy, v3: M split and transposed once per call
// =================================================================================================
// Mt planes: for each (q, k) of the call, hi and lo bf16 pairs of M^J_col laid out [col][J] with J
// zero-padded to NIp16 = NI rounded up to 16, so a lane's 4 consecutive J are one 16-byte load.
// The (q, k) block starts at mt_base(q) + moff[q][k] / NI_q * NIp16.
__device__ __forceinline__ int64_t mt_qbase(const Dev& d, int q0, int q) {
    int64_t b = 0;
    for (int qq = q0; qq < q; ++qq) {
        const int ni = d.ni[qq];
        b += (d.mpre[qq + 1] - d.mpre[qq]) / ni * ((ni + 15) / 16 * 16);
    }
    return b;
}

__global__ __launch_bounds__(256) void k_split_mt(Dev d, int q0, int q, const float2* __restrict__ M,
                                                  uint32_t* __restrict__ mt, int64_t mtplane) {
    __shared__ float2 tile[32][33];
    const int nk = d.nk, k = blockIdx.y;
    const int NI = d.ni[q], NIp16 = (NI + 15) / 16 * 16;
    const int Kk = d.nb[k] * d.nb[d.kmq[q * nk + k]];
    const int ntj = (NIp16 + 31) / 32;
    const int j0 = (blockIdx.x % ntj) * 32, c0 = (blockIdx.x / ntj) * 32;
    if (c0 >= Kk) return;
    const float2* A = M + (d.mpre[q] - d.mpre[q0]) + d.moff[q * nk + k];
    const int64_t ob = mt_qbase(d, q0, q) + d.moff[q * nk + k] / NI * NIp16;
    uint32_t* mh = mt + ob;
    uint32_t* ml = mt + mtplane + ob;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int J = j0 + r, col = c0 + tx;
        tile[r][tx] = (J < NI && col < Kk) ? A[int64_t(J) * Kk + col] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int col = c0 + r, J = j0 + tx;
        if (col < Kk && J < NIp16) {
            const float2 v = tile[tx][r];
            uint32_t h, l;
            split2(v.x, v.y, h, l);
            mh[int64_t(col) * NIp16 + J] = h;
            ml[int64_t(col) * NIp16 + J] = l;
        }
    }
}

// =================================================================================================
// 32x32x16 MFMA helpers
// =================================================================================================
// v_mfma_f32_32x32x16_bf16 sustains close to the BF16 peak on gfx950 where the 16x16x32 shape
// reaches about half of it, so these kernels use 32 x 32 output tiles and a K-step of 8 complex
// elements.  Operand layout (lane l, 64 lanes): A row l % 32, B column l % 32, each with the 8
// consecutive bf16 of K = 4 (l / 32) + e, e < 4 complex elements; the 16 accumulators of lane l hold
// rows 8 g + 4 (l / 32) + r (acc index 4 g + r) of column l % 32.
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ floatx16 mfma32(u32x4 a, u32x4 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
template <int PR>
__device__ __forceinline__ floatx16 mfma32p(u32x4 a, u32x4 b, floatx16 c) {
    if constexpr (PR == PREC_F16X3)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                      0, 0, 0);
    else
        return mfma32(a, b, c);
}
__device__ __forceinline__ void zero16(floatx16& x) {
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = 0.f;
}
// =================================================================================================
// v7 self-energy: LDS double-buffered 32x32x16 contraction
// =================================================================================================
// Work-group = 4 waves in a 2 x 2 grid over 64 rows I and 128 columns c = (n, m) of one k block,
// for T tau points.  The reduction over J advances in stages of 16; each stage of the U planes
// (T x 64 rows x 16 J, hi and lo) and of the split, transposed M (128 columns x 16 J, hi and lo)
// is loaded once per work-group into registers while the previous stage is multiplied out of
// LDS, then written to the other LDS buffer: one barrier per stage, and the global latency hides
// behind 96 MFMAs per wave.
constexpr int S7_KS = 16;         // J per stage
constexpr int S7_RS = S7_KS + 4;  // LDS row stride in u32 (80 B: conflict-free 16-B reads)

template <int T, int OCC = 1>
__global__ __launch_bounds__(256, OCC) void k_sig7(Dev d, int q0, const float2* __restrict__ M,
                                              const double* __restrict__ G,
                                              const char* __restrict__ wsc, int64_t plane,
                                              const uint32_t* __restrict__ mt, int64_t mtplane,
                                              double* __restrict__ Sig, Order od, int ntI, int ntC) {
    __shared__ uint32_t As[2][2][T][64][S7_RS];  // [buffer][hi, lo][tau][row][J]
    __shared__ uint32_t Bs[2][2][128][S7_RS];    // [buffer][hi, lo][column][J]
    int qrel, r, c;
    if (!work_item(od, qrel, r, c)) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r32 = lane & 31, h2 = lane >> 5;
    const int wi = wave & 1, wc = wave >> 1;
    const int nk = d.nk, ntau = d.ntau, nbmax = d.nbmax;
    const int q = q0 + qrel;
    const int tg = r / ntI, ti = r - tg * ntI;
    const int k = c / ntC, tc = c - k * ntC;
    const int kq = d.kmq[q * nk + k];
    const int nm = d.nb[kq], NI = d.ni[q];
    const int Kk = d.nb[k] * nm;
    const int i0 = ti * 64, c0 = tc * 128, t0 = tg * T;
    if (i0 >= NI || c0 >= Kk) return;  // uniform over the work-group
    const int NIp = (NI + PAD - 1) / PAD * PAD, NIp16 = (NI + 15) / 16 * 16;
    int64_t wq = 0;
    for (int qq = q0; qq < q; ++qq) {
        const int np = (d.ni[qq] + PAD - 1) / PAD * PAD;
        wq += int64_t(ntau) * np * np;
    }
    // one base pointer per operand (the lo planes are at fixed offsets), so that every load is a
    // plain global load
    const uint32_t* wbase = reinterpret_cast<const uint32_t*>(wsc) + wq;
    const uint32_t* mbase = mt + mt_qbase(d, q0, q) + d.moff[q * nk + k] / NI * NIp16;

    // this thread's share of a stage: 2T chunks of the U planes, 4 of the M planes (16 B each)
    constexpr int NA = 2 * T, NB = 4;
    int64_t aoff[NA];
    int alds[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int id = tid + 256 * i;
        const int aq = id & 3, ar = (id >> 2) & 63, tp = id >> 8;
        const int at = tp % T, ap = tp / T;
        const int tau = min(t0 + at, ntau - 1);
        aoff[i] = ap * plane + (int64_t(tau) * NIp + i0 + ar) * NIp + 4 * aq;
        alds[i] = ((ap * T + at) * 64 + ar) * S7_RS + 4 * aq;  // within one buffer of As
    }
    int64_t boff[NB];
    int blds[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int id = tid + 256 * i;
        const int bq = id & 3, bc = (id >> 2) & 127, bp = id >> 9;
        boff[i] = bp * mtplane + int64_t(min(c0 + bc, Kk - 1)) * NIp16 + 4 * bq;
        blds[i] = (bp * 128 + bc) * S7_RS + 4 * bq;
    }
    u32x4 ra[NA], rb[NB];
    auto gload = [&](int J0) {
#pragma unroll
        for (int i = 0; i < NA; ++i) ra[i] = *reinterpret_cast<const u32x4*>(wbase + aoff[i] + J0);
#pragma unroll
        for (int i = 0; i < NB; ++i) rb[i] = *reinterpret_cast<const u32x4*>(mbase + boff[i] + J0);
    };
    auto lstore = [&](int buf) {
        uint32_t* a = &As[buf][0][0][0][0];
        uint32_t* b = &Bs[buf][0][0][0];
#pragma unroll
        for (int i = 0; i < NA; ++i) *reinterpret_cast<u32x4*>(a + alds[i]) = ra[i];
#pragma unroll
        for (int i = 0; i < NB; ++i) *reinterpret_cast<u32x4*>(b + blds[i]) = rb[i];
    };
    // fragments of one 8-J step: A for every tau (hi, lo), B for both column tiles (hi, lo)
    auto lread = [&](int buf, int kk, u32x4 (&fa)[T][2], u32x4 (&fb)[2][2]) {
        const int jo = 8 * kk + 4 * h2;
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int p = 0; p < 2; ++p)
                fb[b][p] = reinterpret_cast<const u32x4*>(&Bs[buf][p][64 * wc + 32 * b + r32][0])[jo / 4];
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int p = 0; p < 2; ++p)
                fa[t][p] = reinterpret_cast<const u32x4*>(&As[buf][p][t][32 * wi + r32][0])[jo / 4];
    };

    floatx16 acc[2][T][2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int t = 0; t < T; ++t) {
            zero16(acc[b][t][0]);
            zero16(acc[b][t][1]);
        }
    auto compute = [&](const u32x4 (&fa)[T][2], const u32x4 (&fb)[2][2]) {
        u32x4 bre[2][2], bim[2][2];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    bre[b][p][e] = conj_pk(fb[b][p][e]);
                    bim[b][p][e] = swap_pk(fb[b][p][e]);
                }
#pragma unroll
        for (int t = 0; t < T; ++t) {
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                acc[b][t][0] = mfma32(fa[t][0], bre[b][0], acc[b][t][0]);
                acc[b][t][1] = mfma32(fa[t][0], bim[b][0], acc[b][t][1]);
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                acc[b][t][0] = mfma32(fa[t][0], bre[b][1], acc[b][t][0]);
                acc[b][t][1] = mfma32(fa[t][0], bim[b][1], acc[b][t][1]);
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                acc[b][t][0] = mfma32(fa[t][1], bre[b][0], acc[b][t][0]);
                acc[b][t][1] = mfma32(fa[t][1], bim[b][0], acc[b][t][1]);
            }
        }
    };

    // U is zero below the diagonal: the reduction starts at the work-group's first row
    const int ns = (NIp16 - i0) / S7_KS;
    gload(i0);
    lstore(0);
    __syncthreads();
    for (int s = 0; s < ns; ++s) {
        const int buf = s & 1;
        if (s + 1 < ns) gload(i0 + (s + 1) * S7_KS);
        if constexpr (OCC == 1) {
            u32x4 fa0[T][2], fb0[2][2], fa1[T][2], fb1[2][2];
            lread(buf, 0, fa0, fb0);
            lread(buf, 1, fa1, fb1);  // in flight while step 0 multiplies
            // keep the compiler from sinking the step-1 reads next to their use
            __builtin_amdgcn_sched_barrier(0);
            compute(fa0, fb0);
            __builtin_amdgcn_sched_barrier(0);
            compute(fa1, fb1);
        } else {
            // two work-groups per CU cover each other's LDS and barrier latency
#pragma unroll
            for (int kk = 0; kk < S7_KS / 8; ++kk) {
                u32x4 fa[T][2], fb[2][2];
                lread(buf, kk, fa, fb);
                compute(fa, fb);
            }
        }
        if (s + 1 < ns) lstore(buf ^ 1);
        __syncthreads();
    }

    // epilogue: Re(conj(M) Y) over this wave's rows, weighted by G_m, summed per band n
    const float2* A = M + (d.mpre[q] - d.mpre[q0]) + d.moff[q * nk + k];
    const double sc = 2.0 * d.scale;  // both triangles of U
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int it = t0 + t;
        if (it >= ntau) break;
        double part[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int col = c0 + 64 * wc + 32 * b + r32;
            float s = 0.f;
            if (col < Kk) {
#pragma unroll
                for (int x = 0; x < 16; ++x) {
                    const int I = i0 + 32 * wi + 8 * (x >> 2) + 4 * h2 + (x & 3);
                    if (I < NI) {
                        const float2 m = A[int64_t(I) * Kk + col];
                        s += m.x * acc[b][t][0][x] + m.y * acc[b][t][1][x];
                    }
                }
            }
            double v = s;
            v += __shfl_xor(v, 32);
            if (col < Kk) v *= G[(int64_t(kq) * nbmax + (col - (col / nm) * nm)) * ntau + it];
            part[b] = v;
        }
        const int cb = c0 + 64 * wc;
        if (cb >= Kk) continue;
        const int nlo = cb / nm, nhi = (min(cb + 64, Kk) - 1) / nm;
        for (int nx = nlo; nx <= nhi; ++nx) {
            double v = 0.0;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int col = cb + 32 * b + r32;
                if (col < Kk && col / nm == nx) v += part[b];
            }
#pragma unroll
            for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0) atomicAdd(&Sig[(int64_t(k) * nbmax + nx) * ntau + it], sc * v);
        }
    }
}

// =================================================================================================
// pair-space polarization (vZ)
// =================================================================================================
// The weight g_K(tau) = G_n(k,tau) G_m(k-q,beta-tau) is real, so with Z_IJ,K = M^I_K conj(M^J_K)
//     P_IJ(tau) = s sum_k sum_K Z_IJ,K g_K(tau)
// is a real GEMM per component: rows = pairs (I, J), reduction = K, columns = tau.  Z is formed on
// the fly from the rows of M (4 FLOP per complex element, shared by every tau), and g is a small
// table per (q, k) that k_gtab writes once per call as bf16 hi/lo planes [tau][K] -- no operand is
// rescaled per tau.  Against the complex GEMM this halves the MFMA work (complex x real instead of
// complex x complex) and the VALU work per MFMA.
constexpr int GZ_T = 96;   // tau columns per work-group (three 32-wide MFMA tiles)
constexpr int GZ_KS = 32;  // K per stage (default)
constexpr int GZ_KPAD = 64;  // the g planes are padded in K to a multiple of the largest stage
// K terms summed in the FP32 accumulators between two flushes into the FP64 P.  The FP32 rounding of
// these sums dominates the split precisions' error: flushing every 16384 terms instead would save 11%
// of the kernel's time at NI = 700, but raised P's error 2-4x (1.3e-7 -> 4.5e-7 at the NI = 400 block
// shapes, which the screen amplifies ~5x into W~ and Sigma).
constexpr int GZ_FLUSH = 4096;

// g planes of q0..q0+nq-1: for each (q, k) two bf16 planes [TP][KP], TP = Ntau rounded up to GZ_T,
// KP = K rounded up to GZ_KPAD
__device__ __host__ __forceinline__ int gz_tp(int ntau) { return (ntau + GZ_T - 1) / GZ_T * GZ_T; }
__device__ __forceinline__ int64_t gz_block(const Dev& d, int q0, int q, int k) {
    int64_t off = 0;
    for (int qq = q0; qq <= q; ++qq)
        for (int kk = 0; kk < (qq == q ? k : d.nk); ++kk) {
            const int K = d.nb[kk] * d.nb[d.kmq[qq * d.nk + kk]];
            off += int64_t(2) * gz_tp(d.ntau) * ((K + GZ_KPAD - 1) / GZ_KPAD * GZ_KPAD);
        }
    return off;  // in bf16 elements
}

// tau points the pair-space polarization computes: all of them, or i <= (N - 1) / 2 with the mirror
int tau_points_computed(const Dev& d, const Host& h) { return d.tau_mirror ? (h.ntau + 1) / 2 : h.ntau; }

// P(tau_i) = P(tau_{N-1-i}) for the points i >= nt_eff (whole planes, after the mirror below the diagonal)
__global__ __launch_bounds__(256) void k_tau_mirror(double2* __restrict__ P, int NI, int ntau, int nt_eff) {
    const int64_t nn = int64_t(NI) * NI;
    const int i = nt_eff + int(blockIdx.y);
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e < nn) P[int64_t(i) * nn + e] = P[int64_t(ntau - 1 - i) * nn + e];
}

// ---- F16X3 operand scales ------------------------------------------------------------------------
// A fill kernel rather than a memset, so that the calls stay capturable in a graph.
__global__ __launch_bounds__(256) void k_fill_u64(unsigned long long* __restrict__ p, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0ull;
}
// largest value among the block's threads, then one atomic max on the bits (order-preserving for
// non-negative doubles)
__device__ __forceinline__ void block_max_atomic(double v, unsigned long long* out) {
    __shared__ double part[4];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double b = fmax(fmax(part[0], part[1]), fmax(part[2], part[3]));
        atomicMax(out, static_cast<unsigned long long>(__double_as_longlong(b)));
    }
}
// max |M^I_K|^2 over the n complex elements of one q's block
__global__ __launch_bounds__(256) void k_mmax(const float2* __restrict__ M, int64_t n,
                                              unsigned long long* __restrict__ out) {
    double v = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        const float2 a = M[i];
        v = fmax(v, double(a.x) * a.x + double(a.y) * a.y);
    }
    block_max_atomic(v, out);
}
// max |Re|, |Im| of W~(q, tau) for the tau plane blockIdx.y of one q
__global__ __launch_bounds__(256) void k_wmax(const double2* __restrict__ W, int NI,
                                              unsigned long long* __restrict__ out) {
    const int64_t nn = int64_t(NI) * NI;
    const double2* Wt = W + int64_t(blockIdx.y) * nn;
    double v = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < nn; i += int64_t(gridDim.x) * 256) {
        const double2 a = Wt[i];
        v = fmax(v, fmax(fabs(a.x), fabs(a.y)));
    }
    block_max_atomic(v, out + blockIdx.y);
}
// max_n |G_n(k, tau)| for every (k, tau)
__global__ __launch_bounds__(256) void k_gmax(Dev d, const double* __restrict__ G) {
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= d.nk * d.ntau) return;
    const int k = id / d.ntau, t = id - k * d.ntau;
    double v = 0.0;
    for (int n = 0; n < d.nb[k]; ++n) v = fmax(v, fabs(G[(int64_t(k) * d.nbmax + n) * d.ntau + t]));
    d.g_max[id] = v;
}
// exponent of the polarization weights of (q, tau): max_K |g_K(tau)| over the blocks of q is
// max_k g_max(k, tau) g_max(k - q, beta - tau), attained by the two largest factors
__global__ __launch_bounds__(256) void k_gexp(Dev d, int q0, int nq) {
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= nq * d.ntau) return;
    const int q = q0 + id / d.ntau, t = id % d.ntau;
    double u = 0.0;
    for (int k = 0; k < d.nk; ++k)
        u = fmax(u, d.g_max[k * d.ntau + t] * d.g_max[d.kmq[q * d.nk + k] * d.ntau + (d.ntau - 1 - t)]);
    d.e_g[q * d.ntau + t] = u > 0.0 ? 14 - exp_above(u) : 0;
}
// the maxima of M for q0..q0+nq-1 (polarization and self-energy) and of W~ (self-energy)
void launch_scales(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M, const void* W) {
    MSGW_LAUNCH(k_fill_u64, dim3(ceil_div(nq, 256)), dim3(256), 0, s, d.mx_m + q0, nq);
    if (W) MSGW_LAUNCH(k_fill_u64, dim3(ceil_div(int64_t(nq) * h.ntau, 256)), dim3(256), 0, s,
                       d.mx_w + int64_t(q0) * h.ntau, nq * h.ntau);
    for (int q = q0; q < q0 + nq; ++q) {
        const int64_t n = h.mpre[q + 1] - h.mpre[q];
        MSGW_LAUNCH(k_mmax, dim3(unsigned(std::min<int64_t>(ceil_div(n, 256), 4096))), dim3(256), 0, s,
                    (const float2*)M + (h.mpre[q] - h.mpre[q0]), n, d.mx_m + q);
        if (W) {
            const int64_t nn = int64_t(h.ni[q]) * h.ni[q];
            MSGW_LAUNCH(k_wmax, dim3(unsigned(std::min<int64_t>(ceil_div(nn, 256), 64)), h.ntau), dim3(256), 0, s,
                        (const double2*)W + (h.ppre[q] - h.ppre[q0]), h.ni[q], d.mx_w + int64_t(q) * h.ntau);
        }
    }
    MSGW_HIP(hipGetLastError());
}

// one thread per (tau, K pair): writes hi and lo of g for two consecutive K.  gz points at the planes
// of q; the offset of block k inside them is summed over the k' < k by the whole work-group.
template <int PR>
__global__ __launch_bounds__(256) void k_gtab(Dev d, int q, const double* __restrict__ G,
                                              uint32_t* __restrict__ gz) {
    __shared__ int64_t part[4];
    const int k = blockIdx.y, nk = d.nk, ntau = d.ntau, nbmax = d.nbmax;
    const int kq = d.kmq[q * nk + k];
    const int nm = d.nb[kq], Kk = d.nb[k] * nm;
    const int KP = (Kk + GZ_KPAD - 1) / GZ_KPAD * GZ_KPAD;
    const int TP = gz_tp(ntau);
    int64_t o = 0;
    for (int kk = threadIdx.x; kk < k; kk += 256) {
        const int K = d.nb[kk] * d.nb[d.kmq[q * nk + kk]];
        o += int64_t(2) * TP * ((K + GZ_KPAD - 1) / GZ_KPAD * GZ_KPAD);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) o += __shfl_xor(o, m);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = o;
    __syncthreads();
    const int64_t off = part[0] + part[1] + part[2] + part[3];  // bf16 elements, even
    const int id = blockIdx.x * 256 + threadIdx.x;
    const int npair = KP / 2;
    if (id >= TP * npair) return;
    const int t = id / npair, K0 = 2 * (id - t * npair);
    // F16X3: the column tau is scaled by 2^e_g(q, tau)
    const double gs = (PR == PREC_F16X3 && t < ntau) ? ldexp(1.0, d.e_g[q * ntau + t]) : 1.0;
    float g[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int K = K0 + e;
        g[e] = 0.f;
        if (t < ntau && K < Kk) {
            const int n = K / nm, m = K - n * nm;
            g[e] = float(G[(int64_t(k) * nbmax + n) * ntau + t] *
                         G[(int64_t(kq) * nbmax + m) * ntau + (ntau - 1 - t)] * gs);
        }
    }
    uint32_t h, l;
    split_pair<PR>(g[0], g[1], h, l);
    uint32_t* hp = gz + (off >> 1);
    hp[int64_t(t) * (KP / 2) + K0 / 2] = h;
    hp[int64_t(TP + t) * (KP / 2) + K0 / 2] = l;
}

// Work-group = 2 WI waves over a block of 4 WI rows I x 16 rows J (64 WI pairs); wave w owns the 32
// pairs I = I0 + 4 (w % WI) + p / 8, J = J0 + 8 (w / WI) + p % 8 (p = lane % 32) for all 96 tau
// columns.  Each stage brings KS K of the block's 4 WI + 16 rows of M and of the g planes through LDS
// (double buffered); each lane forms Z for its pair and 8 K per MFMA step and splits it into bf16
// hi/lo.  A larger WI shares every staged g plane among more pairs.
// NTT 32-wide tau tiles per work item (a chunk of CW = 32 NTT tau columns): three for the chunks of 96,
// one or two for a tail chunk; the launch covers ntc chunks starting at tau t0.
// NBUF = 2: stage s + 1 is loaded into registers during stage s and written to the other LDS buffer
// after it.  NBUF = 3: the buffer written after stage s is the one for stage s + 2, so stage s + 1 is
// already in LDS while stage s runs and the Z of its first step is formed during the last MFMAs of
// stage s (one barrier per stage either way).
// One work item of the pair-space polarization: 4 WI rows I from I0 = 4 WI r, 16 columns J from
// J0 = 16 (c / ntc), tau chunk c % ntc of the launch, over all k blocks of q = q0 + qrel.
template <int OCC, int KS, int WI, int NTT, int NBUF, int PR>
__device__ __forceinline__ void polz_item(const Dev& d, int q0, const float2* __restrict__ M,
                                          const uint32_t* __restrict__ gz, double2* __restrict__ P, int qrel,
                                          int r, int c, int t0, int ntc, int nt_eff) {
    constexpr int NT = 128 * WI, XROWS = 4 * WI + 16, CW = 32 * NTT;
    static_assert(KS % GZ_KS == 0, "stages hold whole 32-K slabs of the g planes");
    static_assert((XROWS * KS) % NT == 0 && (2 * CW * KS / 8) % NT == 0, "stage split over threads");
    constexpr int XR = 2 * KS + 4, GR = KS / 2 + 4, NX = XROWS * KS / NT, NG = 2 * CW * KS / 8 / NT;
    static_assert(NBUF == 2 || (NBUF == 3 && (KS / 16) % 2 == 0), "three buffers need an even step count");
    __shared__ float Xs[NBUF][XROWS][XR];     // [buffer][row: 4 WI rows I then 16 rows J][K re, im]
    __shared__ uint32_t Gs[NBUF][2][CW][GR];  // [buffer][hi, lo][tau][K pair]
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r32 = lane & 31, h2 = lane >> 5;
    const int q = q0 + qrel, nk = d.nk, ntau = d.ntau;
    const int NI = d.ni[q];
    const int cj = c / ntc, tc = c - cj * ntc;  // tau chunk tc of this launch
    const int I0 = r * 4 * WI, J0 = cj * 16, TP = gz_tp(ntau), tb = t0 + CW * tc;
    if (I0 >= NI || J0 >= NI || J0 + 16 <= I0) return;  // uniform; below the diagonal: mirrored later
    const float2* Mq = M + (d.mpre[q] - d.mpre[q0]);
    double2* Pq = P + (d.ppre[q] - d.ppre[q0]);
    const int64_t gq = gz_block(d, q0, q, 0);
    // F16X3: M is scaled by 2^em as it is staged, the g planes by 2^e_g(q, tau) (k_gtab)
    const int em = PR == PREC_F16X3 ? f16_exp_m(d.mx_m[q]) : 0;
    const float fm = PR == PREC_F16X3 ? ldexpf(1.f, em) : 1.f;

    // staging per thread: NX complex elements of the M rows and NG 16-B chunks of the g planes
    float2 rx[NX];
    u32x4 rg[NG];
    struct Blk {
        const float2* A;
        const uint32_t* g;
        int Kk, KP, k;
    };
    auto block_of = [&](int kx) {
        Blk b;
        b.k = kx;
        const int kq = d.kmq[q * nk + kx];
        b.Kk = d.nb[kx] * d.nb[kq];
        b.KP = (b.Kk + GZ_KPAD - 1) / GZ_KPAD * GZ_KPAD;
        b.A = Mq + d.moff[q * nk + kx];
        return b;
    };
    // blocks are visited in k order: the g planes of block k follow those of block k - 1
    auto next_block = [&](const Blk& prev, int kx) {
        Blk b = block_of(kx);
        b.g = prev.g + int64_t(TP) * prev.KP;
        return b;
    };
    // Byte offsets of this thread's staged elements from the block's base pointers, 32-bit (the host
    // checks that a block's M rows and g planes fit), recomputed when the block changes: a stage then
    // needs only a uniform base per block and slab.  Rows past NI and K past the block's K read the
    // nearest valid element instead of zeros: such rows only form pairs that are never stored, and the
    // g planes are zero for K past the block's K, so those terms add exact zeros.
    uint32_t xo[NX], go[NG];
    int offk = -1;
    constexpr int CH = KS / 8;  // 16-B chunks per g row of a stage
    auto set_offsets = [&](const Blk& b) {
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            const int id = tid + NT * i;             // XROWS rows x KS
            const int row = id / KS, kc = id % KS;
            const int R = row < 4 * WI ? I0 + row : J0 + row - 4 * WI;
            xo[i] = uint32_t(min(R, NI - 1) * b.Kk + kc) * uint32_t(sizeof(float2));
        }
#pragma unroll
        for (int i = 0; i < NG; ++i) {
            const int id = tid + NT * i;             // 2 planes x CW tau x CH chunks of 4 u32
            const int pl = id / (CW * CH), rem = id - pl * CW * CH;
            const int t = rem / CH, ch = rem % CH;
            go[i] = uint32_t((pl * TP + tb + t) * b.KP) * 2u + 16u * uint32_t(ch);
        }
        offk = b.k;
    };
    auto gload = [&](const Blk& b, int slab) {
        const int K0 = slab * KS;
        if (b.k != offk) set_offsets(b);
        const char* gb = reinterpret_cast<const char*>(b.g) + 2 * int64_t(K0);
#pragma unroll
        for (int i = 0; i < NG; ++i) rg[i] = *reinterpret_cast<const u32x4*>(gb + go[i]);
        if (K0 + KS <= b.Kk) {
            const char* xb = reinterpret_cast<const char*>(b.A + K0);
#pragma unroll
            for (int i = 0; i < NX; ++i) rx[i] = *reinterpret_cast<const float2*>(xb + xo[i]);
        } else {  // the last slab of a block whose K is not a multiple of KS
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                const int id = tid + NT * i;
                const int row = id / KS, kc = id % KS;
                const int R = row < 4 * WI ? I0 + row : J0 + row - 4 * WI;
                rx[i] = b.A[int64_t(min(R, NI - 1)) * b.Kk + min(K0 + kc, b.Kk - 1)];
            }
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            const int id = tid + NT * i;
            const int row = id / KS, kc = id % KS;
            float2 x = rx[i];
            if constexpr (PR == PREC_F16X3) {
                x.x *= fm;
                x.y *= fm;
            }
            *reinterpret_cast<float2*>(&Xs[buf][row][2 * kc]) = x;
        }
#pragma unroll
        for (int i = 0; i < NG; ++i) {
            const int id = tid + NT * i;
            const int pl = id / (CW * CH), rem = id - pl * CW * CH;
            const int t = rem / CH, ch = rem % CH;
            *reinterpret_cast<u32x4*>(&Gs[buf][pl][t][4 * ch]) = rg[i];
        }
    };

    floatx16 acc[NTT][2];  // [tau tile][re, im]
#pragma unroll
    for (int tt = 0; tt < NTT; ++tt) {
        zero16(acc[tt][0]);
        zero16(acc[tt][1]);
    }
    const int ri = 4 * (wave % WI) + (r32 >> 3), rj = 4 * WI + 8 * (wave / WI) + (r32 & 7);
    // Z = x_I conj(x_J) for this lane's pair and K = 16 kk + 8 h2 + e, e < 8, split into bf16 hi/lo
    auto zform = [&](int buf, int kk, u32x4 (&z)[4]) {
        const float* xi = &Xs[buf][ri][2 * (16 * kk + 8 * h2)];
        const float* xj = &Xs[buf][rj][2 * (16 * kk + 8 * h2)];
        float zr[8], zi[8];
#pragma unroll
        for (int e4 = 0; e4 < 4; ++e4) {
            const float4 a = *reinterpret_cast<const float4*>(xi + 4 * e4);
            const float4 b = *reinterpret_cast<const float4*>(xj + 4 * e4);
            zr[2 * e4] = a.x * b.x + a.y * b.y;
            zi[2 * e4] = a.y * b.x - a.x * b.y;
            zr[2 * e4 + 1] = a.z * b.z + a.w * b.w;
            zi[2 * e4 + 1] = a.w * b.z - a.z * b.w;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if constexpr (PR == PREC_F16X3) {
                uint32_t h, l;
                split_f16(zr[2 * e], zr[2 * e + 1], h, l);
                z[0][e] = h;
                z[1][e] = l;
                split_f16(zi[2 * e], zi[2 * e + 1], h, l);
                z[2][e] = h;
                z[3][e] = l;
            } else {
                uint32_t h;
                h = pk_bf16(zr[2 * e], zr[2 * e + 1]);
                z[0][e] = h;
                z[1][e] = pk_bf16(zr[2 * e] - bf_lo_perm(h), zr[2 * e + 1] - bf_hi(h));
                h = pk_bf16(zi[2 * e], zi[2 * e + 1]);
                z[2][e] = h;
                z[3][e] = pk_bf16(zi[2 * e] - bf_lo_perm(h), zi[2 * e + 1] - bf_hi(h));
            }
        }
    };
    // the 6 NTT MFMAs of one 16-K step: Z (re hi, re lo, im hi, im lo) against g (hi, lo) per tau tile
    auto mmas = [&](int buf, int kk, const u32x4 (&z)[4]) {
#pragma unroll
        for (int tt = 0; tt < NTT; ++tt) {
            const u32x4* grow = reinterpret_cast<const u32x4*>(&Gs[buf][0][32 * tt + r32][0]);
            const u32x4* lrow = reinterpret_cast<const u32x4*>(&Gs[buf][1][32 * tt + r32][0]);
            const u32x4 gh = grow[2 * kk + h2], gl = lrow[2 * kk + h2];
            acc[tt][0] = mfma32p<PR>(z[0], gh, acc[tt][0]);
            acc[tt][1] = mfma32p<PR>(z[2], gh, acc[tt][1]);
            acc[tt][0] = mfma32p<PR>(z[0], gl, acc[tt][0]);
            acc[tt][1] = mfma32p<PR>(z[2], gl, acc[tt][1]);
            acc[tt][0] = mfma32p<PR>(z[1], gh, acc[tt][0]);
            acc[tt][1] = mfma32p<PR>(z[3], gh, acc[tt][1]);
        }
    };
    // software pipeline over the 16-K steps of a stage: the VALU work that forms Z for step kk + 1 is
    // interleaved with the MFMAs of step kk
    auto compute_stage = [&](int buf) {
        u32x4 za[4], zb[4];
        zform(buf, 0, za);
#pragma unroll
        for (int kk = 0; kk < KS / 16; ++kk) {
            if (kk & 1) {
                mmas(buf, kk, zb);
                if (kk + 1 < KS / 16) zform(buf, kk + 1, za);
            } else {
                mmas(buf, kk, za);
                if (kk + 1 < KS / 16) zform(buf, kk + 1, zb);
            }
            if (kk + 1 < KS / 16) {
#pragma unroll
                for (int i = 0; i < 6 * NTT; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
                    __builtin_amdgcn_sched_group_barrier(0x002, 18 / NTT, 0);  // then the VALU share
                }
            }
        }
    };
    // three buffers: z holds the Z of step 0 on entry and that of step 0 of the stage in nbuf on exit
    // (formed during the last step; when no stage follows it is formed from stale LDS and not used)
    auto compute_stage3 = [&](int buf, int nbuf, u32x4 (&za)[4]) {
        u32x4 zb[4];
#pragma unroll
        for (int kk = 0; kk < KS / 16; ++kk) {
            if (kk & 1) {
                mmas(buf, kk, zb);
                zform(kk + 1 < KS / 16 ? buf : nbuf, (kk + 1) % (KS / 16), za);
            } else {
                mmas(buf, kk, za);
                zform(buf, kk + 1, zb);
            }
#pragma unroll
            for (int i = 0; i < 6 * NTT; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
                __builtin_amdgcn_sched_group_barrier(0x002, 18 / NTT, 0);  // then the VALU share
            }
        }
        // pin the next stage's Z here, so that its forming is not moved behind the loop's branches and
        // stays interleaved with the last MFMAs
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) asm volatile("" : "+v"(za[i][j]));
    };

    const double sc = d.scale;
    // s, and for F16X3 the scales of the operands undone, for the tau column it (clamped to the mesh)
    auto col_scale = [&](int it) {
        if constexpr (PR == PREC_F16X3)
            return ldexp(sc, -(2 * em + d.e_g[q * d.ntau + min(it, d.ntau - 1)]));
        else
            return sc;
    };
    bool first = true;
    // P += s acc for this lane's 16 pairs per tau tile.  With one work-group per CU the partial sums
    // already in P are read in batches of 8 from clamped (always valid) addresses before any store,
    // so a batch costs one memory round trip; only the valid elements are written.  With two the
    // registers for that are lacking and each element is read and written in turn.
    constexpr int FB = 8;
    auto flush = [&]() {
        int z = 0;  // opaque zero: keeps the output addresses out of the main loop
        asm volatile("" : "+v"(z));
        if constexpr (OCC > 1) {
#pragma unroll
            for (int tt = 0; tt < NTT; ++tt) {
                const int it = tb + 32 * tt + r32 + z;
                const double cs = col_scale(it);
#pragma unroll
                for (int x = 0; x < 16; ++x) {
                    const int p = 8 * (x >> 2) + 4 * h2 + (x & 3);
                    const int I = I0 + 4 * (wave % WI) + (p >> 3), J = J0 + 8 * (wave / WI) + (p & 7);
                    if (it < nt_eff && I < NI && J < NI) {
                        double2* pp = &Pq[(int64_t(it) * NI + I) * NI + J];
                        double re = cs * double(acc[tt][0][x]);
                        double im = cs * double(acc[tt][1][x]);
                        if (!first) {
                            const double2 o = *pp;
                            re += o.x;
                            im += o.y;
                        }
                        *pp = make_double2(re, im);
                    }
                }
                zero16(acc[tt][0]);
                zero16(acc[tt][1]);
            }
            first = false;
            return;
        }
#pragma unroll
        for (int tt = 0; tt < NTT; ++tt) {
            const int it = tb + 32 * tt + r32 + z;
            const int itc = min(it, nt_eff - 1);
            const double cs = col_scale(itc);
#pragma unroll
            for (int x0 = 0; x0 < 16; x0 += FB) {
                double2 o[FB];
#pragma unroll
                for (int x = 0; x < FB; ++x) o[x] = make_double2(0.0, 0.0);
                if (!first) {
#pragma unroll
                    for (int x = 0; x < FB; ++x) {
                        const int p = 8 * ((x0 + x) >> 2) + 4 * h2 + ((x0 + x) & 3);
                        const int I = I0 + 4 * (wave % WI) + (p >> 3), J = J0 + 8 * (wave / WI) + (p & 7);
                        o[x] = Pq[(int64_t(itc) * NI + min(I, NI - 1)) * NI + min(J, NI - 1)];
                    }
                }
#pragma unroll
                for (int x = 0; x < FB; ++x) {
                    const int p = 8 * ((x0 + x) >> 2) + 4 * h2 + ((x0 + x) & 3);
                    const int I = I0 + 4 * (wave % WI) + (p >> 3), J = J0 + 8 * (wave / WI) + (p & 7);
                    if (it < nt_eff && I < NI && J < NI)
                        Pq[(int64_t(it) * NI + I) * NI + J] =
                            make_double2(o[x].x + cs * double(acc[tt][0][x0 + x]),
                                         o[x].y + cs * double(acc[tt][1][x0 + x]));
                }
            }
            zero16(acc[tt][0]);
            zero16(acc[tt][1]);
        }
        first = false;
    };

    // stages run over (k, slab); the FP32 accumulators go to FP64 every GZ_FLUSH terms
    // k blocks [kb0, kb1) (all of them unless a partial range is set); a range that starts past k = 0
    // adds to P
    const int kend = d.kb1;
    int k = d.kb0, slab = 0, since = 0;
    first = k == 0;
    Blk blk = block_of(k);
    blk.g = gz + (gz_block(d, q0, q, k) >> 1);
    int nsl = (blk.KP + KS - 1) / KS;
    while (nsl == 0 && k + 1 < kend) {
        blk = next_block(blk, ++k);
        nsl = (blk.KP + KS - 1) / KS;
    }
    if constexpr (NBUF == 3) {
        // (k, slab, blk, nsl) is the load cursor, two stages ahead of the stage computed
        auto advance = [&]() {
            ++slab;
            while (slab >= nsl && k + 1 < kend) {
                blk = next_block(blk, ++k);
                slab = 0;
                nsl = (blk.KP + KS - 1) / KS;
            }
        };
        gload(blk, 0);
        lstore(0);
        advance();
        bool e1 = slab < nsl;  // stage s + 1 exists
        if (e1) {
            gload(blk, slab);
            lstore(1);
            advance();
        }
        __syncthreads();
        u32x4 z0[4];
        zform(0, 0, z0);
        int buf = 0;
        while (true) {
            const bool e2 = e1 && slab < nsl;  // stage s + 2 exists
            if (e2) gload(blk, slab);
            const int nb1 = buf == NBUF - 1 ? 0 : buf + 1, nb2 = nb1 == NBUF - 1 ? 0 : nb1 + 1;
            compute_stage3(buf, nb1, z0);
            since += KS;
            if (since >= GZ_FLUSH || !e1) {
                flush();
                since = 0;
            }
            if (!e1) break;
            if (e2) {
                lstore(nb2);
                advance();
            }
            __syncthreads();
            buf = nb1;
            e1 = e2;
        }
        return;
    }
    gload(blk, 0);
    lstore(0);
    __syncthreads();
    int buf = 0;
    while (true) {
        int k2 = k, s2 = slab + 1, n2 = nsl;
        Blk b2 = blk;
        while (s2 >= n2 && k2 + 1 < kend) {
            ++k2;
            s2 = 0;
            b2 = next_block(b2, k2);
            n2 = (b2.KP + KS - 1) / KS;
        }
        const bool more = s2 < n2;
        if (more) gload(b2, s2);
        compute_stage(buf);
        since += KS;
        if (since >= GZ_FLUSH || !more) {
            flush();
            since = 0;
        }
        if (!more) break;
        lstore(buf ^ 1);
        __syncthreads();
        buf ^= 1;
        k = k2;
        slab = s2;
        nsl = n2;
        blk = b2;
    }
}

template <int OCC, int KS, int WI, int NTT, int NBUF = 2, int PR = PREC_BF16X3>
__global__ __launch_bounds__(128 * WI, OCC) void k_polz(Dev d, int q0, const float2* __restrict__ M,
                                                        const uint32_t* __restrict__ gz,
                                                        double2* __restrict__ P, Order od, int t0, int ntc,
                                                        int nt_eff) {
    int qrel, r, c;
    if (!work_item(od, qrel, r, c)) return;
    polz_item<OCC, KS, WI, NTT, NBUF, PR>(d, q0, M, gz, P, qrel, r, c, t0, ntc, nt_eff);
}

// The persistent polarization's queue, built on the device (so that a captured call replays it):
// the items (qrel, r, c) of every q of the call, the q in decreasing cost (the padded K of their k blocks;
// equal costs keep the q order) and each q's items in row-major (r, c) order; part[x] is the first item
// whose preceding items cost at least x/8 of the total, part[0] = 0, part[8] = n; the 8 counters are
// cleared.  One work-group of 256 threads, nq <= 127.
__global__ __launch_bounds__(256) void k_polz_qbuild(Dev d, int q0, int nq, int wi4, int ntc, int* __restrict__ items,
                                                     int* __restrict__ part, int* __restrict__ counter) {
    __shared__ long long cost[128], cstart[128];
    __shared__ int cnt[128], order[128], istart[128];
    const int tid = threadIdx.x;
    if (tid < nq) {
        const int q = q0 + tid, NI = d.ni[q];
        long long c = 0;
        for (int k = d.kb0; k < d.kb1; ++k) {
            const int K = d.nb[k] * d.nb[d.kmq[int64_t(q) * d.nk + k]];
            c += (K + GZ_KPAD - 1) / GZ_KPAD * GZ_KPAD;
        }
        const int nblk = (NI + 15) / 16;
        int m = 0;
        for (int r = 0; r * wi4 < NI; ++r) m += (nblk - r * wi4 / 16) * ntc;
        cost[tid] = c;
        cnt[tid] = m;
    }
    __syncthreads();
    if (tid < nq) {
        int rank = 0;
        for (int u = 0; u < nq; ++u) rank += (cost[u] > cost[tid] || (cost[u] == cost[tid] && u < tid)) ? 1 : 0;
        order[rank] = tid;
    }
    __syncthreads();
    if (tid == 0) {
        long long cs = 0;
        int is = 0;
        for (int s = 0; s < nq; ++s) {
            const int t = order[s];
            cstart[s] = cs;
            istart[s] = is;
            cs += cost[t] * cnt[t];
            is += cnt[t];
        }
        cstart[nq] = cs;  // the total
        istart[nq] = is;  // n
    }
    __syncthreads();
    for (int s = 0; s < nq; ++s) {
        const int t = order[s], NI = d.ni[q0 + t];
        const int nblk = (NI + 15) / 16, nr = (NI + wi4 - 1) / wi4;
        for (int r = tid; r < nr; r += 256) {
            int base = istart[s];
            for (int rp = 0; rp < r; ++rp) base += (nblk - rp * wi4 / 16) * ntc;
            const int c0 = r * wi4 / 16 * ntc;
            for (int c = c0; c < nblk * ntc; ++c) items[base + c - c0] = (t << 24) | (r << 12) | c;
        }
    }
    if (tid >= 1 && tid < 8) {
        const long long th = cstart[nq] * tid / 8;
        int p = istart[nq];
        for (int s = 0; s < nq; ++s) {
            const int t = order[s];
            if (cnt[t] > 0 && cstart[s] + (long long)(cnt[t] - 1) * cost[t] >= th) {
                p = istart[s] + (th <= cstart[s] ? 0 : int((th - cstart[s] + cost[t] - 1) / cost[t]));
                break;
            }
        }
        part[tid] = p;
    }
    if (tid == 0) {
        part[0] = 0;
        part[8] = istart[nq];
    }
    if (tid < 8) counter[tid] = 0;
}

// Persistent form: a fixed set of work-groups (the CUs' worth) takes items from a device queue per XCD.
// k_polz_qbuild lists the call's working items (all q of the batch) in decreasing cost, cuts the list into 8
// contiguous parts of equal cost (one per XCD, so the items that share M rows stay on one L2) and a
// work-group on XCD x takes the next item of part x from counter x until the part is exhausted; every
// work-group leaves the loop when its part is empty.  items: qrel << 24 | r << 12 | c.
template <int OCC, int KS, int WI, int NTT, int NBUF = 2, int PR = PREC_BF16X3>
__global__ __launch_bounds__(128 * WI, OCC) void k_polz_queue(Dev d, int q0, const float2* __restrict__ M,
                                                              const uint32_t* __restrict__ gz,
                                                              double2* __restrict__ P, const int* __restrict__ items,
                                                              const int* __restrict__ part, int* __restrict__ counter,
                                                              int t0, int ntc, int nt_eff) {
    __shared__ int s_item;
    const int x = int(blockIdx.x & 7);
    const int n = part[x + 1] - part[x];
    while (true) {
        if (threadIdx.x == 0) {
            const int i = atomicAdd(&counter[x], 1);
            s_item = i < n ? items[part[x] + i] : -1;
        }
        __syncthreads();
        const int it = s_item;
        __syncthreads();  // s_item is read by all before the next item's write
        if (it < 0) return;
        polz_item<OCC, KS, WI, NTT, NBUF, PR>(d, q0, M, gz, P, it >> 24, (it >> 12) & 4095, it & 4095, t0, ntc,
                                              nt_eff);
        __syncthreads();  // the item's LDS reads are done before the next item stages into LDS
    }
}

// =================================================================================================
// pair-space self-energy (vZ)
// =================================================================================================
// With the Hermitian part H of W~ and the pair product Z_K,IJ = M^I_K conj(M^J_K) of the polarization,
//     Re sum_IJ conj(a_I) W~_IJ a_J = sum_{I <= J} c_IJ (Re H_IJ Re Z_IJ + Im H_IJ Im Z_IJ),
// with a = column K of M, c_IJ = 2 above the diagonal and 1 on it (conj(a_I) a_J = conj(Z_IJ); the
// anti-Hermitian part of W~ adds only an imaginary amount).  Hence
//     Sigma_n(k,tau) = s sum_m G_m(k-q,tau) sum_pairs [Re Z w_re + Im Z w_im](K, tau),  w = c H,
// a real GEMM with rows = K, reduction = (pair, re/im) and columns = tau.  The weights are cut into
// blocks of 8 I x 8 J pairs (upper triangle of blocks), stored as bf16 hi/lo planes; a work-group
// keeps one weight block in LDS at a time and all its waves reuse it for 64 rows K each.
constexpr int SZ_WR = 64 + 4;  // LDS row stride of a weight block (u32): 8 steps x 8 pairs + pad
// weight blocks between two epilogues (32 blocks: 4096 terms per FP32 accumulator; 128 blocks would
// save 3.6% of the time at NI = 700 but double Sigma's error at the full shapes)
constexpr int SZ_FLUSH_BLOCKS = 32;

__device__ __host__ __forceinline__ int sz_nb8(int ni) { return (ni + 7) / 8; }
__device__ __host__ __forceinline__ int64_t sz_blocks(int ni) {
    const int n = sz_nb8(ni);
    return int64_t(n) * (n + 1) / 2;
}
// u32 elements of the weight planes of one q (hi and lo)
__device__ __host__ __forceinline__ int64_t sz_wq(int ni, int ntau) {
    return 2 * sz_blocks(ni) * gz_tp(ntau) * 64;
}
// fp32 transposed M of q0..q0+nq-1, [k][K][NIp8] complex, NIp8 = NI rounded up to 8
__device__ __host__ __forceinline__ int sz_np8(int ni) { return (ni + 7) / 8 * 8; }

// transposed FP32 M of one q: mt[k][K][NIp8], zero-padded in I (F16X3: scaled by 2^e_m(q))
template <int PR>
__global__ __launch_bounds__(256) void k_trans32(Dev d, int q0, int q, const float2* __restrict__ M,
                                                 float2* __restrict__ mt) {
    __shared__ float2 tile[32][33];
    const int nk = d.nk, k = d.kb0 + int(blockIdx.y);
    const int NI = d.ni[q], NP = sz_np8(NI);
    const int Kk = d.nb[k] * d.nb[d.kmq[q * nk + k]];
    const int nti = (NP + 31) / 32;
    const int i0 = (blockIdx.x % nti) * 32, c0 = (blockIdx.x / nti) * 32;
    if (c0 >= Kk) return;
    const float2* A = M + (d.mpre[q] - d.mpre[q0]) + d.moff[q * nk + k];
    int64_t ob = 0;
    for (int qq = q0; qq < q; ++qq) ob += (d.mpre[qq + 1] - d.mpre[qq]) / d.ni[qq] * sz_np8(d.ni[qq]);
    float2* T = mt + ob + d.moff[q * nk + k] / NI * NP;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const float fm = PR == PREC_F16X3 ? ldexpf(1.f, f16_exp_m(d.mx_m[q])) : 1.f;
    for (int r = ty; r < 32; r += 8) {
        const int I = i0 + r, col = c0 + tx;
        float2 a = (I < NI && col < Kk) ? A[int64_t(I) * Kk + col] : make_float2(0.f, 0.f);
        if constexpr (PR == PREC_F16X3) {
            a.x *= fm;
            a.y *= fm;
        }
        tile[r][tx] = a;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int col = c0 + r, I = i0 + tx;
        if (col < Kk && I < NP) T[int64_t(col) * NP + I] = tile[tx][r];
    }
}

// weight blocks of one q: for block (bi, bj), bj >= bi, tau row t and step s (I = 8 bi + s), the
// 8 pairs J = 8 bj + j hold (w_re, w_im) = c_IJ (Re H_IJ, Im H_IJ) as packed bf16 (f16 for F16X3,
// scaled by 2^e_w(q, tau)), hi and lo planes.  mxw: the maxima of W~ of this q per tau (F16X3).
template <int PR>
__global__ __launch_bounds__(256) void k_wpair(const double2* __restrict__ W, int NI, int ntau,
                                               const unsigned long long* __restrict__ mxw,
                                               uint32_t* __restrict__ wz) {
    const int TP = gz_tp(ntau), nb = sz_nb8(NI);
    const int64_t nblk = sz_blocks(NI);
    const int64_t id = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (id >= nblk * TP * 64) return;
    const int j = int(id & 7), s = int((id >> 3) & 7);
    const int64_t bt = id >> 6;
    const int t = int(bt % TP);
    int64_t b = bt / TP;
    int bi = 0;  // block b -> (bi, bj): rows of the upper triangle of blocks, bi ascending
    while (b >= nb - bi) {
        b -= nb - bi;
        ++bi;
    }
    const int bj = bi + int(b);
    const int I = 8 * bi + s, J = 8 * bj + j;
    float re = 0.f, im = 0.f;
    if (t < ntau && I < NI && J < NI && J >= I) {
        const double2* Wt = W + int64_t(t) * NI * NI;
        const double2 a = Wt[int64_t(I) * NI + J], m = Wt[int64_t(J) * NI + I];
        // c_IJ H_IJ = c_IJ (W_IJ + conj W_JI) / 2
        const double c = (J > I ? 1.0 : 0.5) * (PR == PREC_F16X3 ? ldexp(1.0, f16_exp_w(mxw[t])) : 1.0);
        re = float(c * (a.x + m.x));
        im = J > I ? float(c * (a.y - m.y)) : 0.f;
    }
    uint32_t h, l;
    split_pair<PR>(re, im, h, l);
    const int64_t blk = id >> 6;  // (block, tau) row of 64 u32
    wz[blk * 64 + 8 * s + j] = h;
    wz[nblk * TP * 64 + blk * 64 + 8 * s + j] = l;
}

// Work-group = 8 waves over 512 rows K of one (q, k) block and one tau chunk of NTT 32-wide tiles
// (three, or one or two for a tail chunk; the launch covers ntc chunks from tau t0); wave w owns
// rows K0 + 64 w .. + 63 as two 32-row MFMA tiles.  The work-group walks the weight blocks in order;
// each block (48 KB, hi and lo) is staged through LDS (double-buffered) while the previous one is
// used.  Every lane forms Z for its rows K and 4 pairs per MFMA step from the transposed FP32 M
// (the 8 values a_I of the block row stay in registers across the block row), splits it into
// hi/lo halves (bf16 or f16), and the FP32 accumulators go through the epilogue (G_m weight, sum over
// the m of each band n, FP64 atomic) every SZ_FLUSH_BLOCKS blocks.
template <int OCC, int NTT, int PR = PREC_BF16X3>
__device__ __forceinline__ void sigz_item(const Dev& d, int q0, const double* __restrict__ G,
                                          const float2* __restrict__ mt, const uint32_t* __restrict__ wz,
                                          double* __restrict__ Sig, int t0, int qrel, int k, int kc, int tc) {
    constexpr int CW = 32 * NTT;
    __shared__ uint32_t Ws[2][2][CW][SZ_WR];  // [buffer][hi, lo][tau][8 s x 8 j]
    // a_I, I = 8 bi .. 8 bi + 7, of each thread's second row K: a slot per thread, written and read by
    // that thread only (it frees the registers that hold the weight fragments one tau tile ahead)
    __shared__ float2 As1[8][512];
    const int nk = d.nk, ntau = d.ntau, nbmax = d.nbmax;
    const int TP = gz_tp(ntau);
    // work item: (q, k, K chunk of 512, tau chunk)
    const int q = q0 + qrel;
    const int kq = d.kmq[q * nk + k];
    const int nm = d.nb[kq], Kk = d.nb[k] * nm;
    const int K0 = kc * 512;
    if (K0 >= Kk) return;  // uniform
    const int NI = d.ni[q], NP = sz_np8(NI), nb = sz_nb8(NI);
    const int64_t nblk = sz_blocks(NI);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r32 = lane & 31, h2 = lane >> 5;
    const int tb = t0 + CW * tc;  // first tau of the chunk

    int64_t mq = 0, wq = 0;
    for (int qq = q0; qq < q; ++qq) {
        mq += (d.mpre[qq + 1] - d.mpre[qq]) / d.ni[qq] * sz_np8(d.ni[qq]);
        wq += sz_wq(d.ni[qq], ntau);
    }
    const float2* T = mt + mq + d.moff[q * nk + k] / NI * NP;
    const uint32_t* wq0 = wz + wq;  // hi plane of q; the lo plane follows at nblk * TP * 64
    const int64_t wlo = nblk * TP * 64;

    // this lane's two rows K (one per 32-row tile); rows past Kk read row Kk - 1 and are masked in
    // the epilogue
    // byte offsets of the rows from the work-group's base T (uniform base + 32-bit lane offset)
    uint32_t trow[2];
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
        trow[kt] = uint32_t(min(K0 + 64 * wave + 32 * kt + r32, Kk - 1)) * uint32_t(NP * sizeof(float2));
    const char* Tb = reinterpret_cast<const char*>(T);

    // staging of one plane (hi or lo) of a weight block: CW tau x 16 chunks of 16 B, NTT per thread;
    // the two planes of the next block are loaded in the two halves of the current one
    u32x4 rw[NTT];
    auto wload = [&](int64_t b, int pl) {
        // the chunk's CW tau rows of 64 u32 are contiguous: chunk id sits at 16 id bytes
        const char* src = reinterpret_cast<const char*>(wq0 + (pl * wlo + (b * TP + tb) * 64));
#pragma unroll
        for (int i = 0; i < NTT; ++i)
            rw[i] = *reinterpret_cast<const u32x4*>(src + (uint32_t(16 * tid) + uint32_t(8192 * i)));
    };
    auto wstore = [&](int buf, int pl) {
#pragma unroll
        for (int i = 0; i < NTT; ++i) {
            const int id = tid + 512 * i;
            const int t = id >> 4, ch = id & 15;
            *reinterpret_cast<u32x4*>(&Ws[buf][pl][t][4 * ch]) = rw[i];
        }
    };

    floatx16 acc[2][NTT];
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
        for (int tt = 0; tt < NTT; ++tt) zero16(acc[kt][tt]);

    const double sc = d.scale;
    // F16X3: the transposed M carries 2^e_m (k_trans32) and the weights 2^e_w(q, tau) (k_wpair)
    const int em2 = PR == PREC_F16X3 ? 2 * f16_exp_m(d.mx_m[q]) : 0;
    // epilogue on the accumulators: weight each row K = (n, m) by G_m(k-q, tau), sum the rows of
    // each band n and add to Sigma_n(k, tau)
    const double* Gq = G + int64_t(kq) * nbmax * ntau;  // G_m(k - q, tau) = Gq[m * ntau + tau]
    auto flush = [&]() {
        int z = 0;  // opaque zero: keeps the loop-invariant G loads of this epilogue out of the loop
        asm volatile("" : "+v"(z));
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            const int kb = K0 + 64 * wave + 32 * kt;  // first row of the tile (wave-uniform)
            if (kb >= Kk) continue;
            const int nlo = kb / nm, nhi = (min(kb + 32, Kk) - 1) / nm;
#pragma unroll
            for (int tt = 0; tt < NTT; ++tt) {
                const int it = tb + 32 * tt + r32;
                const int itc = min(it, ntau - 1);
                double cs = sc;
                if constexpr (PR == PREC_F16X3) cs = ldexp(sc, -(em2 + f16_exp_w(d.mx_w[q * ntau + itc])));
                for (int nx = nlo; nx <= nhi; ++nx) {
                    // the 16 weights are loaded together from clamped (always valid) rows m, so the
                    // epilogue waits once per band instead of once per element
                    float gw[16];
#pragma unroll
                    for (int x = 0; x < 16; ++x) {
                        const int K = kb + 8 * (x >> 2) + 4 * h2 + (x & 3);
                        const int m = min(max(K - nx * nm, 0), nm - 1);
                        gw[x] = float(Gq[m * ntau + itc + z]);
                    }
                    float v = 0.f;  // 16 terms; the run totals are summed in FP64
#pragma unroll
                    for (int x = 0; x < 16; ++x) {
                        const int K = kb + 8 * (x >> 2) + 4 * h2 + (x & 3);
                        if (K < Kk && K / nm == nx) v += acc[kt][tt][x] * gw[x];
                    }
                    v += __shfl_xor(v, 32);
                    if (h2 == 0 && it < ntau)
                        atomicAdd(&Sig[(int64_t(k) * nbmax + nx) * ntau + it], cs * double(v));
                }
                zero16(acc[kt][tt]);
            }
        }
    };

    float4 ai[4];      // a_I, I = 8 bi .. 8 bi + 7, of the first row (re, im pairs in float4); the
                       // second row's are in As1
    float4 aj[2][2];   // a_J, J = 8 bj + 4 h2 .. + 3
    auto load_ai = [&](int bi) {
        float4 a1[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            ai[e] = *reinterpret_cast<const float4*>(Tb + (trow[0] + uint32_t(64 * bi + 16 * e)));
            a1[e] = *reinterpret_cast<const float4*>(Tb + (trow[1] + uint32_t(64 * bi + 16 * e)));
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            As1[2 * e][tid] = make_float2(a1[e].x, a1[e].y);
            As1[2 * e + 1][tid] = make_float2(a1[e].z, a1[e].w);
        }
    };
    // the hi and lo weight fragments of MFMA step s, tau tile tt
    auto bload = [&](int bf, int s, int tt, u32x4& bh, u32x4& bl) {
        bh = reinterpret_cast<const u32x4*>(&Ws[bf][0][32 * tt + r32][0])[2 * s + h2];
        bl = reinterpret_cast<const u32x4*>(&Ws[bf][1][32 * tt + r32][0])[2 * s + h2];
    };
    auto load_aj = [&](int bj, float4 (&dst)[2][2]) {
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
#pragma unroll
            for (int e = 0; e < 2; ++e)
                dst[kt][e] =
                    *reinterpret_cast<const float4*>(Tb + (trow[kt] + uint32_t(64 * bj + 32 * h2 + 16 * e)));
    };

    int bi = 0, bj = 0;
    float4 ajn[2][2];  // a_J of the next block, loaded one block ahead
    load_ai(0);
    load_aj(0, aj);
    wload(0, 0);
    wstore(0, 0);
    wload(0, 1);
    wstore(0, 1);
    __syncthreads();
    int buf = 0;
    int64_t b = 0;
    // blocks in runs of SZ_FLUSH_BLOCKS (128 terms each per FP32 accumulator), each run followed by the
    // epilogue
    while (b < nblk) {
        const int64_t bend = b + SZ_FLUSH_BLOCKS < nblk ? b + SZ_FLUSH_BLOCKS : nblk;
        for (; b < bend; ++b) {
            int bi2 = bi, bj2 = bj + 1;
            if (bj2 >= nb) {
                ++bi2;
                bj2 = bi2;
            }
            const bool more = b + 1 < nblk;
            // the next block's a_J and weights are in flight while this block computes
            if (more) {
                load_aj(bj2, ajn);
                wload(b + 1, 0);
            }
            // 8 MFMA steps: step s pairs I = 8 bi + s with J = 8 bj + 4 h2 .. + 3 (this lane's half).
            // The weight fragments of the next tau tile (of the next step's first tile after the last)
            // are read from LDS before the MFMAs of the current one, and the second row's a_I of the
            // next step during the current step.
            float2 a1 = As1[0][tid];
            u32x4 bh, bl;
            bload(buf, 0, 0, bh, bl);
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                if (s == 4 && more) {  // the other buffer is not read in this block
                    wstore(buf ^ 1, 0);
                    wload(b + 1, 1);
                }
                u32x4 zh[2], zl[2];
#pragma unroll
                for (int kt = 0; kt < 2; ++kt) {
                    float ar, aim;
                    if (kt == 0) {
                        const float4 a4 = ai[s >> 1];
                        ar = (s & 1) ? a4.z : a4.x;
                        aim = (s & 1) ? a4.w : a4.y;
                    } else {
                        ar = a1.x;
                        aim = a1.y;
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float4 c4 = aj[kt][j >> 1];
                        const float cr = (j & 1) ? c4.z : c4.x, ci = (j & 1) ? c4.w : c4.y;
                        const float zr = ar * cr + aim * ci, zi = aim * cr - ar * ci;
                        uint32_t h, l;
                        split_pair<PR>(zr, zi, h, l);
                        zh[kt][j] = h;
                        zl[kt][j] = l;
                    }
                }
                if (s < 7) a1 = As1[s + 1][tid];
#pragma unroll
                for (int tt = 0; tt < NTT; ++tt) {
                    u32x4 bhn, bln;
                    if (tt + 1 < NTT) bload(buf, s, tt + 1, bhn, bln);
                    else if (s < 7) bload(buf, s + 1, 0, bhn, bln);
                    // the reads above are issued before these MFMAs
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int kt = 0; kt < 2; ++kt) {
                        acc[kt][tt] = mfma32p<PR>(zh[kt], bh, acc[kt][tt]);
                        acc[kt][tt] = mfma32p<PR>(zh[kt], bl, acc[kt][tt]);
                        acc[kt][tt] = mfma32p<PR>(zl[kt], bh, acc[kt][tt]);
                    }
                    if (tt + 1 < NTT || s < 7) {
                        bh = bhn;
                        bl = bln;
                    }
                }
                // keeps the Z of later steps from being formed (and held) ahead of time
                __builtin_amdgcn_sched_barrier(0);
            }
            if (!more) break;
#pragma unroll
            for (int kt = 0; kt < 2; ++kt) {
                aj[kt][0] = ajn[kt][0];
                aj[kt][1] = ajn[kt][1];
            }
            if (bi2 != bi) load_ai(bi2);  // once per row of blocks
            wstore(buf ^ 1, 1);
            __syncthreads();
            buf ^= 1;
            bi = bi2;
            bj = bj2;
        }
        flush();
        if (b + 1 >= nblk && b < bend) break;  // the last block was handled inside the run
    }
}

template <int OCC, int NTT, int PR = PREC_BF16X3>
__global__ __launch_bounds__(512, OCC) void k_sigz(Dev d, int q0, const double* __restrict__ G,
                                                   const float2* __restrict__ mt,
                                                   const uint32_t* __restrict__ wz,
                                                   double* __restrict__ Sig, int nkc, int t0, int ntc) {
    int w = blockIdx.x;
    const int tc = w % ntc;
    w /= ntc;
    const int kc = w % nkc;
    w /= nkc;
    const int nkr = d.kb1 - d.kb0;
    sigz_item<OCC, NTT, PR>(d, q0, G, mt, wz, Sig, t0, w / nkr, d.kb0 + w % nkr, kc, tc);
}

// Persistent form, as k_polz_queue: items qrel << 24 | k << 16 | kc << 8 | tc from per-XCD queues.
template <int OCC, int NTT, int PR = PREC_BF16X3>
__global__ __launch_bounds__(512, OCC) void k_sigz_queue(Dev d, int q0, const double* __restrict__ G,
                                                         const float2* __restrict__ mt,
                                                         const uint32_t* __restrict__ wz, double* __restrict__ Sig,
                                                         const int* __restrict__ items, const int* __restrict__ part,
                                                         int* __restrict__ counter, int t0) {
    __shared__ int s_item;
    const int x = int(blockIdx.x & 7);
    const int n = part[x + 1] - part[x];
    while (true) {
        if (threadIdx.x == 0) {
            const int i = atomicAdd(&counter[x], 1);
            s_item = i < n ? items[part[x] + i] : -1;
        }
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it < 0) return;
        sigz_item<OCC, NTT, PR>(d, q0, G, mt, wz, Sig, t0, it >> 24, (it >> 16) & 255, (it >> 8) & 255, it & 255);
        __syncthreads();
    }
}

// =================================================================================================
// variants (tile shapes) and dispatch
// =================================================================================================
using PolFn = void (*)(const Dev&, const Host&, hipStream_t, int, int, const void*, const double*, void*);
using SigFn = void (*)(const Dev&, const Host&, hipStream_t, int, int, const void*, const double*,
                       const char*, int64_t, void*);

template <int WI, int WJ, int T, int PREC, bool PF = false>
void run_pol(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
             const double* G, void* P) {
    int maxi = 0;
    for (int q = q0; q < q0 + nq; ++q) maxi = std::max(maxi, h.ni[q]);
    const int ntI = ceil_div(maxi, 16 * WI), ntJ = ceil_div(maxi, 16 * WJ), ntG = ceil_div(h.ntau, T);
    const Order od = make_order(ntG * ntI, ntJ, nq);
    launch_order(od, 64, [&](dim3 g, const Order& o) {
        MSGW_LAUNCH((k_pol<WI, WJ, T, PREC, PF>), g, dim3(64), 0, s, d, q0, (const float2*)M, G,
                           (double2*)P, o, ntI);
    });
}

template <int WI, int WJ, int T, int PREC>
void run_sig(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
             const double* G, const char* wsc, int64_t plane, void* Sig) {
    int maxi = 0, maxc = 0;
    for (int q = q0; q < q0 + nq; ++q) {
        maxi = std::max(maxi, h.ni[q]);
        for (int k = 0; k < h.nk; ++k)
            maxc = std::max(maxc, h.nb[k] * h.nb[h.kmq[size_t(q) * h.nk + k]]);
    }
    static_assert(16 * WI <= PAD, "row tiles must fit in the padded W~ planes");
    const int ntI = ceil_div(maxi, 16 * WI), ntC = ceil_div(maxc, 16 * WJ), ntG = ceil_div(h.ntau, T);
    const Order od = make_order(ntG * ntI, h.nk * ntC, nq);
    launch_order(od, 64, [&](dim3 g, const Order& o) {
        MSGW_LAUNCH((k_sig<WI, WJ, T, PREC>), g, dim3(64), 0, s, d, q0, (const float2*)M, G, wsc,
                           plane, (double*)Sig, o, ntI, ntC);
    });
}

using Sig3Fn = void (*)(const Dev&, const Host&, hipStream_t, int, int, const void*, const double*,
                        const char*, int64_t, const uint32_t*, int64_t, void*);

// bf16 elements of the g planes of q0..q0+nq-1
int64_t gz_elems(const Host& h, int q0, int nq) {
    int64_t n = 0;
    for (int q = q0; q < q0 + nq; ++q)
        for (int k = 0; k < h.nk; ++k) {
            const int K = h.nb[k] * h.nb[h.kmq[size_t(q) * h.nk + k]];
            n += int64_t(2) * gz_tp(h.ntau) * round_up(K, GZ_KPAD);
        }
    return n;
}

template <int OCC, int SR, int SC, int KS = GZ_KS, int WI = 2, int NBUF = 2, int PR = PREC_BF16X3, bool QUEUE = false>
void run_polz(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
              const double* G, void* P) {
    int maxi = 0, maxk = 0;
    for (int q = q0; q < q0 + nq; ++q) {
        maxi = std::max(maxi, h.ni[q]);
        for (int k = 0; k < h.nk; ++k)
            maxk = std::max(maxk, h.nb[k] * h.nb[h.kmq[size_t(q) * h.nk + k]]);
    }
    if (size_t(gz_elems(h, q0, nq)) * 2 > scratch_mfma_bytes(d, h))
        throw Error(MSGW_ENOMEM, "workspace too small for the g planes");
    // the kernel addresses one block's M rows and g planes with 32-bit byte offsets
    if (int64_t(maxi) * maxk * 8 >= (int64_t(1) << 32) ||
        int64_t(2) * gz_tp(h.ntau) * round_up(maxk, GZ_KPAD) * 2 >= (int64_t(1) << 31))
        throw Error(MSGW_ENOTSUP, "a (q, k) block too large for the pair-space polarization");
    uint32_t* gz = reinterpret_cast<uint32_t*>(scratch_mfma(d, h));
    const unsigned gx = unsigned(ceil_div(gz_tp(h.ntau) * round_up(maxk, GZ_KPAD) / 2, 256));
    if (PR == PREC_F16X3 && !d.kreuse) {
        launch_scales(d, h, s, q0, nq, M, nullptr);
        MSGW_LAUNCH(k_gmax, dim3(ceil_div(int64_t(h.nk) * h.ntau, 256)), dim3(256), 0, s, d, G);
        MSGW_LAUNCH(k_gexp, dim3(ceil_div(int64_t(nq) * h.ntau, 256)), dim3(256), 0, s, d, q0, nq);
        MSGW_HIP(hipGetLastError());
    }
    for (int q = q0; q < q0 + nq && !d.kreuse; ++q) {
        MSGW_LAUNCH(k_gtab<PR>, dim3(gx, h.nk), dim3(256), 0, s, d, q, G, gz + gz_elems(h, q0, q - q0) / 2);
        MSGW_HIP(hipGetLastError());
    }
    // tau in chunks of three 32-wide tiles, the last chunk with the one or two tiles left; with the
    // tau mirror only the points i <= (N - 1) / 2 (the others are copied afterwards)
    const int nt_eff = tau_points_computed(d, h);
    const int ntiles = ceil_div(nt_eff, 32), n3 = ntiles / 3, rest = ntiles % 3;
    auto launch = [&](auto kern, int t0, int ntc) {
        const Order od = make_order_st(ceil_div(maxi, 4 * WI), ceil_div(maxi, 16) * ntc, nq, SR, SC * ntc);
        // row r (4 WI rows I from I0) works on the 16-wide column blocks cj with J0 < NI and J0 + 16 > I0
        auto rows = [&](int qrel, int r, int& lo, int& hi) {
            const int NI = h.ni[q0 + qrel], I0 = r * 4 * WI;
            lo = I0 / 16 * ntc;
            hi = I0 < NI ? ceil_div(NI, 16) * ntc : lo;
        };
        launch_order(od, 128 * WI, [&](dim3 g, const Order& o) {
            MSGW_LAUNCH(kern, g, dim3(128 * WI), 0, s, d, q0, (const float2*)M, (const uint32_t*)gz, (double2*)P, o,
                        t0, ntc, nt_eff);
        }, rows);
    };
    // the persistent form: the call's working items in decreasing cost (the k blocks' padded K of their
    // q), cut into 8 contiguous parts of equal cost, one queue per XCD in the scratch after the g planes
    const size_t gz_bytes = size_t(gz_elems(h, q0, nq)) * 2;
    auto launch_queue = [&](auto kern, int t0, int ntc) {
        if (nq > 127) throw Error(MSGW_ENOTSUP, "the polarization's work queue takes at most 127 q per call");
        // the item count (k_polz_qbuild lists them): row r holds the column blocks from r * 4 WI / 16 on
        size_t n = 0;
        for (int qrel = 0; qrel < nq; ++qrel) {
            const int NI = h.ni[q0 + qrel], nblk = ceil_div(NI, 16);
            for (int r = 0; r * 4 * WI < NI; ++r) n += size_t(nblk - r * 4 * WI / 16) * ntc;
        }
        if (n == 0) return;
        // [items (n)] [part (9)] [pad] [counters (8)]
        const size_t off_cnt = size_t(round_up(int(n + 9), 2));
        const size_t bytes = sizeof(int) * (off_cnt + 8);
        if (gz_bytes + 256 + bytes > scratch_mfma_bytes(d, h))
            throw Error(MSGW_ENOMEM, "workspace too small for the polarization's work queue");
        int* dev = reinterpret_cast<int*>(scratch_mfma(d, h) + scratch_al(gz_bytes));
        MSGW_LAUNCH(k_polz_qbuild, dim3(1), dim3(256), 0, s, d, q0, nq, 4 * WI, ntc, dev, dev + n, dev + off_cnt);
        int dev_id = 0, cus = 0;
        MSGW_HIP(hipGetDevice(&dev_id));
        MSGW_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id));
        const unsigned grid = unsigned(8 * ceil_div(cus, 8) * OCC);
        MSGW_LAUNCH(kern, dim3(grid), dim3(128 * WI), 0, s, d, q0, (const float2*)M, (const uint32_t*)gz, (double2*)P,
                    dev, dev + n, dev + off_cnt, t0, ntc, nt_eff);
        MSGW_HIP(hipGetLastError());
    };
    record_kernel_event(d, MSGW_OP_POLARIZATION, false, s);
    if constexpr (QUEUE) {
        if (n3 > 0) launch_queue(k_polz_queue<OCC, KS, WI, 3, NBUF, PR>, 0, n3);
        if (rest == 1) launch_queue(k_polz_queue<OCC, KS, WI, 1, NBUF, PR>, 96 * n3, 1);
        if (rest == 2) launch_queue(k_polz_queue<OCC, KS, WI, 2, NBUF, PR>, 96 * n3, 1);
    } else {
        if (n3 > 0) launch(k_polz<OCC, KS, WI, 3, NBUF, PR>, 0, n3);
        if (rest == 1) launch(k_polz<OCC, KS, WI, 1, NBUF, PR>, 96 * n3, 1);
        if (rest == 2) launch(k_polz<OCC, KS, WI, 2, NBUF, PR>, 96 * n3, 1);
    }
    record_kernel_event(d, MSGW_OP_POLARIZATION, true, s);
}

// pair-space self-energy: needs only the raw W~ (FP64), so it runs its own conversions
template <int PR, bool QUEUE = false>
void run_sigz(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
              const double* G, const void* W, void* Sig) {
    int64_t nmt = 0, nwz = 0;
    int maxk = 0;
    for (int q = q0; q < q0 + nq; ++q) {
        nmt += (h.mpre[q + 1] - h.mpre[q]) / h.ni[q] * sz_np8(h.ni[q]);
        nwz += sz_wq(h.ni[q], h.ntau);
        for (int k = 0; k < h.nk; ++k) maxk = std::max(maxk, h.nb[k] * h.nb[h.kmq[size_t(q) * h.nk + k]]);
    }
    if (size_t(nmt) * 8 + size_t(nwz) * 4 > scratch_mfma_bytes(d, h))
        throw Error(MSGW_ENOMEM, "workspace too small for the pair-space self-energy");
    float2* mt = reinterpret_cast<float2*>(scratch_mfma(d, h));
    uint32_t* wz = reinterpret_cast<uint32_t*>(mt + nmt);
    if (PR == PREC_F16X3 && !d.kreuse) launch_scales(d, h, s, q0, nq, M, W);
    int64_t woff = 0;
    for (int q = q0; q < q0 + nq; ++q) {
        const int NI = h.ni[q];
        const unsigned gx = ceil_div(sz_np8(NI), 32) * ceil_div(maxk, 32);
        MSGW_LAUNCH(k_trans32<PR>, dim3(gx, d.kb1 - d.kb0), dim3(256), 0, s, d, q0, q, (const float2*)M, mt);
        MSGW_HIP(hipGetLastError());
        const int64_t n = sz_blocks(NI) * gz_tp(h.ntau) * 64;
        if (!d.kreuse) {
            MSGW_LAUNCH(k_wpair<PR>, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, s,
                        (const double2*)W + (h.ppre[q] - h.ppre[q0]), NI, h.ntau,
                        (const unsigned long long*)(d.mx_w + int64_t(q) * h.ntau), wz + woff);
            MSGW_HIP(hipGetLastError());
        }
        woff += sz_wq(NI, h.ntau);
    }
    // tau in chunks of three 32-wide tiles, the last chunk with the one or two tiles left
    const int nkc = ceil_div(maxk, 512), ntiles = ceil_div(h.ntau, 32), n3 = ntiles / 3, rest = ntiles % 3;
    auto launch = [&](auto kern, int t0, int ntc) {
        MSGW_LAUNCH(kern, dim3(ceil_div(int64_t(nq) * (d.kb1 - d.kb0) * nkc * ntc, 1)), dim3(512), 0, s, d, q0, G,
                    (const float2*)mt, (const uint32_t*)wz, (double*)Sig, nkc, t0, ntc);
        MSGW_HIP(hipGetLastError());
    };
    // the persistent form: items in decreasing cost (weight blocks x rows of the K chunk), 8 parts of
    // equal cost, in the scratch after the transposed M and the weight blocks
    const size_t used = scratch_al(size_t(nmt) * 8 + size_t(nwz) * 4);
    auto launch_queue = [&](auto kern, int t0, int ntc) {
        // the queue is built on the host and uploaded, which a captured graph could not replay
        hipStreamCaptureStatus capturing = hipStreamCaptureStatusNone;
        MSGW_HIP(hipStreamIsCapturing(s, &capturing));
        if (capturing != hipStreamCaptureStatusNone)
            throw Error(MSGW_ENOTSUP, "the persistent self-energy variant cannot be captured in a graph");
        static thread_local std::vector<int> host;  // refilled only after its previous upload has run
        static thread_local hipEvent_t uploaded = nullptr;
        if (uploaded) MSGW_HIP(hipEventSynchronize(uploaded));
        else MSGW_HIP(hipEventCreateWithFlags(&uploaded, hipEventDisableTiming));
        if (nq > 127) throw Error(MSGW_ENOTSUP, "the self-energy's work queue takes at most 127 q per call");
        std::vector<std::pair<int64_t, int>> it;
        for (int qrel = 0; qrel < nq; ++qrel) {
            const int q = q0 + qrel;
            for (int k = d.kb0; k < d.kb1; ++k) {
                const int Kk = h.nb[k] * h.nb[h.kmq[size_t(q) * h.nk + k]];
                for (int kc = 0; kc * 512 < Kk; ++kc)
                    for (int tc = 0; tc < ntc; ++tc)
                        it.push_back({int64_t(std::min(512, Kk - kc * 512)) * sz_blocks(h.ni[q]),
                                      (qrel << 24) | (k << 16) | (kc << 8) | tc});
            }
        }
        if (it.empty()) return;
        std::stable_sort(it.begin(), it.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
        int64_t total = 0;
        for (const auto& e : it) total += e.first;
        const size_t n = it.size(), off_cnt = round_up(int(n + 9), 2);
        host.assign(off_cnt + 8, 0);
        int x = 1;
        int64_t run = 0;
        for (size_t i = 0; i < n; ++i) {
            host[i] = it[i].second;
            while (x < 8 && run >= total * x / 8) host[n + x++] = int(i);
            run += it[i].first;
        }
        while (x < 8) host[n + x++] = int(n);
        host[n + 8] = int(n);
        const size_t bytes = sizeof(int) * host.size();
        if (used + bytes > scratch_mfma_bytes(d, h))
            throw Error(MSGW_ENOMEM, "workspace too small for the self-energy's work queue");
        int* dev = reinterpret_cast<int*>(scratch_mfma(d, h) + used);
        MSGW_HIP(hipMemcpyAsync(dev, host.data(), bytes, hipMemcpyHostToDevice, s));
        MSGW_HIP(hipEventRecord(uploaded, s));
        MSGW_LAUNCH(k_fill_u64, dim3(1), dim3(256), 0, s, reinterpret_cast<unsigned long long*>(dev + off_cnt), 4);
        int dev_id = 0, cus = 0;
        MSGW_HIP(hipGetDevice(&dev_id));
        MSGW_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id));
        MSGW_LAUNCH(kern, dim3(unsigned(8 * ceil_div(cus, 8))), dim3(512), 0, s, d, q0, G, (const float2*)mt,
                    (const uint32_t*)wz, (double*)Sig, dev, dev + n, dev + off_cnt, t0);
        MSGW_HIP(hipGetLastError());
    };
    record_kernel_event(d, MSGW_OP_SELF_ENERGY, false, s);
    if constexpr (QUEUE) {
        if (n3 > 0) launch_queue(k_sigz_queue<1, 3, PR>, 0, n3);
        if (rest == 1) launch_queue(k_sigz_queue<1, 1, PR>, 96 * n3, 1);
        if (rest == 2) launch_queue(k_sigz_queue<1, 2, PR>, 96 * n3, 1);
    } else {
        if (n3 > 0) launch(k_sigz<1, 3, PR>, 0, n3);
        if (rest == 1) launch(k_sigz<1, 1, PR>, 96 * n3, 1);
        if (rest == 2) launch(k_sigz<1, 2, PR>, 96 * n3, 1);
    }
    record_kernel_event(d, MSGW_OP_SELF_ENERGY, true, s);
}

template <int T, int SR = 4, int SC = 8, int OCC = 1>
void run_sig7(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
              const double* G, const char* wsc, int64_t plane, const uint32_t* mt, int64_t mtplane,
              void* Sig) {
    int maxi = 0, maxc = 0;
    for (int q = q0; q < q0 + nq; ++q) {
        maxi = std::max(maxi, h.ni[q]);
        for (int k = 0; k < h.nk; ++k)
            maxc = std::max(maxc, h.nb[k] * h.nb[h.kmq[size_t(q) * h.nk + k]]);
    }
    static_assert(64 <= PAD, "row tiles must fit in the padded W~ planes");
    const int ntI = ceil_div(maxi, 64), ntC = ceil_div(maxc, 128), ntG = ceil_div(h.ntau, T);
    const Order od = make_order_st(ntG * ntI, h.nk * ntC, nq, SR, SC);
    launch_order(od, 256, [&](dim3 g, const Order& o) {
        MSGW_LAUNCH((k_sig7<T, OCC>), g, dim3(256), 0, s, d, q0, (const float2*)M, G, wsc, plane, mt,
                           mtplane, (double*)Sig, o, ntI, ntC);
    });
}

struct PolVariant {
    const char* name;
    PolFn fn;
    bool ranged = false;  // honours a partial k range (pair space)
};
using SigZFn = void (*)(const Dev&, const Host&, hipStream_t, int, int, const void*, const double*,
                        const void*, void*);
struct SigVariant {
    const char* name;
    SigFn fn;      // W~ planes only
    Sig3Fn fn3;    // W~ planes + split transposed M
    SigZFn fnz = nullptr;  // raw W~ (runs its own conversions)
};

// index 0 of each table is the default (the fastest on the metric's 5x5x5-k, 128-band, NI = 700 shapes for
// F16X3; on the 4x4x4-k, 64-band, NI = 400 shapes for the others)
const PolVariant kPolBF16[] = {
    {"pair-space 16x16 pairs K64 st4x8 3-buffer", run_polz<1, 4, 8, 64, 4, 3>, true},
    {"pair-space 16x16 pairs K64 st4x8", run_polz<1, 4, 8, 64, 4>, true},
    {"pair-space 8x16 pairs 2 WG/CU st4x16 K64", run_polz<2, 4, 16, 64>, true},
    {"pair-space 8x16 pairs 2 WG/CU st4x16", run_polz<2, 4, 16>, true},
    {"WI2 WJ2 T2", run_pol<2, 2, 2, PREC_BF16X3>},
};
const PolVariant kPolF16[] = {
    {"pair-space 16x16 pairs K64 3-buffer persistent LPT queue", run_polz<1, 4, 8, 64, 4, 3, PREC_F16X3, true>, true},
    {"pair-space 16x16 pairs K64 st4x8 3-buffer", run_polz<1, 4, 8, 64, 4, 3, PREC_F16X3>, true},
    {"pair-space 16x16 pairs K64 st4x8", run_polz<1, 4, 8, 64, 4, 2, PREC_F16X3>, true},
    {"pair-space 8x16 pairs 2 WG/CU st4x16 K64", run_polz<2, 4, 16, 64, 2, 2, PREC_F16X3>, true},
    {"pair-space 8x16 pairs 2 WG/CU st4x16", run_polz<2, 4, 16, GZ_KS, 2, 2, PREC_F16X3>, true},
};
const PolVariant kPolFP32[] = {
    {"WI2 WJ2 T4", run_pol<2, 2, 4, PREC_FP32>},
    {"WI2 WJ2 T2", run_pol<2, 2, 2, PREC_FP32>},
};
const SigVariant kSigBF16[] = {
    {"pair-space 512 K x 8x8-pair blocks", nullptr, nullptr, run_sigz<PREC_BF16X3>},
    {"LDS 2-stage 64x128 T2 2 WG/CU st8x8", nullptr, run_sig7<2, 8, 8, 2>},
    {"WI2 WJ4 T4", run_sig<2, 4, 4, PREC_BF16X3>, nullptr},
};
const SigVariant kSigF16[] = {
    {"pair-space 512 K x 8x8-pair blocks", nullptr, nullptr, run_sigz<PREC_F16X3>},
    {"pair-space 512 K x 8x8-pair blocks persistent LPT queue", nullptr, nullptr, run_sigz<PREC_F16X3, true>},
};
const SigVariant kSigFP32[] = {
    {"WI2 WJ2 T4", run_sig<2, 2, 4, PREC_FP32>, nullptr},
    {"WI2 WJ4 T2", run_sig<2, 4, 2, PREC_FP32>, nullptr},
};

template <class V, size_t N>
constexpr int count_of(const V (&)[N]) {
    return int(N);
}

int64_t plane_elems(const Host& h, int q0, int nq) {
    int64_t n = 0;
    for (int q = q0; q < q0 + nq; ++q) {
        const int np = round_up(h.ni[q], PAD);
        n += int64_t(h.ntau) * np * np;
    }
    return n;
}

// elements of one plane of the split, transposed M for q0..q0+nq-1
int64_t mt_elems(const Host& h, int q0, int nq) {
    int64_t n = 0;
    for (int q = q0; q < q0 + nq; ++q) n += (h.mpre[q + 1] - h.mpre[q]) / h.ni[q] * round_up(h.ni[q], 16);
    return n;
}

}  // namespace

namespace {
const PolVariant* pol_table(int precision, int* n) {
    switch (precision) {
        case MSGW_BF16X3: *n = count_of(kPolBF16); return kPolBF16;
        case MSGW_F16X3: *n = count_of(kPolF16); return kPolF16;
        case MSGW_FP32: *n = count_of(kPolFP32); return kPolFP32;
        default: *n = 0; return nullptr;
    }
}
const SigVariant* sig_table(int precision, int* n) {
    switch (precision) {
        case MSGW_BF16X3: *n = count_of(kSigBF16); return kSigBF16;
        case MSGW_F16X3: *n = count_of(kSigF16); return kSigF16;
        case MSGW_FP32: *n = count_of(kSigFP32); return kSigFP32;
        default: *n = 0; return nullptr;
    }
}
}  // namespace

int mfma_variant_count(int op, int precision) {
    int n = 0;
    if (op == MSGW_OP_POLARIZATION) pol_table(precision, &n);
    if (op == MSGW_OP_SELF_ENERGY) sig_table(precision, &n);
    return n;
}

const char* mfma_variant_name(int op, int precision, int v) {
    if (v < 0 || v >= mfma_variant_count(op, precision)) return nullptr;
    int n;
    if (op == MSGW_OP_POLARIZATION) return pol_table(precision, &n)[v].name;
    return sig_table(precision, &n)[v].name;
}

size_t mfma_scratch_bytes(const Host& h, int nq_max) {
    // for the q range of one self_energy call: padded W~ planes and the split, transposed M planes,
    // 8 bytes per complex element each (complex64 for FP32, hi + lo bf16 pairs for BF16X3); for one
    // polarization call: the bf16 g planes of the pair-space kernel (2 bytes each)
    int64_t best = 0;
    for (int q = 0; q + nq_max <= h.nk; ++q) {
        best = std::max(best, 8 * (round_up(int(std::min<int64_t>(plane_elems(h, q, nq_max), 1 << 30)), 64) +
                                   mt_elems(h, q, nq_max)));
        // the persistent forms' work queues (items, 8 part bounds, 8 counters; at most max(n3, 1) tau chunks)
        const int64_t nch = std::max<int64_t>(1, ceil_div(h.ntau, 32) / 3);
        int64_t pq = 0, sq = 0;
        for (int qq = q; qq < q + nq_max; ++qq) {
            pq += int64_t(ceil_div(h.ni[qq], 16)) * ceil_div(h.ni[qq], 16) * nch;
            for (int k = 0; k < h.nk; ++k) sq += ceil_div(h.nb[k] * h.nb[h.kmq[size_t(qq) * h.nk + k]], 512) * nch;
        }
        best = std::max(best, int64_t(scratch_al(size_t(2 * gz_elems(h, q, nq_max)))) + 4 * (pq + 32));
        int64_t zs = 0;  // pair-space self-energy: FP32 transposed M and the weight blocks
        for (int qq = q; qq < q + nq_max; ++qq)
            zs += 8 * ((h.mpre[qq + 1] - h.mpre[qq]) / h.ni[qq] * sz_np8(h.ni[qq])) + 4 * sz_wq(h.ni[qq], h.ntau);
        best = std::max(best, int64_t(scratch_al(size_t(zs))) + 4 * (sq + 32));
    }
    return size_t(best);
}

int launch_pol_mfma(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
                    const double* G, int precision, int variant, void* P) {
    if (h.nbmax > NB_LDS) return MSGW_ENOTSUP;
    int n = 0;
    const PolVariant* table = pol_table(precision, &n);
    if (variant < 0 || variant >= n) return MSGW_EINVAL;
    const PolVariant& V = table[variant];
    if ((d.kb0 != 0 || d.kb1 != h.nk) && !V.ranged) return MSGW_ENOTSUP;
    V.fn(d, h, s, q0, nq, M, G, P);
    const int nt_eff = V.ranged ? tau_points_computed(d, h) : h.ntau;  // only the pair-space kernels mirror
    for (int q = q0; q < q0 + nq; ++q) {
        const int nt = ceil_div(h.ni[q], CW_TILE);
        double2* Pq = (double2*)P + (h.ppre[q] - h.ppre[q0]);
        MSGW_LAUNCH(k_herm_fill, dim3(nt * nt, nt_eff), dim3(256), 0, s, Pq, h.ni[q]);
        MSGW_HIP(hipGetLastError());
        if (nt_eff < h.ntau) {
            MSGW_LAUNCH(k_tau_mirror, dim3(ceil_div(int64_t(h.ni[q]) * h.ni[q], 256), h.ntau - nt_eff), dim3(256), 0,
                        s, Pq, h.ni[q], h.ntau, nt_eff);
            MSGW_HIP(hipGetLastError());
        }
    }
    return MSGW_OK;
}

int launch_sig_mfma(const Dev& d, const Host& h, hipStream_t s, int q0, int nq, const void* M,
                    const double* G, const void* W, int precision, int variant, void* Sig) {
    const int nv = mfma_variant_count(MSGW_OP_SELF_ENERGY, precision);
    if (variant < 0 || variant >= nv) return MSGW_EINVAL;
    int nt = 0;
    const SigVariant& V = sig_table(precision, &nt)[variant];
    if ((d.kb0 != 0 || d.kb1 != h.nk) && !V.fnz) return MSGW_ENOTSUP;
    if (V.fnz) {
        V.fnz(d, h, s, q0, nq, M, G, W, Sig);
        return MSGW_OK;
    }
    const int64_t plane = plane_elems(h, q0, nq);
    const int64_t wsz = round_up(int(std::min<int64_t>(plane, 1 << 30)), 64);  // W~ planes, 256-B aligned
    const int64_t mtp = V.fn3 ? mt_elems(h, q0, nq) : 0;
    if (plane >= (int64_t(1) << 30) || size_t(wsz + mtp) * 8 > scratch_mfma_bytes(d, h)) return MSGW_ENOMEM;
    char* sc = scratch_mfma(d, h);
    int64_t off = 0;
    for (int q = q0; q < q0 + nq; ++q) {
        const int NI = h.ni[q], NIp = round_up(NI, PAD);
        const int64_t n = int64_t(h.ntau) * NIp * NIp;
        const double2* Wq = (const double2*)W + (h.ppre[q] - h.ppre[q0]);
        static_assert(PAD % CW_TILE == 0, "conversion tiles must divide the padded planes");
        const int nt = NIp / CW_TILE;
        MSGW_LAUNCH(k_convert_w, dim3(nt * nt, h.ntau), dim3(256), 0, s, Wq, NI, NIp,
                           precision, reinterpret_cast<float2*>(sc) + off,
                           reinterpret_cast<uint32_t*>(sc) + off,
                           reinterpret_cast<uint32_t*>(sc) + plane + off);
        MSGW_HIP(hipGetLastError());
        off += n;
    }
    if (!V.fn3) {
        V.fn(d, h, s, q0, nq, M, G, sc, plane, Sig);
        return MSGW_OK;
    }
    uint32_t* mt = reinterpret_cast<uint32_t*>(sc) + 2 * wsz;
    for (int q = q0; q < q0 + nq; ++q) {
        int maxc = 0;
        for (int k = 0; k < h.nk; ++k) maxc = std::max(maxc, h.nb[k] * h.nb[h.kmq[size_t(q) * h.nk + k]]);
        const unsigned gx = ceil_div(round_up(h.ni[q], 16), 32) * ceil_div(maxc, 32);
        MSGW_LAUNCH(k_split_mt, dim3(gx, h.nk), dim3(256), 0, s, d, q0, q, (const float2*)M, mt, mtp);
        MSGW_HIP(hipGetLastError());
    }
    V.fn3(d, h, s, q0, nq, M, G, sc, plane, mt, mtp, Sig);
    return MSGW_OK;
}

}  // namespace msgw
