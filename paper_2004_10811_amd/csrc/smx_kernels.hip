// Memory-bound kernels of the submatrix path: gather + shift + Gershgorin
// bound, scatter of the own columns of D with the energy/trace partials, the
// fixed-order final reduction, and validation of K's values.
#include "smx_internal.h"

#include <algorithm>

namespace smx {

namespace {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

__device__ inline void atomic_max_nonneg(unsigned long long *addr, double v)
{
    // For non-negative doubles the IEEE bit patterns order like the values;
    // NaN is mapped to +Inf so that it is never lost.
    if (!(v == v)) v = __builtin_huge_val();
    atomicMax(addr, (unsigned long long)__double_as_longlong(v));
}

__device__ inline double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Gather (submatrix assembly, Sec. III-A step 1): one thread per row r of the
// padded submatrix, looping over its columns block by block.  Consecutive
// threads write consecutive rows of one column (coalesced), and the row sum
// of |A_g| feeds the Gershgorin bound s_g = ||A_g||_inf.
// ---------------------------------------------------------------------------
template <bool WRITE>
__global__ __launch_bounds__(256)
void gather_shift_kernel(const int2 *__restrict__ chunks, const GroupDesc *__restrict__ groups,
                         const RowInfo *__restrict__ rinfo, const int32_t *__restrict__ bmap,
                         const int32_t *__restrict__ boffs, const int64_t *__restrict__ valoff,
                         const double *__restrict__ kvals, double mu, double *__restrict__ x0,
                         unsigned long long *__restrict__ scale_bits)
{
    const int2 ch = chunks[blockIdx.x];
    const GroupDesc gd = groups[ch.x];
    const int r = ch.y + (int)threadIdx.x;
    const int npad = gd.npad;
    const bool live = r < npad;
    double *xg = x0 + gd.off;
    double m = gather_row(gd, r, rinfo, bmap, boffs, valoff, kvals, mu, [&](int c, double v) {
        if (WRITE && live) xg[r + (int64_t)c * npad] = v;
    });
    // padding columns: identity on the padded diagonal
    if (WRITE)
        for (int c = gd.n; c < npad; c++)
            if (live) xg[r + (int64_t)c * npad] = (r == c) ? 1.0 : 0.0;
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) atomic_max_nonneg(scale_bits + ch.x, m);
}

// ---------------------------------------------------------------------------
// Scatter (Sec. III-A step 3): for every stored block (I, J) of an own
// column J of group g, D_IJ = (delta_IJ I - S_g[I rows, J cols]) / 2.  The
// sign S_g is either a X_k (full matrix, a = 1/s_g only when the result is
// X_0) or the own-column buffer of the last polish step.  Also writes the
// block's <D_IJ, K_IJ> and, for diagonal blocks, tr D_JJ.  One wave per block.
// ---------------------------------------------------------------------------
template <int FROM_THIN>
__global__ __launch_bounds__(256)
void scatter_kernel(int64_t nblocks, const int64_t *__restrict__ plist, const ScatterDesc *__restrict__ sd,
                    const int64_t *__restrict__ valoff, const GroupDesc *__restrict__ groups,
                    const double *__restrict__ x0, const double *__restrict__ x1,
                    const int32_t *__restrict__ kfinal, const unsigned long long *__restrict__ scale_bits,
                    const double *__restrict__ kvals, double *__restrict__ dvals,
                    double *__restrict__ part_e, double *__restrict__ part_n)
{
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= nblocks) return;
    const int64_t p = plist ? plist[i] : i;
    const ScatterDesc d = sd[p];
    const GroupDesc gd = groups[d.g];
    const double *xs;
    int col0;
    double a = 1.0;
    if (FROM_THIN) {
        xs = x0 + gd.thin_off;
        col0 = d.ocol;
    } else {
        const int kf = kfinal[d.g];
        xs = ((kf & 1) ? x1 : x0) + gd.off;
        col0 = d.oj;
        if (kf == 0) {
            const double s = __longlong_as_double((long long)scale_bits[d.g]);
            a = s > 0.0 ? 1.0 / s : 0.0;
        }
    }
    const int bi = d.bij & 0xffff, bj = d.bij >> 16;
    const bool diag = (d.oi == d.oj);
    const int64_t vo = valoff[p];
    const int nel = bi * bj;
    double e = 0.0, tr = 0.0;
    for (int t = lane; t < nel; t += 64) {
        const int rr = t % bi, cc = t / bi;
        const double s = a * xs[(int64_t)(d.oi + rr) + (int64_t)(col0 + cc) * gd.npad];
        const double dv = 0.5 * ((diag && rr == cc) ? 1.0 : 0.0) - 0.5 * s;
        dvals[vo + t] = dv;
        e += dv * kvals[vo + t];
        if (diag && rr == cc) tr += dv;
    }
    e = wave_sum(e);
    tr = wave_sum(tr);
    if (lane == 0) {
        part_e[p] = e;
        part_n[p] = tr;
    }
}

// ---------------------------------------------------------------------------
// FP64 polish on the own columns only.  D needs only the group's own columns
// of the polished sign, X_{k+p}[:, own] = X_{k+p} E (E selects the own
// columns), and every polished iterate is a polynomial in the bulk result X:
// X_{j+1} = 1.5 X_j - 0.5 X_j^3.  The host side evaluates X_{k+p} E by thin
// products Y = X Z with n_pad x m_own blocks Z (column-major, leading
// dimension n_pad), so the p FP64 steps cost 3^p - 1 passes over X instead
// of 2p dense products.
// ---------------------------------------------------------------------------
// The polish reads the bulk result X where the bulk left it: an FP64 slab, or
// the words (FP16 / BF16 words, or FP32 values) of the group's final
// bulk step, converted on the fly to exactly the FP64 value the words stand
// for (sum of the words over the power-of-two scale).
enum XKind { X_F64 = 0, X_F16x2 = 1, X_BF16x3 = 2, X_BF16x1 = 3, X_F32 = 4 };

__device__ inline double f16w(unsigned short w) { return (double)(float)__builtin_bit_cast(_Float16, w); }
__device__ inline double bf16w(unsigned short w) { return (double)__builtin_bit_cast(float, ((unsigned int)w) << 16); }

template <int K>
__device__ constexpr int x_nw() { return K == X_F16x2 ? 2 : (K == X_BF16x3 ? 3 : 1); }

// Base of group g's bulk result, in elements of the storage type.
template <int K>
__device__ inline const void *x_base(const XSource &xs, const GroupDesc &gd, int g)
{
    if constexpr (K == X_F64) {
        return xs.f64 + gd.off;
    } else if constexpr (K == X_F32) {
        const unsigned short *w = (xs.kfinal[g] & 1) ? xs.w1 : xs.w0;
        return reinterpret_cast<const float *>(w) + gd.off;
    } else {
        return ((xs.kfinal[g] & 1) ? xs.w1 : xs.w0) + (int64_t)x_nw<K>() * gd.off;
    }
}

// Offset of element (r, c) = x_row(r) + c * x_col_stride(ld) from the group's base.
template <int K>
__device__ inline int64_t x_row(int r)
{
    if constexpr (K == X_F64 || K == X_F32)
        return r;
    else
        return (int64_t)(r >> 5) * (32 * x_nw<K>()) + (r & 31);
}
template <int K>
__device__ inline int64_t x_col_stride(int ld)
{
    return (int64_t)ld * ((K == X_F64 || K == X_F32) ? 1 : x_nw<K>());
}

// Power-of-two scale of the stored words (FP16 words hold x * 2^15).
template <int K>
__device__ constexpr double x_word_scale() { return K == X_F16x2 ? 1.0 / 32768.0 : 1.0; }

// X[r, c] and X[r + 1, c] (r even) at offset e = x_row(r) + c * x_col_stride(ld);
// UNSCALED: without the factor x_word_scale (the caller applies it exactly,
// e.g. to the other operand of a product).
template <int K, bool UNSCALED = false>
__device__ inline d2v x_pair(const void *base, int64_t e)
{
    if constexpr (K == X_F64) {
        return *reinterpret_cast<const d2v *>(reinterpret_cast<const double *>(base) + e);
    } else if constexpr (K == X_F32) {
        const float2 f = *reinterpret_cast<const float2 *>(reinterpret_cast<const float *>(base) + e);
        return d2v{(double)f.x, (double)f.y};
    } else {
        const unsigned short *w = reinterpret_cast<const unsigned short *>(base);
        constexpr int NW = x_nw<K>();
        d2v v;
#pragma unroll
        for (int q = NW - 1; q >= 0; q--) {
            const unsigned int u = *reinterpret_cast<const unsigned int *>(w + 32 * q + e);
            const unsigned short lo = (unsigned short)(u & 0xffffu), hi = (unsigned short)(u >> 16);
            const double a = K == X_F16x2 ? f16w(lo) : bf16w(lo), b = K == X_F16x2 ? f16w(hi) : bf16w(hi);
            if (q == NW - 1) {
                v = d2v{a, b};
            } else {
                v.x += a;
                v.y += b;
            }
        }
        if constexpr (K == X_F16x2 && !UNSCALED) v *= x_word_scale<K>();
        return v;
    }
}

template <int K>
__global__ __launch_bounds__(256)
void own_gather_kernel(const GroupDesc *__restrict__ groups, const int32_t *__restrict__ own_list, XSource xs,
                       double *__restrict__ o, int g0)
{
    const int g = g0 + blockIdx.y;
    const GroupDesc gd = groups[g];
    const int r = 2 * (blockIdx.x * 256 + threadIdx.x);
    if (r >= gd.npad) return;
    const void *xb = x_base<K>(xs, gd, g);
    const int64_t rp = x_row<K>(r), cs = x_col_stride<K>(gd.npad);
    for (int c = 0; c < gd.m_own; c++) {
        const d2v v = x_pair<K>(xb, rp + (int64_t)own_list[gd.own_off + c] * cs);
        *reinterpret_cast<d2v *>(o + gd.thin_off + r + (int64_t)c * gd.npad) = v;
    }
}

// MODE 0: y = X z.  MODE 1: y = 1.5 o - 0.5 X z.  X is symmetric; a lane owns
// two consecutive rows (16-B loads, 64 lanes = 128 rows = one contiguous 1-KB
// segment of a column of X per k, eight k in flight) and MW accumulator
// columns per pass; z is staged in LDS 128 rows at a time, row-major, so that
// one broadcast 16-B read gives two columns.  Rows k >= n of X and z are not needed: X[r, k] = 0 for
// r < n <= k, and rows r >= n of the result are exactly zero.
template <int MODE, int MW, int K>
__global__ __launch_bounds__(256)
void thin_mul_kernel(const GroupDesc *__restrict__ groups, XSource xs,
                     const double *__restrict__ z, const double *__restrict__ o, double *__restrict__ y, int g0)
{
    constexpr int KC = 128;                           // rows of z per LDS stage
    constexpr int U = 4;                              // rows of X in flight per lane (4 ran faster than 2, 8 or 16)
    __shared__ __attribute__((aligned(16))) double zs[KC][MW + 2];
    const int g = g0 + blockIdx.y;
    const GroupDesc gd = groups[g];
    const int npad = gd.npad;
    const int row0 = blockIdx.x * 512;
    if (row0 >= npad) return;                         // whole block beyond this group
    const int r = row0 + 2 * (int)threadIdx.x;        // rows r, r + 1 (npad is even)
    const bool live = r < npad;
    const void *xg = x_base<K>(xs, gd, g);
    const int64_t rp = x_row<K>(r), cs = x_col_stride<K>(npad);
    for (int c0 = 0; c0 < gd.m_own; c0 += MW) {
        const int nc = min(MW, gd.m_own - c0);
        d2v acc[MW];
#pragma unroll
        for (int c = 0; c < MW; c++) acc[c] = d2v{0.0, 0.0};
        for (int k0 = 0; k0 < gd.n; k0 += KC) {
            __syncthreads();
            for (int t = threadIdx.x; t < KC * MW; t += 256) {
                const int kk = t % KC, cc = t / KC;
                const int kr = k0 + kk;
                // the word scale goes onto z (a power of two: every product is unchanged)
                zs[kk][cc] = (kr < gd.n && cc < nc) ? z[gd.thin_off + kr + (int64_t)(c0 + cc) * npad] * x_word_scale<K>()
                                                    : 0.0;
            }
            __syncthreads();
            const int kend = min(KC, gd.n - k0);
            if (live) {
                const int64_t e0 = rp + (int64_t)k0 * cs;
                int kk = 0;
                for (; kk + U <= kend; kk += U) {
                    d2v xv[U];
#pragma unroll
                    for (int u = 0; u < U; u++) xv[u] = x_pair<K, true>(xg, e0 + (int64_t)(kk + u) * cs);
#pragma unroll
                    for (int u = 0; u < U; u++)
#pragma unroll
                        for (int c = 0; c < MW; c += 2) {
                            const d2v zv = *reinterpret_cast<const d2v *>(&zs[kk + u][c]);
                            acc[c].x = fma(xv[u].x, zv.x, acc[c].x);
                            acc[c].y = fma(xv[u].y, zv.x, acc[c].y);
                            acc[c + 1].x = fma(xv[u].x, zv.y, acc[c + 1].x);
                            acc[c + 1].y = fma(xv[u].y, zv.y, acc[c + 1].y);
                        }
                }
                for (; kk < kend; kk++) {
                    const d2v xv = x_pair<K, true>(xg, e0 + (int64_t)kk * cs);
#pragma unroll
                    for (int c = 0; c < MW; c += 2) {
                        const d2v zv = *reinterpret_cast<const d2v *>(&zs[kk][c]);
                        acc[c].x = fma(xv.x, zv.x, acc[c].x);
                        acc[c].y = fma(xv.y, zv.x, acc[c].y);
                        acc[c + 1].x = fma(xv.x, zv.y, acc[c + 1].x);
                        acc[c + 1].y = fma(xv.y, zv.y, acc[c + 1].y);
                    }
                }
            }
        }
        if (live) {
#pragma unroll
            for (int c = 0; c < MW; c++) {
                if (c >= nc) continue;
                const int64_t idx = gd.thin_off + r + (int64_t)(c0 + c) * npad;
                d2v v = acc[c];
                if (MODE == 1) {
                    const d2v ov = *reinterpret_cast<const d2v *>(o + idx);
                    v = d2v{1.5 * ov.x - 0.5 * v.x, 1.5 * ov.y - 0.5 * v.y};
                }
                *reinterpret_cast<d2v *>(y + idx) = v;
            }
        }
    }
}

// The same thin products on the matrix cores (v_mfma_f64_16x16x4_f64, FP64)
// for a bulk result held as words or FP32.  X is symmetric, so row r of X is
// its column r, whose K-consecutive entries are contiguous: a lane reads 8
// consecutive rows of one column per word (one 16-B load each; eight values
// per 16 B for FP32 reads two) and the wave's output rows need no LDS for
// X.  Wave w of a workgroup owns output rows 32 w .. + 31 of the workgroup's
// 128 (two 16-row blocks b) and 16 CB output columns per pass (CB 16-column
// blocks: one when every group owns at most 16 columns, else two).  Per K step of 32: lane l supplies, for
// product t (0 .. 7), A[i][kk] = X[r0 + 16 b + l % 16, k0 + 8 kk + t] with
// kk = l / 16 and B[kk][j] = Z[k0 + 8 kk + t, 16 cb + l % 16] from LDS, so the
// eight products of a block cover its 32 K values once.  Z goes to LDS 128
// rows at a time with the storage's power-of-two word scale on it (every
// product unchanged, the words are read unscaled).  The next K step's words
// are loaded while the matrix cores work on the current one.  Rows of Z at
// or beyond n are zero (X's padding never contributes); output rows at or
// beyond n come out exactly zero (identity padding times zero rows of Z).
template <int K>
__device__ constexpr int tm_loads() { return K == X_F32 ? 2 : x_nw<K>(); }
// 16-row blocks per wave: two keep the kernel at three waves per SIMD (four
// took two waves per SIMD and ran 0.9% slower per D on water1024; one, at four
// waves per SIMD, 5% slower per launch)
constexpr int kThinRB = 2;
constexpr int kThinRows = 64 * kThinRB;                // output rows per workgroup

// Element t (0 .. 7) of the 8 consecutive rows a lane loaded, as the unscaled
// FP64 sum of its words (exact).
template <int K>
__device__ inline double tm_value(const u4 *raw, int t)
{
    if constexpr (K == X_F32) {
        const unsigned int u = raw[t >> 2][t & 3];
        return (double)__builtin_bit_cast(float, u);
    } else {
        constexpr int NW = x_nw<K>();
        double v = 0.0;
#pragma unroll
        for (int w = NW - 1; w >= 0; w--) {
            const unsigned int u = raw[w][t >> 1];
            const unsigned short h = (t & 1) ? (unsigned short)(u >> 16) : (unsigned short)(u & 0xffffu);
            const double a = K == X_F16x2 ? f16w(h) : bf16w(h);
            v = (w == NW - 1) ? a : v + a;
        }
        return v;
    }
}

// Work item w = (group w / gx, row block w % gx).  The grid is a multiple of 8
// workgroups, which the hardware deals round-robin over the 8 XCDs; workgroup
// L takes item (L % 8) * (grid / 8) + L / 8, so that each XCD works through
// one contiguous range of items and the row blocks of a group share the XCD's
// L2 for their reads of the group's Z.
template <int MODE, int K, int CB>
__global__ __launch_bounds__(256, 3)
void thin_mfma_kernel(const GroupDesc *__restrict__ groups, XSource xs, const double *__restrict__ z,
                      const double *__restrict__ o, double *__restrict__ y, int g0, int gx, int nwork)
{
    constexpr int KC = 128;                           // rows of Z per LDS stage
    constexpr int ZS = 33;                            // LDS row stride of the staged Z (doubles)
    constexpr int NL = tm_loads<K>();
    constexpr int RB = kThinRB;
    __shared__ double zs[KC * ZS];
    const int item = (int)(blockIdx.x & 7) * (int)(gridDim.x >> 3) + (int)(blockIdx.x >> 3);
    if (item >= nwork) return;                        // padding of the grid to a multiple of 8
    const int g = g0 + item / gx;
    const GroupDesc gd = groups[g];
    const int npad = gd.npad;
    const int row0 = (item % gx) * (64 * RB);
    if (row0 >= npad) return;                         // whole workgroup beyond this group
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rw = row0 + 16 * RB * wave;             // first output row of this wave
    const bool live = rw < npad;                      // wave-uniform
    const int li = lane & 15, q = lane >> 4;
    const void *xg = x_base<K>(xs, gd, g);
    // word layout: column c starts at c * npad * NW halves, K step s at s * 32 * NW, word w at + 32 w
    auto src = [&](int b, int k0, int w) -> const u4 * {
        const int c = min(rw + 16 * b + li, npad - 1);    // rows beyond n_pad are never stored
        if constexpr (K == X_F32)
            return reinterpret_cast<const u4 *>(reinterpret_cast<const float *>(xg) + (int64_t)c * npad + k0 + 8 * q +
                                                4 * w);
        else
            return reinterpret_cast<const u4 *>(reinterpret_cast<const unsigned short *>(xg) +
                                                (int64_t)c * npad * x_nw<K>() + (int64_t)k0 * x_nw<K>() + 32 * w + 8 * q);
    };
    constexpr double zscale = x_word_scale<K>();
    const int nk = npad / 32;
    for (int c0 = 0; c0 < gd.m_own; c0 += 16 * CB) {
        f64x4 acc[RB][CB];
#pragma unroll
        for (int b = 0; b < RB; b++)
#pragma unroll
            for (int cb = 0; cb < CB; cb++) acc[b][cb] = f64x4{0.0, 0.0, 0.0, 0.0};
        u4 ra[RB][NL], rb[RB][NL];
        if (live) {
#pragma unroll
            for (int b = 0; b < RB; b++)
#pragma unroll
                for (int w = 0; w < NL; w++) ra[b][w] = *src(b, 0, w);
        }
        // one K step with the words in rc, the next step's loaded into rn
        auto kstep = [&](int kt, u4 (&rc)[RB][NL], u4 (&rn)[RB][NL]) {
            if (kt % (KC / 32) == 0) {
                const int ks = kt * 32;
                __syncthreads();                      // every wave is done with the previous stage
                // consecutive lanes take consecutive rows of one column of Z
                // (coalesced reads; the LDS writes, 33 doubles apart, are at
                // most two-way bank conflicted).  A lane keeps one row kk of Z
                // and takes columns tid / KC + 2 m; its loads go out ZB at a time,
                // all in flight before their LDS writes (every lane loads: rows
                // and columns outside Z read its last row or column, and the
                // value is replaced by zero afterwards)
                static_assert(256 == 2 * KC, "a lane's row kk = tid % KC, its first column tid / KC in {0, 1}");
                constexpr int ZU = KC * 32 / 256, ZB = 8;
                const int kk = tid & (KC - 1), kr = ks + kk;
                const double *zr = z + gd.thin_off + min(kr, gd.n - 1);
#pragma unroll
                for (int m0 = 0; m0 < ZU; m0 += ZB) {
                    double zv[ZB];
#pragma unroll
                    for (int m = 0; m < ZB; m++) {
                        const int col = c0 + tid / KC + 2 * (m0 + m);
                        zv[m] = zr[(int64_t)min(col, gd.m_own - 1) * npad];
                    }
#pragma unroll
                    for (int m = 0; m < ZB; m++) {
                        const int col = c0 + tid / KC + 2 * (m0 + m);
                        if (!(kr < gd.n && col < gd.m_own)) zv[m] = 0.0;
                    }
#pragma unroll
                    for (int m = 0; m < ZB; m++) zs[kk * ZS + tid / KC + 2 * (m0 + m)] = zv[m] * zscale;
                }
                __syncthreads();
            }
            if (!live) return;
            // the next step's words (unconditionally: the last step reloads its
            // own, so that no load sits under a branch, where the compiler would
            // wait for it at once)
            {
                const int kn = min(kt + 1, nk - 1) * 32;
#pragma unroll
                for (int b = 0; b < RB; b++)
#pragma unroll
                    for (int w = 0; w < NL; w++) rn[b][w] = *src(b, kn, w);
            }
            const double *zr = zs + ((kt % (KC / 32)) * 32 + 8 * q) * ZS + li;
#pragma unroll
            for (int t = 0; t < 8; t++) {
                double bz[CB];
#pragma unroll
                for (int cb = 0; cb < CB; cb++) bz[cb] = zr[t * ZS + 16 * cb];
#pragma unroll
                for (int b = 0; b < RB; b++) {
                    const double a = tm_value<K>(rc[b], t);
#pragma unroll
                    for (int cb = 0; cb < CB; cb++)
                        acc[b][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bz[cb], acc[b][cb], 0, 0, 0);
                }
            }
        };
        for (int kt = 0; kt < nk; kt += 2) {
            kstep(kt, ra, rb);
            if (kt + 1 < nk) kstep(kt + 1, rb, ra);
        }
        if (live) {
            // lane l, register v of block (b, cb): row 16 b + l / 16 + 4 v, column 16 cb + l % 16
#pragma unroll
            for (int b = 0; b < RB; b++)
#pragma unroll
                for (int cb = 0; cb < CB; cb++) {
                    const int col = c0 + 16 * cb + li;
                    if (col >= gd.m_own) continue;
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int r = rw + 16 * b + q + 4 * v;
                        if (r >= npad) continue;
                        const int64_t idx = gd.thin_off + r + (int64_t)col * npad;
                        double val = acc[b][cb][v];
                        if (MODE == 1) val = 1.5 * o[idx] - 0.5 * val;
                        y[idx] = val;
                    }
                }
        }
    }
}

// a <- 1.5 a - 0.5 c on the own-column blocks (in place in c: c = 1.5 a - 0.5 c).
__global__ __launch_bounds__(256)
void thin_combine_kernel(const GroupDesc *__restrict__ groups, const double *__restrict__ a,
                         double *__restrict__ c, int g0)
{
    const GroupDesc gd = groups[g0 + blockIdx.y];
    const int64_t tot = (int64_t)gd.npad * gd.m_own;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256)
        c[gd.thin_off + e] = 1.5 * a[gd.thin_off + e] - 0.5 * c[gd.thin_off + e];
}

// max |b - E| over the true rows and the own columns -> residual slot of the group.
__global__ __launch_bounds__(256)
void thin_resid_kernel(const GroupDesc *__restrict__ groups, const int32_t *__restrict__ own_list,
                       const double *__restrict__ b, IterState it, int slot, int g0)
{
    const int g = g0 + blockIdx.y;
    const GroupDesc gd = groups[g];
    double rmax = 0.0;
    const int64_t tot = (int64_t)gd.npad * gd.m_own;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int r = (int)(e % gd.npad), c = (int)(e / gd.npad);
        if (r >= gd.n) continue;
        double d = fabs(b[gd.thin_off + e] - (r == own_list[gd.own_off + c] ? 1.0 : 0.0));
        if (!(d <= 1.7976931348623157e308)) d = __builtin_huge_val();
        rmax = fmax(rmax, d);
    }
    rmax = wave_max(rmax);
    if ((threadIdx.x & 63) == 0) atomic_max_nonneg(it.resid_bits + (int64_t)g * it.resid_stride + slot, rmax);
}

// Convergence of the own-column polish: r = max|X_{k+p-1}^2 E - E| is the
// residual one step before the returned iterate, and one Newton-Schulz step
// maps an eigenvalue with 1 - x^2 = r to one with 1 - x'^2 = 3r^2/4 + r^3/4.
// The group is flagged not converged (bit 0) unless 3r^2/4 <= tol, the FP64
// stopping rule applied to the returned iterate; non-finite r sets bit 1.
__global__ __launch_bounds__(256)
void polish_flags_kernel(int ngroups, IterState it, int slot, double tol, int g0)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= ngroups) return;
    const int g = g0 + q;
    const double r = __longlong_as_double((long long)it.resid_bits[(int64_t)g * it.resid_stride + slot]);
    int fl = it.flags[g];
    if (!(r <= 1.7976931348623157e308)) fl |= 2;
    else if (!(0.75 * r * r <= tol)) fl |= 1;
    it.flags[g] = fl;
}

// out2[0] = groups with flag bit 0 (not converged), out2[1] = groups with bit 1
// (non-finite), over flags[0 .. ngroups-1]; one workgroup, no atomics.
__global__ __launch_bounds__(1024)
void count_flags_kernel(int ngroups, const int32_t *__restrict__ flags, int32_t *__restrict__ out2)
{
    __shared__ int s0[16], s1[16];
    const int t = threadIdx.x;
    int c0 = 0, c1 = 0;
    for (int g = t; g < ngroups; g += 1024) {
        c0 += flags[g] & 1;
        c1 += (flags[g] >> 1) & 1;
    }
    for (int o = 32; o > 0; o >>= 1) {
        c0 += __shfl_xor(c0, o, 64);
        c1 += __shfl_xor(c1, o, 64);
    }
    if ((t & 63) == 0) {
        s0[t >> 6] = c0;
        s1[t >> 6] = c1;
    }
    __syncthreads();
    if (t == 0) {
        int a0 = 0, a1 = 0;
        for (int w = 0; w < 16; w++) {
            a0 += s0[w];
            a1 += s1[w];
        }
        out2[0] = a0;
        out2[1] = a1;
    }
}

// Fixed-order sum of the per-block partials (one workgroup): deterministic.
// Lane t adds the entries t, t + 1024, t + 2048, ... in that order (a wave
// reads 512 consecutive bytes per step), then a fixed tree.
__global__ __launch_bounds__(1024)
void reduce_kernel(int64_t n, const double *__restrict__ pe, const double *__restrict__ pn,
                   double *__restrict__ out2)
{
    __shared__ double se[16], sn[16];
    const int t = threadIdx.x;
    double e = 0.0, tr = 0.0;
    for (int64_t i = t; i < n; i += 1024) {
        e += pe[i];
        tr += pn[i];
    }
    // fixed tree: within waves by xor shuffles, then across the 16 waves in order
    e = wave_sum(e);
    tr = wave_sum(tr);
    if ((t & 63) == 0) {
        se[t >> 6] = e;
        sn[t >> 6] = tr;
    }
    __syncthreads();
    if (t == 0) {
        double ae = 0.0, an = 0.0;
        for (int w = 0; w < 16; w++) {
            ae += se[w];
            an += sn[w];
        }
        out2[0] = an;
        out2[1] = ae;
    }
}

// Validation of K's values: max|K_IJ - K_JI^T| and max|K| (NaN/Inf -> +Inf).
__global__ __launch_bounds__(256)
void check_values_kernel(int64_t nblocks, const int64_t *__restrict__ valoff,
                         const int32_t *__restrict__ brow, const int32_t *__restrict__ bcol,
                         const int64_t *__restrict__ mirror, const double *__restrict__ kv,
                         unsigned long long *__restrict__ out2)
{
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    double asym = 0.0, amax = 0.0;
    if (p < nblocks) {
        const int bi = brow[p], bj = bcol[p];
        const int64_t q = mirror[p];
        const double *a = kv + valoff[p];
        const double *b = kv + valoff[q];          // block (J, I): bj x bi
        for (int t = lane; t < bi * bj; t += 64) {
            const int rr = t % bi, cc = t / bi;
            const double x = a[t];
            const double y = b[cc + (int64_t)rr * bj];
            double dz = fabs(x - y);
            double ax = fabs(x);
            if (!(ax <= 1.7976931348623157e308)) { ax = __builtin_huge_val(); dz = ax; }
            asym = fmax(asym, dz);
            amax = fmax(amax, ax);
        }
    }
    asym = wave_max(asym);
    amax = wave_max(amax);
    if (lane == 0 && p < nblocks) {
        atomic_max_nonneg(out2 + 0, asym);
        atomic_max_nonneg(out2 + 1, amax);
    }
}

// Xd_0 = -a I on the true block (a = 1/s_g), one group per blockIdx.y.
__global__ __launch_bounds__(256)
void tangent_init_kernel(const GroupDesc *__restrict__ groups, const unsigned long long *__restrict__ scale_bits,
                         double *__restrict__ xd, int g0)
{
    const GroupDesc gd = groups[g0 + blockIdx.y];
    const int64_t tot = (int64_t)gd.npad * gd.npad;
    const double s = __longlong_as_double((long long)scale_bits[g0 + blockIdx.y]);
    const double a = s > 0.0 ? 1.0 / s : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t r = e % gd.npad, c = e / gd.npad;
        xd[gd.off + e] = (r == c && r < gd.n) ? -a : 0.0;
    }
}

// part[g] = sum of Xd_kfinal over the group's own diagonal, in list order.
__global__ __launch_bounds__(64)
void own_trace_kernel(const GroupDesc *__restrict__ groups, const int32_t *__restrict__ own_list,
                      const double *__restrict__ xd0, const double *__restrict__ xd1,
                      const int32_t *__restrict__ kfinal, double *__restrict__ part, int g0)
{
    const int g = g0 + blockIdx.x;
    const GroupDesc gd = groups[g];
    const double *xd = ((kfinal[g] & 1) ? xd1 : xd0) + gd.off;
    double acc = 0.0;
    for (int q = threadIdx.x; q < gd.m_own; q += 64) {
        const int c = own_list[gd.own_off + q];
        acc += xd[c + (int64_t)c * gd.npad];
    }
    acc = wave_sum(acc);
    if (threadIdx.x == 0) part[g] = acc;
}

}  // namespace

hipError_t launch_tangent_init(hipStream_t st, int g0, int ngroups, int max_npad, const GroupDesc *groups,
                               const unsigned long long *scale_bits, double *xd)
{
    if (ngroups <= 0) return hipSuccess;
    const int64_t tot = (int64_t)max_npad * max_npad;
    const dim3 grid((unsigned)std::min<int64_t>((tot + 2047) / 2048, 4096), (unsigned)ngroups);
    hipLaunchKernelGGL(tangent_init_kernel, grid, dim3(256), 0, st, groups, scale_bits, xd, g0);
    return hipGetLastError();
}

hipError_t launch_own_trace(hipStream_t st, int g0, int ngroups, const GroupDesc *groups, const int32_t *own_list,
                            const double *xd0, const double *xd1, const int32_t *kfinal, double *part)
{
    if (ngroups <= 0) return hipSuccess;
    hipLaunchKernelGGL(own_trace_kernel, dim3(ngroups), dim3(64), 0, st, groups, own_list, xd0, xd1, kfinal, part, g0);
    return hipGetLastError();
}

hipError_t launch_gather(hipStream_t st, int nchunks, const int2 *chunks, const GroupDesc *groups,
                         const RowInfo *rinfo, const int32_t *bmap, const int32_t *boffs,
                         const int64_t *valoff, const double *kvals, double mu, double *x0,
                         unsigned long long *scale_bits)
{
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_shift_kernel<true>, dim3(nchunks), dim3(256), 0, st, chunks, groups,
                       rinfo, bmap, boffs, valoff, kvals, mu, x0, scale_bits);
    return hipGetLastError();
}

hipError_t launch_gather_bound(hipStream_t st, int nchunks, const int2 *chunks, const GroupDesc *groups,
                               const RowInfo *rinfo, const int32_t *bmap, const int32_t *boffs,
                               const int64_t *valoff, const double *kvals, double mu,
                               unsigned long long *scale_bits)
{
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_shift_kernel<false>, dim3(nchunks), dim3(256), 0, st, chunks, groups,
                       rinfo, bmap, boffs, valoff, kvals, mu, nullptr, scale_bits);
    return hipGetLastError();
}

hipError_t launch_scatter(hipStream_t st, int64_t nblocks, const int64_t *plist, const ScatterDesc *sd,
                          const int64_t *valoff, const GroupDesc *groups, const double *x0,
                          const double *x1, const IterState &it, const double *kvals,
                          double *dvals, double *part_e, double *part_n, int from_thin)
{
    if (nblocks <= 0) return hipSuccess;
    const int64_t grid = (nblocks + 3) / 4;
    if (from_thin)
        hipLaunchKernelGGL(scatter_kernel<1>, dim3((unsigned)grid), dim3(256), 0, st, nblocks, plist, sd, valoff,
                           groups, x0, x1, it.kfinal, it.scale_bits, kvals, dvals, part_e, part_n);
    else
        hipLaunchKernelGGL(scatter_kernel<0>, dim3((unsigned)grid), dim3(256), 0, st, nblocks, plist, sd, valoff,
                           groups, x0, x1, it.kfinal, it.scale_bits, kvals, dvals, part_e, part_n);
    return hipGetLastError();
}

static int x_kind(const XSource &xs)
{
    if (xs.fmt < 0) return X_F64;
    if (xs.fmt == 2) return X_F32;
    if (xs.fmt == 0 && xs.nw == 2) return X_F16x2;
    if (xs.fmt == 1 && xs.nw == 3) return X_BF16x3;
    if (xs.fmt == 1 && xs.nw == 1) return X_BF16x1;
    return -1;
}

hipError_t launch_own_gather(hipStream_t st, int g0, int ngroups, int max_npad, const GroupDesc *groups,
                             const int32_t *own_list, const XSource &xs, double *out)
{
    if (ngroups <= 0) return hipSuccess;
    const dim3 grid((unsigned)((max_npad / 2 + 255) / 256), (unsigned)ngroups);
#define SMX_OG(K) hipLaunchKernelGGL((own_gather_kernel<K>), grid, dim3(256), 0, st, groups, own_list, xs, out, g0)
    switch (x_kind(xs)) {
    case X_F64: SMX_OG(X_F64); break;
    case X_F16x2: SMX_OG(X_F16x2); break;
    case X_BF16x3: SMX_OG(X_BF16x3); break;
    case X_BF16x1: SMX_OG(X_BF16x1); break;
    case X_F32: SMX_OG(X_F32); break;
    default: return hipErrorInvalidValue;
    }
#undef SMX_OG
    return hipGetLastError();
}

template <int K>
static hipError_t thin_mul_k(hipStream_t st, int mode, int mw, dim3 grid, int g0, const GroupDesc *groups,
                             const XSource &xs, const double *z, const double *o, double *y)
{
#define SMX_TM(M, W) hipLaunchKernelGGL((thin_mul_kernel<M, W, K>), grid, dim3(256), 0, st, groups, xs, z, o, y, g0)
    if (mode == 0) {
        if (mw == 8) SMX_TM(0, 8); else if (mw == 16) SMX_TM(0, 16); else if (mw == 24) SMX_TM(0, 24); else SMX_TM(0, 32);
    } else {
        if (mw == 8) SMX_TM(1, 8); else if (mw == 16) SMX_TM(1, 16); else if (mw == 24) SMX_TM(1, 24); else SMX_TM(1, 32);
    }
#undef SMX_TM
    return hipGetLastError();
}

hipError_t launch_thin_mul(hipStream_t st, int mode, int g0, int ngroups, int max_npad, int max_own,
                           const GroupDesc *groups, const XSource &xs, const double *z, const double *o, double *y)
{
    if (ngroups <= 0 || max_own <= 0) return hipSuccess;
    const dim3 grid((unsigned)((max_npad + 511) / 512), (unsigned)ngroups);
    const int mw = max_own <= 8 ? 8 : (max_own <= 16 ? 16 : (max_own <= 24 ? 24 : 32));
    // the bulk's words (or FP32 values) go through the matrix cores; an FP64
    // slab through the vector units
    const int gx = (max_npad + kThinRows - 1) / kThinRows;
    const int nwork = gx * ngroups;
    const dim3 grid_m((unsigned)((nwork + 7) / 8 * 8));
    // one 16-column block per pass when every group owns at most 16 columns
#define SMX_TMM(KK)                                                                                             \
    do {                                                                                                        \
        if (max_own <= 16) {                                                                                    \
            if (mode == 0)                                                                                      \
                hipLaunchKernelGGL((thin_mfma_kernel<0, KK, 1>), grid_m, dim3(256), 0, st, groups, xs, z, o, y, g0, gx, nwork); \
            else                                                                                                \
                hipLaunchKernelGGL((thin_mfma_kernel<1, KK, 1>), grid_m, dim3(256), 0, st, groups, xs, z, o, y, g0, gx, nwork); \
        } else {                                                                                                \
            if (mode == 0)                                                                                      \
                hipLaunchKernelGGL((thin_mfma_kernel<0, KK, 2>), grid_m, dim3(256), 0, st, groups, xs, z, o, y, g0, gx, nwork); \
            else                                                                                                \
                hipLaunchKernelGGL((thin_mfma_kernel<1, KK, 2>), grid_m, dim3(256), 0, st, groups, xs, z, o, y, g0, gx, nwork); \
        }                                                                                                       \
        return hipGetLastError();                                                                               \
    } while (0)
    switch (x_kind(xs)) {
    case X_F64: return thin_mul_k<X_F64>(st, mode, mw, grid, g0, groups, xs, z, o, y);
    case X_F16x2: SMX_TMM(X_F16x2);
    case X_BF16x3: SMX_TMM(X_BF16x3);
    case X_BF16x1: SMX_TMM(X_BF16x1);
    case X_F32: SMX_TMM(X_F32);
    default: return hipErrorInvalidValue;
    }
#undef SMX_TMM
}

hipError_t launch_thin_combine(hipStream_t st, int g0, int ngroups, int max_npad, int max_own,
                               const GroupDesc *groups, const double *a, double *c)
{
    if (ngroups <= 0 || max_own <= 0) return hipSuccess;
    const int64_t tot = (int64_t)max_npad * max_own;
    const dim3 grid((unsigned)std::min<int64_t>((tot + 1023) / 1024, 1024), (unsigned)ngroups);
    hipLaunchKernelGGL(thin_combine_kernel, grid, dim3(256), 0, st, groups, a, c, g0);
    return hipGetLastError();
}

hipError_t launch_thin_resid(hipStream_t st, int g0, int ngroups, int max_npad, int max_own,
                             const GroupDesc *groups, const int32_t *own_list, const double *b,
                             const IterState &it, int slot)
{
    if (ngroups <= 0 || max_own <= 0) return hipSuccess;
    const int64_t tot = (int64_t)max_npad * max_own;
    const dim3 grid((unsigned)std::min<int64_t>((tot + 1023) / 1024, 1024), (unsigned)ngroups);
    hipLaunchKernelGGL(thin_resid_kernel, grid, dim3(256), 0, st, groups, own_list, b, it, slot, g0);
    return hipGetLastError();
}

hipError_t launch_polish_flags(hipStream_t st, int g0, int ngroups, const IterState &it, int slot, double tol)
{
    if (ngroups <= 0) return hipSuccess;
    hipLaunchKernelGGL(polish_flags_kernel, dim3((unsigned)((ngroups + 255) / 256)), dim3(256), 0, st, ngroups, it,
                       slot, tol, g0);
    return hipGetLastError();
}

// D in another layout of stored values: dst[idx[q]] = src[q] for every q
// (dst was cleared before; the host checked that the indices are in range and
// pairwise distinct).  Grid-stride over q.
__global__ __launch_bounds__(256)
void expand_values_kernel(int64_t n, const int64_t *__restrict__ idx, const double *__restrict__ src,
                          double *__restrict__ dst)
{
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
        dst[idx[q]] = src[q];
}

__global__ __launch_bounds__(256)
void clear_values_kernel(int64_t n, double *__restrict__ dst)
{
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
        dst[q] = 0.0;
}

hipError_t launch_count_flags(hipStream_t st, int ngroups, const int32_t *flags, int32_t *out2)
{
    hipLaunchKernelGGL(count_flags_kernel, dim3(1), dim3(1024), 0, st, ngroups, flags, out2);
    return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t st, int64_t n, const double *part_e, const double *part_n,
                         double *out2)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, n, part_e, part_n, out2);
    return hipGetLastError();
}

hipError_t launch_check_values(hipStream_t st, int64_t nblocks, const int64_t *valoff,
                               const int32_t *blk_rows, const int32_t *blk_cols,
                               const int64_t *mirror, const double *kvals, double *out2)
{
    if (nblocks <= 0) return hipSuccess;
    const int64_t grid = (nblocks + 3) / 4;
    hipLaunchKernelGGL(check_values_kernel, dim3((unsigned)grid), dim3(256), 0, st, nblocks, valoff,
                       blk_rows, blk_cols, mirror, kvals,
                       reinterpret_cast<unsigned long long *>(out2));
    return hipGetLastError();
}

hipError_t launch_expand_values(hipStream_t st, int64_t n_src, const int64_t *idx, const double *src, int64_t n_dst,
                                double *dst)
{
    const int64_t nb_dst = std::min<int64_t>((n_dst + 255) / 256, 8192);
    if (n_dst > 0) hipLaunchKernelGGL(clear_values_kernel, dim3((unsigned)nb_dst), dim3(256), 0, st, n_dst, dst);
    const int64_t nb = std::min<int64_t>((n_src + 255) / 256, 8192);
    if (n_src > 0) hipLaunchKernelGGL(expand_values_kernel, dim3((unsigned)nb), dim3(256), 0, st, n_src, idx, src, dst);
    return hipGetLastError();
}

}  // namespace smx

