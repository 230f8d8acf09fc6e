// Reduced-precision Newton-Schulz products on the gfx950 matrix cores.
//
// The bulk of the sign iteration (Sec. II-B) may run in low precision; the
// paper runs the whole iteration on tensor cores in FP16, "FP16'" (FP16
// multiply, FP32 accumulate) and FP32 and observes energies close to FP64
// (Sec. VI-A, Table I).  Here every iterate is held as NW "words" of a
// 16-bit format (FP16 or BF16): x ~ w0 + w1 + ... with w_{j+1} the rounded
// remainder of x - (w0 + ... + w_j).  A product of two matrices becomes the
// sum of the word products whose combined significance is kept (NW = 1: w0 w0;
// NW = 2: w0 w0 + w0 w1 + w1 w0; NW = 3 adds w1 w1 + w0 w2 + w2 w0), each one
// v_mfma_f32_16x16x32_{f16,bf16}, all accumulated in FP32.  Word products are
// exact in FP32, so the accuracy is set by the word representation and the
// FP32 accumulation.
//
// Same two-product step, tiling, symmetry use (lower tiles + mirror) and
// column-wise operand reads as the FP64 kernel.  The epilogue splits the
// FP32 result back into words, so no higher-precision copy of the iterate is
// kept between steps.  X_0 = A / s_g is produced by a separate conversion
// pass, so no scale is applied here.
//
// Stopping rule of the bulk phase (per group, on the device), on
// tau_k = Tr(I - X_k^2) = sum_i (1 - x_i^2): every eigenvalue of an iterate
// lies in [-1, 1], so tau_k bounds the largest 1 - x_i^2 from above (the
// entrywise max|X_k^2 - I| does not: for a delocalised eigenvector it is
// far smaller than the eigenvalue error).  The group leaves the bulk at X_k
// once tau_k <= switch_tol, or once tau_k stops falling (tau_k >= tau_{k-1},
// or tau_k < 0.1 and tau_k > tau_{k-1} / 2: the floor of the word format), or
// at the step cap;
// the FP64 polish steps follow.  tau_k is reduced in a fixed order (per
// diagonal tile, then over the tiles), so the decision is reproducible.
#include "smx_internal.h"

namespace smx {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int BM = kTile;   // 128

// Power-of-two scale applied to every value before it is split into words.
// FP16 has a 5-bit exponent: subnormal FP16 words keep fewer significant
// bits, so the iterates (|x| <= 1, |w| <= 1.5) are lifted by 2^15 (largest
// word 49152 < 65504).  The leading word then stays normal down to
// |x| ~ 2^-29 and the second word down to |x| ~ 2^-18 (smaller remainders are
// below 2^-29 absolute).  BF16 has the FP32 exponent range and needs no
// scale.  Products carry scale^2, removed exactly in the epilogue.
template <int FMT>
__host__ __device__ constexpr double word_scale() { return FMT == 0 ? 32768.0 : 1.0; }

template <int FMT>
__device__ inline unsigned short to_word(double v);

template <>
__device__ inline unsigned short to_word<0>(double v)   // FP16, round to nearest
{
    const _Float16 h = (_Float16)(float)v;
    return __builtin_bit_cast(unsigned short, h);
}

template <>
__device__ inline unsigned short to_word<1>(double v)   // BF16, round to nearest even
{
    const float f = (float)v;
    unsigned int u = __builtin_bit_cast(unsigned int, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

template <int FMT>
__device__ inline double from_word(unsigned short w);

template <>
__device__ inline double from_word<0>(unsigned short w)
{
    return (double)(float)__builtin_bit_cast(_Float16, w);
}

template <>
__device__ inline double from_word<1>(unsigned short w)
{
    return (double)__builtin_bit_cast(float, ((unsigned int)w) << 16);
}

template <int FMT>
__device__ inline f4 mfma16(const u16x8 &a, const u16x8 &b, const f4 &c)
{
    if constexpr (FMT == 0)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, a), __builtin_bit_cast(b8, b), c, 0, 0, 0);
}

// Word-pair table: products (p, q) kept for NW words, most significant first.
template <int NW>
__host__ __device__ constexpr int npairs() { return NW == 1 ? 1 : (NW == 2 ? 3 : 6); }
__host__ __device__ constexpr int pair_p(int i) { return i == 2 || i == 3 ? 1 : (i == 5 ? 2 : 0); }
__host__ __device__ constexpr int pair_q(int i) { return i == 1 || i == 3 ? 1 : (i == 4 ? 2 : 0); }

// Split v into NW words: each word the rounded remainder of v minus the previous words.
template <int FMT, int NW>
__device__ inline void split_words(double v, unsigned short *out)
{
    double rem = v;
#pragma unroll
    for (int w = 0; w < NW; w++) {
        out[w] = to_word<FMT>(rem);
        rem -= from_word<FMT>(out[w]);
    }
}

__device__ inline double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// tau_k = Tr(I - X_k^2) of a group from the diagonal values 1 - T_ii the
// square wrote for its true rows: lane l sums rows l, l + 64, ... in order,
// then a fixed xor tree, and lane 0's sum is taken.  Every wave of every
// workgroup evaluates the same expression, so all of them (whatever their
// tile shape) see the same bits.
__device__ inline double tau_of(const double *__restrict__ td, int n, int lane)
{
    double s = 0.0;
    for (int i = lane; i < n; i += 64) s += td[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return __shfl(s, 0, 64);
}

// Stopping rule of the bulk at step k (update products, before any work):
// the group leaves the bulk at X_k once tau_k <= switch_tol, or once tau_k
// stops falling (tau_k >= tau_{k-1}, or tau_k < 0.1 and tau_k > tau_{k-1} / 2:
// the floor of the word format), or at the step cap.  The leader (thread 0 of
// the group's first tile) records tau_k and, on leaving, the result step and
// the flags: not converged (bit 0) when the bulk leaves above switch_tol and
// `strict` (every format but single-word BF16, whose floor lies above
// switch_tol by design and whose polished residual decides alone), non-finite
// (bit 1).  Returns true when the group has left the bulk.
__device__ inline bool bulk_stop(const IterState &it, const GroupDesc &gd, int g, int k, bool leader, int lane,
                                 double switch_tol, int kmax, bool strict)
{
    const int64_t base = (int64_t)g * it.resid_stride;
    const double rk = __longlong_as_double((long long)it.resid_bits[base + k]);
    const double tau = tau_of(it.tdiag + gd.rinfo_off, gd.n, lane);
    const double tp = k > 0 ? it.tau_hist[base + k - 1] : __builtin_huge_val();
    const bool finite = (rk <= 1.7976931348623157e308) && (fabs(tau) <= 1.7976931348623157e308);
    // floor of the word format: tau stops halving in the quadratic phase, or
    // stops falling at all (in the linear phase every 1 - x_i^2 shrinks)
    const bool stall = ((tau < 0.1) && (tau > 0.5 * tp)) || (tau >= tp);
    if (leader) it.tau_hist[base + k] = tau;
    if (tau <= switch_tol || stall || k >= kmax || !finite) {
        if (leader) {
            it.done[g] = 1;
            it.kfinal[g] = k;
            it.flags[g] = !finite ? 2 : ((strict && tau > switch_tol) ? 1 : 0);
            atomicAdd(it.ndone, 1);
        }
        return true;
    }
    return false;
}

template <int FMT>
__device__ inline unsigned short to_word_f(float v);
template <>
__device__ inline unsigned short to_word_f<0>(float v)
{
    return __builtin_bit_cast(unsigned short, (_Float16)v);
}
template <>
__device__ inline unsigned short to_word_f<1>(float v)
{
    unsigned int u = __builtin_bit_cast(unsigned int, v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
template <int FMT>
__device__ inline float from_word_f(unsigned short w)
{
    if constexpr (FMT == 0)
        return (float)__builtin_bit_cast(_Float16, w);
    else
        return __builtin_bit_cast(float, ((unsigned int)w) << 16);
}

// Split 8 FP32 values (already scaled) into NW word vectors.  Each remainder
// x - round(x) is exact in FP32, so the words sum to x up to the last word's
// rounding.
template <int FMT, int NW>
__device__ inline void split8(const float *v, u16x8 *wv)
{
#pragma unroll
    for (int e = 0; e < 8; e++) {
        float rem = v[e];
#pragma unroll
        for (int w = 0; w < NW; w++) {
            const unsigned short u = to_word_f<FMT>(rem);
            wv[w][e] = u;
            rem -= from_word_f<FMT>(u);
        }
    }
}

// Eight consecutive entries (rows r0 .. r0 + 7, r0 a multiple of 8) of column
// c of a word-stored matrix, unscaled, in FP32 (the sum of the words is exact
// there): the T that the combine of the third-order Pade step reads at its
// output positions.
template <int FMT, int NW>
__device__ inline void load8_words(const unsigned short *__restrict__ m, int ld, int r0, int c, float *v)
{
    const unsigned short *p = m + word_pos(NW, ld, r0, c);
    u16x8 w[NW];
#pragma unroll
    for (int q = 0; q < NW; q++) w[q] = *reinterpret_cast<const u16x8 *>(p + 32 * q);
#pragma unroll
    for (int e = 0; e < 8; e++) {
        float s = 0.f;
#pragma unroll
        for (int q = NW - 1; q >= 0; q--) s += from_word_f<FMT>(w[q][e]);
        v[e] = s * (float)(1.0 / word_scale<FMT>());
    }
}

// Output value of a product t at (r, c): MODE 0 (Newton-Schulz square)
// W = 1.5 I - 0.5 T; MODE 1 (update) and MODE 2 (Pade square) the product
// itself; MODE 3 (Pade combine, t = (T T)_rc, tv = T_rc)
// W = (15 I - 10 T + 3 T^2) / 8.
template <int MODE>
__device__ inline float out_value(float t, float tv, int r, int c)
{
    if constexpr (MODE == 0) return -0.5f * t + (r == c ? 1.5f : 0.f);
    else if constexpr (MODE == 3) return 0.125f * ((r == c ? 15.f : 0.f) - 10.f * tv + 3.f * t);
    else return t;
}

// Operands go straight from global memory into LDS (global_load_lds_dwordx4,
// no register staging) in K steps of 32: per operand and word a
// [128 columns][32] halves region, 64 B per column, whose four 16-B chunks are
// XOR-swizzled by column so that the matrix-core operand reads (16 columns x
// one chunk) are free of bank conflicts.  One stage per workgroup: the operand traffic
// of one workgroup overlaps the products of the others on the CU.  The
// epilogue stages half of the FP32 tile at a time in LDS, column-major, so
// that 16 consecutive lanes write one 128-row column segment (coalesced 16-B
// stores); the mirror reads the converted words back from the same staging
// (three words: from a second, row-major staging of the FP32 values).
constexpr int BK = 32;
constexpr int CPC = BK / 8;        // 16-B chunks per column, word and K step
constexpr int CST = 132;           // column-major staging: 528-B columns (conflict-free f4 stores)
constexpr int CSTH = 68;           // row-major staging of a 64-column half (three words)

// Slot of chunk 0 of a column: every 8 consecutive columns, and the even and
// the odd columns of every 16, get distinct slots, so a 16-B operand read of
// 16 consecutive columns is free of bank conflicts whether the LDS serves
// 8 lanes per cycle from 32 banks or 16 lanes from 64.
__device__ inline int swz(int col) { return (col ^ (col >> 2)) & 3; }

// s_waitcnt vmcnt(0) (the gfx9 encoding with expcnt and lgkmcnt left at their maxima)
__device__ inline void wait_vm0() { __builtin_amdgcn_s_waitcnt(0x0F70); }
// s_waitcnt lgkmcnt(0) (vmcnt and expcnt left at their maxima): LDS writes done
__device__ inline void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Workgroup barrier without the memory fence of __syncthreads(): the operand
// loads are waited for explicitly; the empty asm statements keep the compiler
// from moving LDS accesses across it.
__device__ inline void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Eight staged floats as two 16-B reads; lanes 4-7 of every 8 read their
// second half first, so the first read of 8 lanes covers 32 distinct banks.
__device__ inline void load8(const float *p, int swap, float *v)
{
    const int o = swap ? 4 : 0;
    const f4 a = *reinterpret_cast<const f4 *>(p + o);
    const f4 b = *reinterpret_cast<const f4 *>(p + (4 - o));
    const f4 lo = swap ? b : a, hi = swap ? a : b;
    v[0] = lo.x; v[1] = lo.y; v[2] = lo.z; v[3] = lo.w;
    v[4] = hi.x; v[5] = hi.y; v[6] = hi.z; v[7] = hi.w;
}

template <int NW>
__host__ __device__ constexpr int words_lds_bytes()
{
    return (2 * NW * BM * BK * 2) > (BM * CSTH * 4) ? (2 * NW * BM * BK * 2) : (BM * CSTH * 4);
}

// RP = 0: operands go straight into LDS by global_load_lds, one K step at a
// time.  RP = 1: the next K step's operands are loaded into registers (whole
// 128-B lines, eight lanes per column) while the matrix cores work on the
// current one from LDS, then written to LDS in the same swizzled layout.
template <int FMT, int NW, int MODE, int RP>
__device__ __forceinline__ void ns_words_tile(const TileDesc td, const GroupDesc *__restrict__ groups,
                                              const unsigned short *__restrict__ xin,
                                              const unsigned short *__restrict__ bin,
                                              unsigned short *__restrict__ out, const IterState &it, int k,
                                              double switch_tol, int kmax)
{
    __shared__ __attribute__((aligned(16))) unsigned char smem[words_lds_bytes<NW>()];
    unsigned short *Ls = reinterpret_cast<unsigned short *>(smem);   // [2 operands][NW][BM][BK]
    float *Cs = reinterpret_cast<float *>(smem);                     // staging after the K loop

    const int g = td.x;
    if (g < 0) return;                  // idle slot of the launch order
    if (it.done[g]) return;
    const int ti = td.y >> 16, tj = td.y & 0xffff;
    const GroupDesc gd = groups[g];
    const int ld = gd.npad;

    if (MODE == 1 && bulk_stop(it, gd, g, k, ti == 0 && tj == 0 && threadIdx.x == 0, threadIdx.x & 63, switch_tol,
                               kmax, NW > 1))
        return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int li = lane & 15;
    const int lg = lane >> 4;

    // Loads: one wave instruction fills 1 KB of LDS = 16 columns x 64 B; lane l
    // fills slot l % 4 of column (wave + 4 q) * 16 + l / 4 with chunk
    // (slot ^ swz(column)) of that column.  Columns beyond ld and the chunk
    // offsets of a K step beyond ld read any valid address instead (their
    // products only reach discarded outputs, or are not issued).
    constexpr int PH = BM * BK;         // halves per operand-word region of LDS
    const unsigned short *srcA[2], *srcB[2];
    int kcoff[2];
#pragma unroll
    for (int q = 0; q < 2; q++) {
        const int cl = (wave + 4 * q) * 16 + lane / CPC;
        kcoff[q] = ((lane % CPC) ^ swz(cl)) * 8;
        srcA[q] = xin + NW * gd.off + word_pos(NW, ld, 0, ti * BM + cl < ld ? ti * BM + cl : 0);
        srcB[q] = bin + NW * gd.off + word_pos(NW, ld, 0, tj * BM + cl < ld ? tj * BM + cl : 0);
    }

    const int row_w = ti * BM + wr * 64, col_w = tj * BM + wc * 64;
    const bool wave_live = (row_w < ld) && (col_w < ld) && !(ti == tj && wr < wc);

    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    const int nk = ld / BK;             // ld is a multiple of 32
    // register-prefetch path: chunk u = tid + 256 q of an operand's K step is
    // 16-B part u % (4 NW) of tile column u / (4 NW) (word p / 4, chunk p % 4);
    // columns beyond ld read column ld - 1 instead (their products reach only
    // discarded outputs).  Offsets are recomputed per load to spare registers.
    constexpr int RQ = RP ? 2 * NW : 1;     // chunks per thread and operand
    u4 stA[RQ], stB[RQ];
    const unsigned short *gA = xin + NW * gd.off, *gB = bin + NW * gd.off;
    auto rp_load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < RQ; q++) {
            const int u = tid + 256 * q;
            const int cl = u / (4 * NW), pp = u % (4 * NW);
            const int ca = min(ti * BM + cl, ld - 1), cb = min(tj * BM + cl, ld - 1);
            // NW n_pad^2 < 2^31 (the host's choice of variant)
            stA[q] = *reinterpret_cast<const u4 *>(gA + (ca * ld * NW + pp * 8 + NW * k0));
            stB[q] = *reinterpret_cast<const u4 *>(gB + (cb * ld * NW + pp * 8 + NW * k0));
        }
    };
    auto rp_store = [&]() {
#pragma unroll
        for (int q = 0; q < RQ; q++) {
            const int u = tid + 256 * q;
            const int cl = u / (4 * NW), pp = u % (4 * NW);
            const int d = (pp / 4) * PH + cl * BK + (((pp % 4) ^ swz(cl)) * 8);
            *reinterpret_cast<u4 *>(Ls + d) = stA[q];
            *reinterpret_cast<u4 *>(Ls + NW * PH + d) = stB[q];
        }
    };
    if constexpr (RP) {
        rp_load(0);
        rp_store();
        wait_lgkm0();
        lds_barrier();
    }
    for (int kt = 0; kt < nk; kt++) {
        const int k0 = kt * BK;
        if constexpr (RP) {
            if (kt + 1 < nk) rp_load(k0 + BK);       // in flight during this step's products
        } else {
#pragma unroll
            for (int w = 0; w < NW; w++)
#pragma unroll
                for (int q = 0; q < 2; q++) {
                    unsigned short *dA = Ls + (0 * NW + w) * PH + (wave + 4 * q) * 16 * BK;
                    unsigned short *dB = Ls + (1 * NW + w) * PH + (wave + 4 * q) * 16 * BK;
                    __builtin_amdgcn_global_load_lds(
                        (const __attribute__((address_space(1))) void *)(srcA[q] + NW * k0 + 32 * w + kcoff[q]),
                        (__attribute__((address_space(3))) void *)dA, 16, 0, 0);
                    __builtin_amdgcn_global_load_lds(
                        (const __attribute__((address_space(1))) void *)(srcB[q] + NW * k0 + 32 * w + kcoff[q]),
                        (__attribute__((address_space(3))) void *)dB, 16, 0, 0);
                }
            wait_vm0();
            lds_barrier();                  // every wave's loads of this step are in LDS
        }
        if (wave_live) {
            u16x8 bv[4][NW];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int cb = wc * 64 + j * 16 + li;
#pragma unroll
                for (int w = 0; w < NW; w++)
                    bv[j][w] = *reinterpret_cast<const u16x8 *>(Ls + (1 * NW + w) * PH + cb * BK + ((lg ^ swz(cb)) * 8));
            }
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int ca = wr * 64 + i * 16 + li;
                u16x8 av[NW];
#pragma unroll
                for (int w = 0; w < NW; w++)
                    av[w] = *reinterpret_cast<const u16x8 *>(Ls + (0 * NW + w) * PH + ca * BK + ((lg ^ swz(ca)) * 8));
#pragma unroll
                for (int pr = npairs<NW>() - 1; pr >= 0; pr--)      // least significant products first
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        acc[i][j] = mfma16<FMT>(av[pair_p(pr)], bv[j][pair_q(pr)], acc[i][j]);
            }
        }
        lds_barrier();                  // every wave is done reading before the next loads land
        if constexpr (RP) {
            if (kt + 1 < nk) {
                rp_store();
                wait_lgkm0();
                lds_barrier();          // the next step's operands are in LDS
            }
        }
    }

    // ---- epilogue, in two rounds over the column halves h of the tile (the
    // waves with wc == h hold them).  Lane l, register v of block (i, j) holds
    // row 16 i + 4 (l / 16) + v and column 16 j + l % 16 of the wave's tile.
    constexpr float inv_s2 = (float)(1.0 / (word_scale<FMT>() * word_scale<FMT>()));
    constexpr float sc = (float)word_scale<FMT>();
    const int n = gd.n;
    const bool diag = (ti == tj);
    unsigned short *og = out + NW * gd.off;
    float rmax = 0.f;
    if constexpr (NW <= 2) {
        // One conversion per element: the pass over the tile's own positions
        // splits every staged value into its words and writes them back in
        // place, one 32-bit (w0 | w1 << 16) per element; the mirror pass then
        // reads those words across the staging columns.  Staging is
        // column-major with the row index XOR-swizzled in 16-B steps by column
        // group of 8, so that the mirror's reads (8 rows x 8 columns per wave
        // instruction) fall on 64 distinct banks.
        auto cpos = [](int col, int row) { return col * CST + (row ^ (((col >> 3) & 7) << 2)); };
        unsigned int *Cw = reinterpret_cast<unsigned int *>(Cs);
        for (int h = 0; h < 2; h++) {
            if (tj * BM + h * 64 >= ld) break;      // the half lies beyond the matrix
            if (wave_live && wc == h) {
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        *reinterpret_cast<f4 *>(&Cs[cpos(j * 16 + li, wr * 64 + i * 16 + lg * 4)]) = acc[i][j];
            }
            __syncthreads();
#pragma unroll 2
            for (int q = 0; q < 4; q++) {
                const int u = tid + 256 * q;
                const int rc = u & 15, cl = u >> 4;
                const int c = tj * BM + h * 64 + cl, r0 = ti * BM + rc * 8;
                if (c >= ld || r0 >= ld) continue;
                if (diag && r0 + 7 < c) continue;
                // rows rc*8 .. +3 and +4 .. +7: two 16-B slots; lanes with rc & 4 read the second first
                const int p0 = cpos(cl, rc * 8), p1 = cpos(cl, rc * 8 + 4);
                const int sw = rc & 4;
                const f4 fa = *reinterpret_cast<const f4 *>(Cs + (sw ? p1 : p0));
                const f4 fb = *reinterpret_cast<const f4 *>(Cs + (sw ? p0 : p1));
                const f4 lo = sw ? fb : fa, hi = sw ? fa : fb;
                float v[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
                float tv[8] = {};
                if constexpr (MODE == 3) load8_words<FMT, NW>(xin + NW * gd.off, ld, r0, c, tv);
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    const int r = r0 + e;
                    const float t = v[e] * inv_s2;
                    if ((MODE == 0 || MODE == 2) && r < n && c < n && r >= c) {
                        float d = fabsf(t - (r == c ? 1.f : 0.f));
                        if (!(d <= 3.4e38f)) d = __builtin_huge_valf();
                        rmax = fmaxf(rmax, d);
                        if (r == c) it.tdiag[gd.rinfo_off + r] = 1.0 - (double)t;
                    }
                    v[e] = out_value<MODE>(t, tv[e], r, c) * sc;
                }
                u16x8 wv[NW];
                split8<FMT, NW>(v, wv);
#pragma unroll
                for (int w = 0; w < NW; w++)
                    *reinterpret_cast<u16x8 *>(og + word_pos(NW, ld, r0, c) + 32 * w) = wv[w];
                u4 pa, pb;
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    pa[e] = (unsigned int)wv[0][e] | (NW == 2 ? ((unsigned int)wv[NW - 1][e] << 16) : 0u);
                    pb[e] = (unsigned int)wv[0][e + 4] | (NW == 2 ? ((unsigned int)wv[NW - 1][e + 4] << 16) : 0u);
                }
                *reinterpret_cast<u4 *>(Cw + p0) = pa;
                *reinterpret_cast<u4 *>(Cw + p1) = pb;
            }
            __syncthreads();                        // every element's words are staged
            // mirror: tile element (rl, cl) goes to (cl, rl) of the matrix; unit (tile
            // row rl, 8-column chunk cc); in a diagonal tile only positions above
            // the diagonal
#pragma unroll 2
            for (int q = 0; q < 4; q++) {
                const int u = tid + 256 * q;
                const int cc = u & 7, rl = u >> 3;
                const int r = ti * BM + rl, c0 = tj * BM + h * 64 + cc * 8;
                if (r >= ld || c0 >= ld) continue;
                if (diag && c0 >= r) continue;
                u16x8 wv[NW];
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    const unsigned int pk = Cw[cpos(cc * 8 + e, rl)];
                    wv[0][e] = (unsigned short)(pk & 0xffffu);
                    if constexpr (NW == 2) wv[NW - 1][e] = (unsigned short)(pk >> 16);
                }
                if (!diag || c0 + 8 <= r) {
#pragma unroll
                    for (int w = 0; w < NW; w++)
                        *reinterpret_cast<u16x8 *>(og + word_pos(NW, ld, c0, r) + 32 * w) = wv[w];
                } else {
                    for (int e = 0; c0 + e < r; e++)
#pragma unroll
                        for (int w = 0; w < NW; w++) og[word_pos(NW, ld, c0, r) + 32 * w + e] = wv[w][e];
                }
            }
            __syncthreads();                        // staging is free for the next half
        }
    } else
    for (int h = 0; h < 2; h++) {
        if (wave_live && wc == h) {
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++)
                    *reinterpret_cast<f4 *>(&Cs[(j * 16 + li) * CST + wr * 64 + i * 16 + lg * 4]) = acc[i][j];
        }
        __syncthreads();
        // the tile's own positions: unit (column cl of the half, 8-row chunk rc);
        // 8-row chunks above the diagonal of a diagonal tile are the mirror's
#pragma unroll 2
        for (int q = 0; q < 4; q++) {
            const int u = tid + 256 * q;
            const int rc = u & 15, cl = u >> 4;
            const int c = tj * BM + h * 64 + cl, r0 = ti * BM + rc * 8;
            if (c >= ld || r0 >= ld) continue;
            if (diag && r0 + 7 < c) continue;
            float v[8];
            load8(&Cs[cl * CST + rc * 8], rc & 4, v);
            float tv[8] = {};
            if constexpr (MODE == 3) load8_words<FMT, NW>(xin + NW * gd.off, ld, r0, c, tv);
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int r = r0 + e;
                const float t = v[e] * inv_s2;
                if ((MODE == 0 || MODE == 2) && r < n && c < n && r >= c) {
                    float d = fabsf(t - (r == c ? 1.f : 0.f));
                    if (!(d <= 3.4e38f)) d = __builtin_huge_valf();
                    rmax = fmaxf(rmax, d);
                    if (r == c) it.tdiag[gd.rinfo_off + r] = 1.0 - (double)t;
                }
                v[e] = out_value<MODE>(t, tv[e], r, c) * sc;
            }
            u16x8 wv[NW];
            split8<FMT, NW>(v, wv);
#pragma unroll
            for (int w = 0; w < NW; w++)
                *reinterpret_cast<u16x8 *>(og + word_pos(NW, ld, r0, c) + 32 * w) = wv[w];
        }
        __syncthreads();                // Cs reads done; direct stores precede the mirror's
        if (wave_live && wc == h) {
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++)
#pragma unroll
                    for (int v = 0; v < 4; v++)
                        Cs[(wr * 64 + i * 16 + lg * 4 + v) * CSTH + j * 16 + li] = acc[i][j][v];
        }
        __syncthreads();
        // mirror: tile element (rl, cl) goes to (cl, rl) of the matrix; unit (tile
        // row rl, 8-column chunk cc); in a diagonal tile only positions above
        // the diagonal
#pragma unroll 2
        for (int q = 0; q < 4; q++) {
            const int u = tid + 256 * q;
            const int cc = u & 7, rl = u >> 3;
            const int r = ti * BM + rl, c0 = tj * BM + h * 64 + cc * 8;
            if (r >= ld || c0 >= ld) continue;
            if (diag && c0 >= r) continue;
            float v[8];
            load8(&Cs[rl * CSTH + cc * 8], cc & 4, v);
            float tv[8] = {};     // T is symmetric: T_{r, c0 + e} from column r
            if constexpr (MODE == 3) load8_words<FMT, NW>(xin + NW * gd.off, ld, c0, r, tv);
#pragma unroll
            for (int e = 0; e < 8; e++) v[e] = out_value<MODE>(v[e] * inv_s2, tv[e], r, c0 + e) * sc;
            u16x8 wv[NW];
            split8<FMT, NW>(v, wv);
            if (!diag || c0 + 8 <= r) {
#pragma unroll
                for (int w = 0; w < NW; w++)
                    *reinterpret_cast<u16x8 *>(og + word_pos(NW, ld, c0, r) + 32 * w) = wv[w];
            } else {
                for (int e = 0; c0 + e < r; e++)
#pragma unroll
                    for (int w = 0; w < NW; w++) og[word_pos(NW, ld, c0, r) + 32 * w + e] = wv[w][e];
            }
        }
        __syncthreads();
    }

    if (MODE == 0 || MODE == 2) {
        double rm = (double)rmax;
        rm = wave_max(rm);
        if (lane == 0)
            atomicMax(it.resid_bits + (int64_t)g * it.resid_stride + k, (unsigned long long)__double_as_longlong(rm));
    }
}

// One 128 x 128 output tile per workgroup (grid = the launch order's tiles).
template <int FMT, int NW, int MODE, int RP>
__global__ __launch_bounds__(256, 2)
void ns_words_kernel(const TileDesc *__restrict__ tiles, const GroupDesc *__restrict__ groups,
                     const unsigned short *__restrict__ xin, const unsigned short *__restrict__ bin,
                     unsigned short *__restrict__ out, IterState it, int k,
                     double switch_tol, int kmax)
{
    ns_words_tile<FMT, NW, MODE, RP>(tiles[blockIdx.x], groups, xin, bin, out, it, k, switch_tol, kmax);
}

// Persistent launch: as many workgroups as the CUs hold at once, each taking
// tiles from work lists, one per XCD (tiles of a group share one list, so
// their operand panels meet in one L2), through an atomic counter per list.
// A workgroup starts with the list of the XCD it runs on (hardware register
// XCC_ID) and then takes what is left in the others, so every tile is taken
// exactly once whatever the placement.  No workgroup waits on another: each
// list's counter only grows, and a workgroup leaves once all eight are past
// their ends.
template <int FMT, int NW, int MODE>
__global__ __launch_bounds__(256, 3)
void ns_words_persistent(const TileDesc *__restrict__ tiles_x, const int32_t *__restrict__ xbeg,
                         int32_t *__restrict__ cnt, const GroupDesc *__restrict__ groups,
                         const unsigned short *__restrict__ xin, const unsigned short *__restrict__ bin,
                         unsigned short *__restrict__ out, IterState it, int k, double switch_tol, int kmax)
{
    __shared__ int s_q;
    // s_getreg of HW_REG_XCC_ID (id 20, bits 3:0)
    const int x0 = (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7);
    for (int d = 0; d < 8; d++) {
        const int x = (x0 + d) & 7;
        const int base = xbeg[x], len = xbeg[x + 1] - base;
        for (;;) {
            if (threadIdx.x == 0) s_q = atomicAdd(cnt + x, 1);
            __syncthreads();
            const int q = s_q;
            __syncthreads();                    // every lane has read s_q before it is taken again
            if (q >= len) break;
            ns_words_tile<FMT, NW, MODE, 0>(tiles_x[base + q], groups, xin, bin, out, it, k, switch_tol, kmax);
            __syncthreads();                    // LDS free for the next tile
        }
    }
}

// ---- 256 x 256 output tiles (one and two words) ---------------------------
// The 128 x 128 tile moves 2 nw x (128 + 128) x 32 bytes from L2 into LDS per
// K step for 128 x 128 x 32 multiply-adds per word product; the operand
// stream (bounded by the L2 requests a CU keeps in flight) then takes longer
// than the matrix-core work.  A 256 x 256 tile halves the bytes per product.
// One workgroup of 512 lanes per CU: eight waves, two per SIMD, wave (wr, wc)
// holds rows 64 wr .. + 63 and columns 128 wc .. + 127 of the tile (128 FP32
// accumulators per lane).  Operands are double-buffered in LDS (two stages of
// 2 nw x 16 KB): the loads of K step t + 1 are in flight while the matrix
// cores work on step t.  Per output element the sequence of matrix-core
// operations (K steps in order, word pairs least significant first) is the
// one of the 128 x 128 kernel, so both tile shapes give the same bits.
// A wave whose 64 x 128 part lies wholly above the diagonal of a diagonal
// tile, or outside the matrix, does no products, and operand column groups
// wholly outside the matrix are not loaded (no output they feed is stored).
constexpr int BM2 = 256;
constexpr int CST2 = 260;          // column-major staging of a 64-column quarter: 1040-B columns

template <int NW>
__host__ __device__ constexpr int words256_lds_bytes()
{
    return (2 * 2 * NW * BM2 * BK * 2) > (64 * CST2 * 4) ? (2 * 2 * NW * BM2 * BK * 2) : (64 * CST2 * 4);
}

template <int FMT, int NW, int MODE>
__global__ __launch_bounds__(512, 1)
void ns_words256_kernel(const TileDesc *__restrict__ tiles, const GroupDesc *__restrict__ groups,
                        const unsigned short *__restrict__ xin, const unsigned short *__restrict__ bin,
                        unsigned short *__restrict__ out, IterState it, int k, double switch_tol, int kmax)
{
    static_assert(NW == 1 || NW == 2, "two stages of three words do not fit the LDS");
    __shared__ __attribute__((aligned(16))) unsigned char smem[words256_lds_bytes<NW>()];
    unsigned short *Ls = reinterpret_cast<unsigned short *>(smem);   // [stage][2 operands][NW][BM2][BK]
    float *Cs = reinterpret_cast<float *>(smem);                     // staging after the K loop

    const TileDesc td = tiles[blockIdx.x];
    const int g = td.x;
    if (g < 0) return;                  // idle slot of the launch order
    if (it.done[g]) return;
    const int ti = td.y >> 16, tj = td.y & 0xffff;
    const GroupDesc gd = groups[g];
    const int ld = gd.npad;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);     // wave-uniform: scalar branches

    if (MODE == 1 && bulk_stop(it, gd, g, k, ti == 0 && tj == 0 && tid == 0, lane, switch_tol, kmax, NW > 1))
        return;

    const int wr = wave >> 1, wc = wave & 1;
    const int li = lane & 15;
    const int lg = lane >> 4;
    const bool diag = (ti == tj);

    // Loads: instruction (operand, word, 16-column group q = wave + 8 qq) fills
    // 1 KB of LDS; lane l fills slot l % 4 of column 16 q + l / 4 with chunk
    // (slot ^ swz(column)) of that column's K step.  Column groups that lie
    // wholly beyond ld are not loaded (their LDS rows feed only products that
    // reach discarded outputs); single columns beyond ld read column 0.
    constexpr int PH = BM2 * BK;        // halves per (operand, word) region
    constexpr int STG = 2 * NW * PH;    // halves per stage
    const unsigned short *srcA[2], *srcB[2];
    int kcoff[2];
#pragma unroll
    for (int qq = 0; qq < 2; qq++) {
        const int cl = (wave + 8 * qq) * 16 + lane / CPC;
        kcoff[qq] = ((lane % CPC) ^ swz(cl)) * 8;
        srcA[qq] = xin + NW * gd.off + word_pos(NW, ld, 0, ti * BM2 + cl < ld ? ti * BM2 + cl : 0);
        srcB[qq] = bin + NW * gd.off + word_pos(NW, ld, 0, tj * BM2 + cl < ld ? tj * BM2 + cl : 0);
    }
    bool ldA[2], ldB[2];                // wave-uniform: the column group has a column inside the matrix
#pragma unroll
    for (int qq = 0; qq < 2; qq++) {
        ldA[qq] = ti * BM2 + (wave + 8 * qq) * 16 < ld;
        ldB[qq] = tj * BM2 + (wave + 8 * qq) * 16 < ld;
    }
    // load instruction m (0 .. 4 NW - 1: operand m & 1, column group qq = (m >> 1) & 1,
    // word m >> 2) of K step kt into stage s
    constexpr int NLD = 4 * NW;
    auto issue_one = [&](int m, int kt, int s) {
        const int o = m & 1, qq = (m >> 1) & 1, w = m >> 2;
        const bool on = o ? ldB[qq] : ldA[qq];
        if (!on) return;
        const unsigned short *src = (o ? srcB[qq] : srcA[qq]) + NW * (kt * BK) + 32 * w + kcoff[qq];
        unsigned short *dst = Ls + s * STG + (o * NW + w) * PH + (wave + 8 * qq) * 16 * BK;
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                         (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
    };
    auto issue = [&](int kt, int s) {
#pragma unroll
        for (int m = 0; m < NLD; m++) issue_one(m, kt, s);
    };

    // waves whose part of the tile holds an output that is stored: inside the
    // matrix and, in a diagonal tile, not entirely above the diagonal
    const int row_w = wr * 64, col_w = wc * 128;          // tile-local
    const bool wave_live = (ti * BM2 + row_w < ld) && (tj * BM2 + col_w < ld) && !(diag && row_w + 63 < col_w);

    f4 acc[4][8];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 8; j++) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    const int nk = ld / BK;             // ld is a multiple of 32
    issue(0, 0);
    wait_vm0();
    lds_barrier();
    for (int kt = 0; kt < nk; kt++) {
        const int s = kt & 1;
        const bool more = kt + 1 < nk;   // stage s ^ 1 was last read before the previous barrier
        if (wave_live) {
            const unsigned short *La = Ls + s * STG;
            const unsigned short *Lb = Ls + s * STG + NW * PH;
            u16x8 av[4][NW], bv[2][NW];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int ca = row_w + i * 16 + li;
#pragma unroll
                for (int w = 0; w < NW; w++)
                    av[i][w] = *reinterpret_cast<const u16x8 *>(La + w * PH + ca * BK + ((lg ^ swz(ca)) * 8));
            }
            auto load_b = [&](int j, u16x8 *dst) {
                const int cb = col_w + j * 16 + li;
#pragma unroll
                for (int w = 0; w < NW; w++)
                    dst[w] = *reinterpret_cast<const u16x8 *>(Lb + w * PH + cb * BK + ((lg ^ swz(cb)) * 8));
            };
            load_b(0, bv[0]);
            // the next K step's operand loads are spread over the column blocks
            // (a wave issues its memory instructions in order, so a burst of
            // them would hold back its products while the address unit drains);
            // the B fragments of column block j + 1 are read while the matrix
            // cores work on block j; the four row blocks interleave so that no
            // product waits on the one before it
#pragma unroll
            for (int j = 0; j < 8; j++) {
                if (more && (j * NLD) % 8 == 0) issue_one(j * NLD / 8, kt + 1, s ^ 1);
                if (j + 1 < 8) load_b(j + 1, bv[(j + 1) & 1]);
#pragma unroll
                for (int pr = npairs<NW>() - 1; pr >= 0; pr--)          // least significant products first
#pragma unroll
                    for (int i = 0; i < 4; i++)
                        acc[i][j] = mfma16<FMT>(av[i][pair_p(pr)], bv[j & 1][pair_q(pr)], acc[i][j]);
            }
        } else if (more) {
            issue(kt + 1, s ^ 1);
        }
        wait_vm0();
        lds_barrier();                  // step t + 1 is in LDS and every wave is done with step t
    }

    // ---- epilogue, in four rounds over 64-column quarters of the tile (the
    // waves with wc == quarter / 2 hold them, in accumulator columns 4 (quarter
    // % 2) .. + 3).  Lane l, register v of block (i, j) holds row 16 i + 4 (l /
    // 16) + v and column 16 j + l % 16 of the wave's part.  As in the 128 x 128
    // kernel: one conversion per element, the words of each element are put
    // back into the staging for the mirror pass, staging rows XOR-swizzled by
    // column group so that the mirror's reads are free of bank conflicts.
    constexpr float inv_s2 = (float)(1.0 / (word_scale<FMT>() * word_scale<FMT>()));
    constexpr float sc = (float)word_scale<FMT>();
    const int n = gd.n;
    unsigned short *og = out + NW * gd.off;
    float rmax = 0.f;
    auto cpos = [](int col, int row) { return col * CST2 + (row ^ (((col >> 3) & 7) << 2)); };
    unsigned int *Cw = reinterpret_cast<unsigned int *>(Cs);
#pragma unroll
    for (int q4 = 0; q4 < 4; q4++) {
        if (tj * BM2 + q4 * 64 >= ld) break;        // the quarter lies beyond the matrix
        if (wave_live && wc == (q4 >> 1)) {
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++)
                    *reinterpret_cast<f4 *>(&Cs[cpos(j * 16 + li, row_w + i * 16 + lg * 4)]) = acc[i][(q4 & 1) * 4 + j];
        }
        __syncthreads();
        // the tile's own positions: unit (column cl of the quarter, 8-row chunk rc)
#pragma unroll 2
        for (int qq = 0; qq < 4; qq++) {
            const int u = tid + 512 * qq;
            const int rc = u & 31, cl = u >> 5;
            const int c = tj * BM2 + q4 * 64 + cl, r0 = ti * BM2 + rc * 8;
            if (c >= ld || r0 >= ld) continue;
            if (diag && r0 + 7 < c) continue;
            const int p0 = cpos(cl, rc * 8), p1 = cpos(cl, rc * 8 + 4);
            const int sw = rc & 4;
            const f4 fa = *reinterpret_cast<const f4 *>(Cs + (sw ? p1 : p0));
            const f4 fb = *reinterpret_cast<const f4 *>(Cs + (sw ? p0 : p1));
            const f4 lo = sw ? fb : fa, hi = sw ? fa : fb;
            float v[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
            float tv[8] = {};
            if constexpr (MODE == 3) load8_words<FMT, NW>(xin + NW * gd.off, ld, r0, c, tv);
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int r = r0 + e;
                const float t = v[e] * inv_s2;
                if ((MODE == 0 || MODE == 2) && r < n && c < n && r >= c) {
                    float d = fabsf(t - (r == c ? 1.f : 0.f));
                    if (!(d <= 3.4e38f)) d = __builtin_huge_valf();
                    rmax = fmaxf(rmax, d);
                    if (r == c) it.tdiag[gd.rinfo_off + r] = 1.0 - (double)t;
                }
                v[e] = out_value<MODE>(t, tv[e], r, c) * sc;
            }
            u16x8 wv[NW];
            split8<FMT, NW>(v, wv);
#pragma unroll
            for (int w = 0; w < NW; w++)
                *reinterpret_cast<u16x8 *>(og + word_pos(NW, ld, r0, c) + 32 * w) = wv[w];
            u4 pa, pb;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                pa[e] = (unsigned int)wv[0][e] | (NW == 2 ? ((unsigned int)wv[NW - 1][e] << 16) : 0u);
                pb[e] = (unsigned int)wv[0][e + 4] | (NW == 2 ? ((unsigned int)wv[NW - 1][e + 4] << 16) : 0u);
            }
            *reinterpret_cast<u4 *>(Cw + p0) = pa;
            *reinterpret_cast<u4 *>(Cw + p1) = pb;
        }
        __syncthreads();                            // every element's words are staged
        // mirror: tile element (rl, cl) goes to (cl, rl) of the matrix; unit (tile
        // row rl, 8-column chunk cc); in a diagonal tile only positions above
        // the diagonal
#pragma unroll 2
        for (int qq = 0; qq < 4; qq++) {
            const int u = tid + 512 * qq;
            const int cc = u & 7, rl = u >> 3;
            const int r = ti * BM2 + rl, c0 = tj * BM2 + q4 * 64 + cc * 8;
            if (r >= ld || c0 >= ld) continue;
            if (diag && c0 >= r) continue;
            u16x8 wv[NW];
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const unsigned int pk = Cw[cpos(cc * 8 + e, rl)];
                wv[0][e] = (unsigned short)(pk & 0xffffu);
                if constexpr (NW == 2) wv[NW - 1][e] = (unsigned short)(pk >> 16);
            }
            if (!diag || c0 + 8 <= r) {
#pragma unroll
                for (int w = 0; w < NW; w++)
                    *reinterpret_cast<u16x8 *>(og + word_pos(NW, ld, c0, r) + 32 * w) = wv[w];
            } else {
                for (int e = 0; c0 + e < r; e++)
#pragma unroll
                    for (int w = 0; w < NW; w++) og[word_pos(NW, ld, c0, r) + 32 * w + e] = wv[w][e];
            }
        }
        __syncthreads();                            // staging is free for the next quarter
    }

    if (MODE == 0 || MODE == 2) {
        double rm = (double)rmax;
        rm = wave_max(rm);
        if (lane == 0)
            atomicMax(it.resid_bits + (int64_t)g * it.resid_stride + k, (unsigned long long)__double_as_longlong(rm));
    }
}

// FP32 products (v_mfma_f32_16x16x4_f32, FP32 accumulation): the iterate is
// held as one FP32 value per element.  Same tiling, symmetry use, LDS loads
// (32 k = 128 B per column and step, chunks swizzled over eight positions),
// stopping rule and epilogue as the word products.
__device__ inline int swz8(int col) { return (col ^ (col >> 3)) & 7; }

__host__ __device__ constexpr int f32_lds_bytes()
{
    return (2 * BM * BK * 4) > (BM * CSTH * 4) ? (2 * BM * BK * 4) : (BM * CSTH * 4);
}

template <int MODE>
__global__ __launch_bounds__(256, 2)
void ns_f32_kernel(const TileDesc *__restrict__ tiles, const GroupDesc *__restrict__ groups,
                   const float *__restrict__ xin, const float *__restrict__ bin,
                   float *__restrict__ out, IterState it, int k, double switch_tol, int kmax)
{
    __shared__ __attribute__((aligned(16))) unsigned char smem[f32_lds_bytes()];
    float *Ls = reinterpret_cast<float *>(smem);                     // [2 operands][BM][BK]
    float *Cs = reinterpret_cast<float *>(smem);                     // staging after the K loop

    const TileDesc td = tiles[blockIdx.x];
    const int g = td.x;
    if (g < 0) return;                  // idle slot of the launch order
    if (it.done[g]) return;
    const int ti = td.y >> 16, tj = td.y & 0xffff;
    const GroupDesc gd = groups[g];
    const int ld = gd.npad;

    if (MODE == 1 && bulk_stop(it, gd, g, k, ti == 0 && tj == 0 && threadIdx.x == 0, threadIdx.x & 63, switch_tol,
                               kmax, true))
        return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int li = lane & 15;
    const int lg = lane >> 4;

    // Loads: one wave instruction fills 1 KB of LDS = 8 columns x 128 B (32
    // floats); lane l fills slot l % 8 of column (wave + 4 q) * 8 + l / 8 with
    // chunk (slot ^ swz8(column)) of that column.  Columns beyond ld read any
    // valid address instead (their products only reach discarded outputs).
    constexpr int PH = BM * BK;         // floats per operand region
    const float *srcA[4], *srcB[4];
    int kcoff[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int cl = (wave + 4 * q) * 8 + lane / 8;
        kcoff[q] = ((lane % 8) ^ swz8(cl)) * 4;
        srcA[q] = xin + gd.off + (int64_t)(ti * BM + cl < ld ? ti * BM + cl : 0) * ld;
        srcB[q] = bin + gd.off + (int64_t)(tj * BM + cl < ld ? tj * BM + cl : 0) * ld;
    }

    const int row_w = ti * BM + wr * 64, col_w = tj * BM + wc * 64;
    const bool wave_live = (row_w < ld) && (col_w < ld) && !(ti == tj && wr < wc);

    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    const int nk = ld / BK;             // ld is a multiple of 32
    for (int kt = 0; kt < nk; kt++) {
        const int k0 = kt * BK;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            float *dA = Ls + 0 * PH + (wave + 4 * q) * 8 * BK;
            float *dB = Ls + 1 * PH + (wave + 4 * q) * 8 * BK;
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(srcA[q] + k0 + kcoff[q]),
                                             (__attribute__((address_space(3))) void *)dA, 16, 0, 0);
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(srcB[q] + k0 + kcoff[q]),
                                             (__attribute__((address_space(3))) void *)dB, 16, 0, 0);
        }
        wait_vm0();
        lds_barrier();                  // every wave's loads of this step are in LDS
        if (wave_live) {
            // two halves of 16 k; lane group lg holds k = 16 h + 4 lg + (0..3), and
            // product j takes component j: the same permutation of k on both sides
#pragma unroll
            for (int h = 0; h < 2; h++) {
                f4 bv[4];
#pragma unroll
                for (int jj = 0; jj < 4; jj++) {
                    const int cb = wc * 64 + jj * 16 + li;
                    bv[jj] = *reinterpret_cast<const f4 *>(Ls + 1 * PH + cb * BK + (((h * 4 + lg) ^ swz8(cb)) * 4));
                }
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const int ca = wr * 64 + i * 16 + li;
                    const f4 av = *reinterpret_cast<const f4 *>(Ls + 0 * PH + ca * BK + (((h * 4 + lg) ^ swz8(ca)) * 4));
#pragma unroll
                    for (int j = 0; j < 4; j++)
#pragma unroll
                        for (int jj = 0; jj < 4; jj++)
                            acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[j], bv[jj][j], acc[i][jj], 0, 0, 0);
                }
            }
        }
        lds_barrier();                  // every wave is done reading before the next loads land
    }

    // ---- epilogue, in two rounds over the column halves h of the tile (the
    // waves with wc == h hold them).  Lane l, register v of block (i, j) holds
    // row 16 i + 4 (l / 16) + v and column 16 j + l % 16 of the wave's tile.
    const int n = gd.n;
    const bool diag = (ti == tj);
    float *og = out + gd.off;
    float rmax = 0.f;
    for (int h = 0; h < 2; h++) {
        if (wave_live && wc == h) {
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++)
                    *reinterpret_cast<f4 *>(&Cs[(j * 16 + li) * CST + wr * 64 + i * 16 + lg * 4]) = acc[i][j];
        }
        __syncthreads();
        // the tile's own positions: unit (column cl of the half, 8-row chunk rc);
        // 8-row chunks above the diagonal of a diagonal tile are the mirror's
#pragma unroll 2
        for (int q = 0; q < 4; q++) {
            const int u = tid + 256 * q;
            const int rc = u & 15, cl = u >> 4;
            const int c = tj * BM + h * 64 + cl, r0 = ti * BM + rc * 8;
            if (c >= ld || r0 >= ld) continue;
            if (diag && r0 + 7 < c) continue;
            float v[8];
            load8(&Cs[cl * CST + rc * 8], rc & 4, v);
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int r = r0 + e;
                const float t = v[e];
                if ((MODE == 0 || MODE == 2) && r < n && c < n && r >= c) {
                    float d = fabsf(t - (r == c ? 1.f : 0.f));
                    if (!(d <= 3.4e38f)) d = __builtin_huge_valf();
                    rmax = fmaxf(rmax, d);
                    if (r == c) it.tdiag[gd.rinfo_off + r] = 1.0 - (double)t;
                }
                v[e] = out_value<MODE>(t, MODE == 3 ? xin[gd.off + r + (int64_t)c * ld] : 0.f, r, c);
            }
            *reinterpret_cast<f4 *>(og + r0 + (int64_t)c * ld) = f4{v[0], v[1], v[2], v[3]};
            *reinterpret_cast<f4 *>(og + r0 + 4 + (int64_t)c * ld) = f4{v[4], v[5], v[6], v[7]};
        }
        __syncthreads();                // Cs reads done; direct stores precede the mirror's
        if (wave_live && wc == h) {
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++)
#pragma unroll
                    for (int v = 0; v < 4; v++)
                        Cs[(wr * 64 + i * 16 + lg * 4 + v) * CSTH + j * 16 + li] = acc[i][j][v];
        }
        __syncthreads();
        // mirror: tile element (rl, cl) goes to (cl, rl) of the matrix; unit (tile
        // row rl, 8-column chunk cc); in a diagonal tile only positions above
        // the diagonal
#pragma unroll 2
        for (int q = 0; q < 4; q++) {
            const int u = tid + 256 * q;
            const int cc = u & 7, rl = u >> 3;
            const int r = ti * BM + rl, c0 = tj * BM + h * 64 + cc * 8;
            if (r >= ld || c0 >= ld) continue;
            if (diag && c0 >= r) continue;
            float v[8];
            load8(&Cs[rl * CSTH + cc * 8], cc & 4, v);
#pragma unroll
            for (int e = 0; e < 8; e++) v[e] = out_value<MODE>(v[e], MODE == 3 ? xin[gd.off + c0 + e + (int64_t)r * ld] : 0.f, r, c0 + e);
            if (!diag || c0 + 8 <= r) {
                *reinterpret_cast<f4 *>(og + c0 + (int64_t)r * ld) = f4{v[0], v[1], v[2], v[3]};
                *reinterpret_cast<f4 *>(og + c0 + 4 + (int64_t)r * ld) = f4{v[4], v[5], v[6], v[7]};
            } else {
                for (int e = 0; c0 + e < r; e++) og[c0 + e + (int64_t)r * ld] = v[e];
            }
        }
        __syncthreads();
    }

    if (MODE == 0 || MODE == 2) {
        double rm = (double)rmax;
        rm = wave_max(rm);
        if (lane == 0)
            atomicMax(it.resid_bits + (int64_t)g * it.resid_stride + k, (unsigned long long)__double_as_longlong(rm));
    }
}


// X_0 = a A_g, a = 1/s_g (the Gershgorin prescaling, bounds from the row-sum
// pass), gathered straight into the word storage: one thread per row of a
// 256-row chunk, as the FP64 gather.
template <int FMT, int NW>
__global__ __launch_bounds__(256)
void gather_words_kernel(const int2 *__restrict__ chunks, const GroupDesc *__restrict__ groups,
                         const RowInfo *__restrict__ rinfo, const int32_t *__restrict__ bmap,
                         const int32_t *__restrict__ boffs, const int64_t *__restrict__ valoff,
                         const double *__restrict__ kvals, double mu,
                         const unsigned long long *__restrict__ scale_bits, unsigned short *__restrict__ dst)
{
    const int2 ch = chunks[blockIdx.x];
    const GroupDesc gd = groups[ch.x];
    const int r = ch.y + (int)threadIdx.x;
    const int ld = gd.npad;
    if (r >= ld) return;
    const double s = __longlong_as_double((long long)scale_bits[ch.x]);
    const double a = s > 0.0 ? 1.0 / s : 0.0;
    unsigned short *d = dst + NW * gd.off;
    auto store = [&](int c, double v) {
        unsigned short w[NW];
        split_words<FMT, NW>(a * v * word_scale<FMT>(), w);
        unsigned short *p = d + word_pos(NW, ld, r, c);
#pragma unroll
        for (int q = 0; q < NW; q++) p[32 * q] = w[q];
    };
    gather_row(gd, r, rinfo, bmap, boffs, valoff, kvals, mu, store);
    // padding columns: exactly the identity (not prescaled): 1 is a fixed point
    // of the iteration, whereas 1/s_g would leave [-1, 1] for s_g < 1
    for (int c = gd.n; c < ld; c++) {
        unsigned short w[NW];
        split_words<FMT, NW>(r == c ? word_scale<FMT>() : 0.0, w);
        unsigned short *p = d + word_pos(NW, ld, r, c);
#pragma unroll
        for (int q = 0; q < NW; q++) p[32 * q] = w[q];
    }
}

// The same for FP32 values (column-major like the FP64 slabs).
__global__ __launch_bounds__(256)
void gather_f32_kernel(const int2 *__restrict__ chunks, const GroupDesc *__restrict__ groups,
                       const RowInfo *__restrict__ rinfo, const int32_t *__restrict__ bmap,
                       const int32_t *__restrict__ boffs, const int64_t *__restrict__ valoff,
                       const double *__restrict__ kvals, double mu,
                       const unsigned long long *__restrict__ scale_bits, float *__restrict__ dst)
{
    const int2 ch = chunks[blockIdx.x];
    const GroupDesc gd = groups[ch.x];
    const int r = ch.y + (int)threadIdx.x;
    const int ld = gd.npad;
    if (r >= ld) return;
    const double s = __longlong_as_double((long long)scale_bits[ch.x]);
    const double a = s > 0.0 ? 1.0 / s : 0.0;
    float *d = dst + gd.off;
    gather_row(gd, r, rinfo, bmap, boffs, valoff, kvals, mu, [&](int c, double v) { d[r + (int64_t)c * ld] = (float)(a * v); });
    for (int c = gd.n; c < ld; c++) d[r + (int64_t)c * ld] = (r == c) ? 1.0f : 0.0f;   // the identity, not prescaled
}

// fp64 copy of the bulk result X_kfinal (sum of its words).
template <int FMT, int NW>
__global__ __launch_bounds__(256)
void words_to_f64_kernel(const GroupDesc *__restrict__ groups, const unsigned short *__restrict__ x0,
                         const unsigned short *__restrict__ x1, const int32_t *__restrict__ kfinal,
                         double *__restrict__ dst, int g0)
{
    const int g = g0 + blockIdx.y;
    const GroupDesc gd = groups[g];
    const int ld = gd.npad;
    const unsigned short *src = ((kfinal[g] & 1) ? x1 : x0) + NW * gd.off;
    for (int c = blockIdx.x; c < ld; c += gridDim.x)
        for (int r = threadIdx.x; r < ld; r += 256) {
            const unsigned short *p = src + word_pos(NW, ld, r, c);
            double v = 0.0;
#pragma unroll
            for (int w = NW - 1; w >= 0; w--) v += from_word<FMT>(p[32 * w]);
            dst[gd.off + r + (int64_t)c * ld] = v * (1.0 / word_scale<FMT>());
        }
}

// FP64 copy of the FP32 bulk result.
__global__ __launch_bounds__(256)
void f32_to_f64_kernel(const GroupDesc *__restrict__ groups, const float *__restrict__ x0,
                       const float *__restrict__ x1, const int32_t *__restrict__ kfinal, double *__restrict__ dst,
                       int g0)
{
    const int g = g0 + blockIdx.y;
    const GroupDesc gd = groups[g];
    const int64_t tot = (int64_t)gd.npad * gd.npad;
    const float *src = ((kfinal[g] & 1) ? x1 : x0) + gd.off;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256)
        dst[gd.off + e] = (double)src[e];
}

template <int FMT, int NW>
hipError_t launch_words_t(hipStream_t st, int mode, int variant, int ntiles, const TileDesc *tiles,
                          const GroupDesc *groups, const unsigned short *x, const unsigned short *b,
                          unsigned short *out, const IterState &it, int k, double switch_tol, int kmax)
{
#define SMX_WK(M, R) hipLaunchKernelGGL((ns_words_kernel<FMT, NW, M, R>), dim3(ntiles), dim3(256), 0, st, tiles, \
                                        groups, x, b, out, it, k, switch_tol, kmax)
    // the register-prefetch stream serves the Newton-Schulz products; the
    // Pade products always use the direct stream
    switch (mode) {
    case 0: if (variant == 1) SMX_WK(0, 1); else SMX_WK(0, 0); break;
    case 1: if (variant == 1) SMX_WK(1, 1); else SMX_WK(1, 0); break;
    case 2: SMX_WK(2, 0); break;
    case 3: SMX_WK(3, 0); break;
    default: return hipErrorInvalidValue;
    }
#undef SMX_WK
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ns_words(hipStream_t st, int fmt, int nw, int mode, int variant, int ntiles, const TileDesc *tiles,
                           const GroupDesc *groups, const unsigned short *x, const unsigned short *b,
                           unsigned short *out, const IterState &it, int k, double switch_tol, int kmax)
{
    if (ntiles <= 0) return hipSuccess;
    if (fmt == 2) {
        const float *xf = reinterpret_cast<const float *>(x), *bf = reinterpret_cast<const float *>(b);
        float *of = reinterpret_cast<float *>(out);
#define SMX_F32(M) hipLaunchKernelGGL(ns_f32_kernel<M>, dim3(ntiles), dim3(256), 0, st, tiles, groups, xf, bf, of, it, \
                                      k, switch_tol, kmax)
        switch (mode) {
        case 0: SMX_F32(0); break;
        case 1: SMX_F32(1); break;
        case 2: SMX_F32(2); break;
        case 3: SMX_F32(3); break;
        default: return hipErrorInvalidValue;
        }
#undef SMX_F32
        return hipGetLastError();
    }
    if (fmt == 0 && nw == 1) return launch_words_t<0, 1>(st, mode, variant, ntiles, tiles, groups, x, b, out, it, k, switch_tol, kmax);
    if (fmt == 0 && nw == 2) return launch_words_t<0, 2>(st, mode, variant, ntiles, tiles, groups, x, b, out, it, k, switch_tol, kmax);
    if (fmt == 1 && nw == 1) return launch_words_t<1, 1>(st, mode, variant, ntiles, tiles, groups, x, b, out, it, k, switch_tol, kmax);
    if (fmt == 1 && nw == 3) return launch_words_t<1, 3>(st, mode, variant, ntiles, tiles, groups, x, b, out, it, k, switch_tol, kmax);
    return hipErrorInvalidValue;
}

hipError_t launch_ns_words_persistent(hipStream_t st, int fmt, int nw, int mode, int nwg, const TileDesc *tiles_x,
                                      const int32_t *xbeg, int32_t *cnt, const GroupDesc *groups,
                                      const unsigned short *x, const unsigned short *b, unsigned short *out,
                                      const IterState &it, int k, double switch_tol, int kmax)
{
    if (nwg <= 0) return hipSuccess;
#define SMX_WP(F, N, M) hipLaunchKernelGGL((ns_words_persistent<F, N, M>), dim3(nwg), dim3(256), 0, st, tiles_x, xbeg, \
                                           cnt, groups, x, b, out, it, k, switch_tol, kmax)
#define SMX_WPM(F, N) switch (mode) {                                  \
        case 0: SMX_WP(F, N, 0); break;                                    \
        case 1: SMX_WP(F, N, 1); break;                                    \
        default: return hipErrorInvalidValue;                              \
        }
    if (fmt == 0 && nw == 2) {
        SMX_WPM(0, 2)
    } else if (fmt == 1 && nw == 1) {
        SMX_WPM(1, 1)
    } else {
        return hipErrorInvalidValue;
    }
#undef SMX_WPM
#undef SMX_WP
    return hipGetLastError();
}

int words_persistent_blocks_per_cu(int fmt, int nw)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    if (fmt == 0 && nw == 2)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ns_words_persistent<0, 2, 0>, 256, 0);
    else if (fmt == 1 && nw == 1)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ns_words_persistent<1, 1, 0>, 256, 0);
    return (e == hipSuccess && nb > 0) ? nb : 2;
}

hipError_t launch_ns_words256(hipStream_t st, int fmt, int nw, int mode, int ntiles, const TileDesc *tiles,
                              const GroupDesc *groups, const unsigned short *x, const unsigned short *b,
                              unsigned short *out, const IterState &it, int k, double switch_tol, int kmax)
{
    if (ntiles <= 0) return hipSuccess;
#define SMX_W2(F, N, M) hipLaunchKernelGGL((ns_words256_kernel<F, N, M>), dim3(ntiles), dim3(512), 0, st, tiles, \
                                           groups, x, b, out, it, k, switch_tol, kmax)
#define SMX_W2M(F, N) switch (mode) {                                           \
        case 0: SMX_W2(F, N, 0); break;                                             \
        case 1: SMX_W2(F, N, 1); break;                                             \
        case 2: SMX_W2(F, N, 2); break;                                             \
        case 3: SMX_W2(F, N, 3); break;                                             \
        default: return hipErrorInvalidValue;                                       \
        }
    if (fmt == 0 && nw == 2) { SMX_W2M(0, 2) }
    else if (fmt == 0 && nw == 1) { SMX_W2M(0, 1) }
    else if (fmt == 1 && nw == 1) { SMX_W2M(1, 1) }
    else return hipErrorInvalidValue;
#undef SMX_W2M
#undef SMX_W2
    return hipGetLastError();
}

hipError_t launch_gather_words(hipStream_t st, int fmt, int nw, int nchunks, const int2 *chunks,
                               const GroupDesc *groups, const RowInfo *rinfo, const int32_t *bmap,
                               const int32_t *boffs, const int64_t *valoff, const double *kvals, double mu,
                               const unsigned long long *scale_bits, unsigned short *dst)
{
    if (nchunks <= 0) return hipSuccess;
#define SMX_GW(F, N) hipLaunchKernelGGL((gather_words_kernel<F, N>), dim3(nchunks), dim3(256), 0, st, chunks, groups, \
                                        rinfo, bmap, boffs, valoff, kvals, mu, scale_bits, dst)
    if (fmt == 2)
        hipLaunchKernelGGL(gather_f32_kernel, dim3(nchunks), dim3(256), 0, st, chunks, groups, rinfo, bmap, boffs,
                           valoff, kvals, mu, scale_bits, reinterpret_cast<float *>(dst));
    else if (fmt == 0 && nw == 1) SMX_GW(0, 1);
    else if (fmt == 0 && nw == 2) SMX_GW(0, 2);
    else if (fmt == 1 && nw == 1) SMX_GW(1, 1);
    else if (fmt == 1 && nw == 3) SMX_GW(1, 3);
    else return hipErrorInvalidValue;
#undef SMX_GW
    return hipGetLastError();
}

hipError_t launch_from_words(hipStream_t st, int fmt, int nw, int g0, int ngroups, int max_npad, const GroupDesc *groups,
                             const unsigned short *x0, const unsigned short *x1, const int32_t *kfinal, double *dst)
{
    if (ngroups <= 0) return hipSuccess;
    const int64_t tot = (int64_t)max_npad * max_npad;
    const dim3 grid((unsigned)std::min<int64_t>((tot + 2047) / 2048, 4096), (unsigned)ngroups);
    const dim3 gridc((unsigned)std::min(max_npad, 4096), (unsigned)ngroups);   // one column per block
#define SMX_FW(F, N) hipLaunchKernelGGL((words_to_f64_kernel<F, N>), gridc, dim3(256), 0, st, groups, x0, x1, kfinal, dst, g0)
    if (fmt == 2)
        hipLaunchKernelGGL(f32_to_f64_kernel, grid, dim3(256), 0, st, groups, reinterpret_cast<const float *>(x0),
                           reinterpret_cast<const float *>(x1), kfinal, dst, g0);
    else if (fmt == 0 && nw == 1) SMX_FW(0, 1);
    else if (fmt == 0 && nw == 2) SMX_FW(0, 2);
    else if (fmt == 1 && nw == 1) SMX_FW(1, 1);
    else if (fmt == 1 && nw == 3) SMX_FW(1, 3);
    else return hipErrorInvalidValue;
#undef SMX_FW
    return hipGetLastError();
}

}  // namespace smx
