// Reduced-precision Newton-Schulz products on the gfx950 matrix cores.
//
// The bulk of the sign iteration (Sec. II-B) may run in low precision; the
// paper runs the whole iteration on tensor cores in FP16, "FP16'" (FP16
// multiply, FP32 accumulate) and FP32 and observes energies close to FP64
// (Sec. VII-A, Table I).  Here every iterate is held as NW "words" of a
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
// once tau_k <= switch_tol, or once tau_k stops falling (tau_k < 0.1 and
// tau_k > tau_{k-1} / 2: the floor of the word format), or at the step cap;
// the FP64 polish steps follow.  tau_k is reduced in a fixed order (per
// diagonal tile, then over the tiles), so the decision is reproducible.
#include "smx_internal.h"

namespace smx {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = kTile;   // 128
constexpr int BK = 32;      // K per MFMA step
constexpr int SK = BK + 8;  // LDS row stride in 16-bit words (80 B: 16-B aligned, conflict-free b128 reads)

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

template <int FMT, int NW>
__device__ inline void split_store(unsigned short *o, int64_t plane, int64_t idx, double v)
{
    double rem = v;
#pragma unroll
    for (int w = 0; w < NW; w++) {
        const unsigned short u = to_word<FMT>(rem);
        o[w * plane + idx] = u;
        rem -= from_word<FMT>(u);
    }
}

__device__ inline double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <int FMT, int NW, int MODE>
__global__ __launch_bounds__(256, 2)
void ns_words_kernel(const TileDesc *__restrict__ tiles, const GroupDesc *__restrict__ groups,
                     const unsigned short *__restrict__ xin, const unsigned short *__restrict__ bin,
                     unsigned short *__restrict__ out, int64_t plane, IterState it, int k,
                     double switch_tol, int kmax)
{
    __shared__ unsigned short As[NW][BM][SK];
    __shared__ unsigned short Bs[NW][BM][SK];

    const TileDesc td = tiles[blockIdx.x];
    const int g = td.x;
    if (it.done[g]) return;
    const int ti = td.y >> 16, tj = td.y & 0xffff;
    const GroupDesc gd = groups[g];
    const int ld = gd.npad;

    if (MODE == 1) {
        const int64_t base = (int64_t)g * it.resid_stride;
        const double rk = __longlong_as_double((long long)it.resid_bits[base + k]);
        const int nt = (ld + BM - 1) / BM;
        double tau = 0.0;
        for (int t = 0; t < nt; t++) tau += it.tau_parts[(int64_t)g * it.tau_nt + t];
        const double tp = k > 0 ? it.tau_hist[base + k - 1] : __builtin_huge_val();
        const bool finite = (rk <= 1.7976931348623157e308) && (fabs(tau) <= 1.7976931348623157e308);
        const bool stall = (tau < 0.1) && (tau > 0.5 * tp);
        if (ti == 0 && tj == 0 && threadIdx.x == 0) it.tau_hist[base + k] = tau;
        if (tau <= switch_tol || stall || k >= kmax || !finite) {
            if (ti == 0 && tj == 0 && threadIdx.x == 0) {
                it.done[g] = 1;
                it.kfinal[g] = k;
                it.flags[g] = finite ? 0 : 2;
                atomicAdd(it.ndone, 1);
            }
            return;
        }
    }

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;

    // staging: thread owns 16 consecutive k (32 B per word plane) of one tile column
    const int lcol = tid >> 1;
    const int lk = (tid & 1) * 16;
    const int ga = ti * BM + lcol;
    const int gb = tj * BM + lcol;
    const bool va = ga < ld, vb = gb < ld;
    const unsigned short *pa = xin + gd.off + (int64_t)ga * ld + lk;
    const unsigned short *pb = bin + gd.off + (int64_t)gb * ld + lk;

    const int row_w = ti * BM + wr * 64, col_w = tj * BM + wc * 64;
    const bool wave_live = (row_w < ld) && (col_w < ld) && !(ti == tj && wr < wc);

    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    u16x8 ra[NW][2], rb[NW][2];
    const u16x8 z8 = {0, 0, 0, 0, 0, 0, 0, 0};
    auto gload = [&](int k0) {
#pragma unroll
        for (int w = 0; w < NW; w++)
#pragma unroll
            for (int h = 0; h < 2; h++) {
                ra[w][h] = va ? *reinterpret_cast<const u16x8 *>(pa + w * plane + k0 + 8 * h) : z8;
                rb[w][h] = vb ? *reinterpret_cast<const u16x8 *>(pb + w * plane + k0 + 8 * h) : z8;
            }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int w = 0; w < NW; w++)
#pragma unroll
            for (int h = 0; h < 2; h++) {
                *reinterpret_cast<u16x8 *>(&As[w][lcol][lk + 8 * h]) = ra[w][h];
                *reinterpret_cast<u16x8 *>(&Bs[w][lcol][lk + 8 * h]) = rb[w][h];
            }
    };

    const int nk = ld / BK;
    const int li = lane & 15;
    const int lq = (lane >> 4) * 8;     // k offset of this lane's 8 operand values
    gload(0);
    for (int kt = 0; kt < nk; kt++) {
        __syncthreads();                // previous step's LDS reads are done
        sstore();
        __syncthreads();
        if (kt + 1 < nk) gload((kt + 1) * BK);
        if (wave_live) {
            u16x8 av[4][NW], bv[4][NW];
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int w = 0; w < NW; w++) {
                    av[i][w] = *reinterpret_cast<const u16x8 *>(&As[w][wr * 64 + i * 16 + li][lq]);
                    bv[i][w] = *reinterpret_cast<const u16x8 *>(&Bs[w][wc * 64 + i * 16 + li][lq]);
                }
#pragma unroll
            for (int pr = npairs<NW>() - 1; pr >= 0; pr--)      // least significant products first
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        acc[i][j] = mfma16<FMT>(av[i][pair_p(pr)], bv[j][pair_q(pr)], acc[i][j]);
        }
    }

    // Epilogue: lane l, register v of block (i, j) holds (row 4*(l/16) + v, column l%16).
    const int n = gd.n;
    double rmax = 0.0;
    double dsum = 0.0;          // sum over this wave's true diagonal of (1 - T_ii)
    if (wave_live) {
#pragma unroll
    for (int i = 0; i < 4; i++) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int c = col_w + j * 16 + li;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int r = row_w + i * 16 + (lane >> 4) * 4 + v;
                const double t = (double)acc[i][j][v] * (1.0 / (word_scale<FMT>() * word_scale<FMT>()));
                double val;
                if (MODE == 0) {
                    if (r < n && c < n) {
                        double d = fabs(t - (r == c ? 1.0 : 0.0));
                        if (!(d <= 1.7976931348623157e308)) d = __builtin_huge_val();
                        rmax = fmax(rmax, d);
                        if (r == c) dsum += 1.0 - t;
                    }
                    val = -0.5 * t + (r == c ? 1.5 : 0.0);
                } else {
                    val = t;
                }
                if (r < ld && c < ld && r >= c) {
                    const double vs = val * word_scale<FMT>();
                    split_store<FMT, NW>(out + gd.off, plane, r + (int64_t)c * ld, vs);
                    if (r > c) split_store<FMT, NW>(out + gd.off, plane, c + (int64_t)r * ld, vs);
                }
            }
        }
    }
    }
    if (MODE == 0) {
        rmax = wave_max(rmax);
        if (lane == 0)
            atomicMax(it.resid_bits + (int64_t)g * it.resid_stride + k, (unsigned long long)__double_as_longlong(rmax));
        if (ti == tj) {
            // fixed-order reduction of the diagonal partials: lanes, then waves
            __shared__ double wsum[4];
            for (int o = 32; o > 0; o >>= 1) dsum += __shfl_xor(dsum, o, 64);
            if (lane == 0) wsum[wave] = dsum;
            __syncthreads();
            if (tid == 0) it.tau_parts[(int64_t)g * it.tau_nt + ti] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
        }
    }
}

// X_0 words = split(a A), a = 1/s_g (the Gershgorin prescaling), one group per blockIdx.y.
template <int FMT, int NW>
__global__ __launch_bounds__(256)
void f64_to_words_kernel(const GroupDesc *__restrict__ groups, const double *__restrict__ src,
                         const unsigned long long *__restrict__ scale_bits, unsigned short *__restrict__ dst,
                         int64_t plane)
{
    const int g = blockIdx.y;
    const GroupDesc gd = groups[g];
    const int64_t tot = (int64_t)gd.npad * gd.npad;
    const double s = __longlong_as_double((long long)scale_bits[g]);
    const double a = s > 0.0 ? 1.0 / s : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256)
        split_store<FMT, NW>(dst + gd.off, plane, e, a * src[gd.off + e] * word_scale<FMT>());
}

// fp64 copy of the bulk result X_kfinal (sum of its words), for the FP64 polish.
template <int FMT, int NW>
__global__ __launch_bounds__(256)
void words_to_f64_kernel(const GroupDesc *__restrict__ groups, const unsigned short *__restrict__ x0,
                         const unsigned short *__restrict__ x1, const int32_t *__restrict__ kfinal,
                         int64_t plane, double *__restrict__ dst)
{
    const int g = blockIdx.y;
    const GroupDesc gd = groups[g];
    const int64_t tot = (int64_t)gd.npad * gd.npad;
    const unsigned short *src = ((kfinal[g] & 1) ? x1 : x0) + gd.off;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        double v = 0.0;
#pragma unroll
        for (int w = NW - 1; w >= 0; w--) v += from_word<FMT>(src[w * plane + e]);
        dst[gd.off + e] = v * (1.0 / word_scale<FMT>());
    }
}

template <int FMT, int NW>
hipError_t launch_words_t(hipStream_t st, int mode, int ntiles, const TileDesc *tiles, const GroupDesc *groups,
                          const unsigned short *x, const unsigned short *b, unsigned short *out, int64_t plane,
                          const IterState &it, int k, double switch_tol, int kmax)
{
    if (mode == 0)
        hipLaunchKernelGGL((ns_words_kernel<FMT, NW, 0>), dim3(ntiles), dim3(256), 0, st, tiles, groups, x, b, out,
                           plane, it, k, switch_tol, kmax);
    else
        hipLaunchKernelGGL((ns_words_kernel<FMT, NW, 1>), dim3(ntiles), dim3(256), 0, st, tiles, groups, x, b, out,
                           plane, it, k, switch_tol, kmax);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ns_words(hipStream_t st, int fmt, int nw, int mode, int ntiles, const TileDesc *tiles,
                           const GroupDesc *groups, const unsigned short *x, const unsigned short *b,
                           unsigned short *out, int64_t plane, const IterState &it, int k, double switch_tol,
                           int kmax)
{
    if (ntiles <= 0) return hipSuccess;
    if (fmt == 0 && nw == 1) return launch_words_t<0, 1>(st, mode, ntiles, tiles, groups, x, b, out, plane, it, k, switch_tol, kmax);
    if (fmt == 0 && nw == 2) return launch_words_t<0, 2>(st, mode, ntiles, tiles, groups, x, b, out, plane, it, k, switch_tol, kmax);
    if (fmt == 1 && nw == 1) return launch_words_t<1, 1>(st, mode, ntiles, tiles, groups, x, b, out, plane, it, k, switch_tol, kmax);
    if (fmt == 1 && nw == 3) return launch_words_t<1, 3>(st, mode, ntiles, tiles, groups, x, b, out, plane, it, k, switch_tol, kmax);
    return hipErrorInvalidValue;
}

hipError_t launch_to_words(hipStream_t st, int fmt, int nw, int ngroups, int max_npad, const GroupDesc *groups,
                           const double *src, const unsigned long long *scale_bits, unsigned short *dst, int64_t plane)
{
    if (ngroups <= 0) return hipSuccess;
    const int64_t tot = (int64_t)max_npad * max_npad;
    const dim3 grid((unsigned)std::min<int64_t>((tot + 2047) / 2048, 4096), (unsigned)ngroups);
    if (fmt == 0 && nw == 1) hipLaunchKernelGGL((f64_to_words_kernel<0, 1>), grid, dim3(256), 0, st, groups, src, scale_bits, dst, plane);
    else if (fmt == 0 && nw == 2) hipLaunchKernelGGL((f64_to_words_kernel<0, 2>), grid, dim3(256), 0, st, groups, src, scale_bits, dst, plane);
    else if (fmt == 1 && nw == 1) hipLaunchKernelGGL((f64_to_words_kernel<1, 1>), grid, dim3(256), 0, st, groups, src, scale_bits, dst, plane);
    else if (fmt == 1 && nw == 3) hipLaunchKernelGGL((f64_to_words_kernel<1, 3>), grid, dim3(256), 0, st, groups, src, scale_bits, dst, plane);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_from_words(hipStream_t st, int fmt, int nw, int ngroups, int max_npad, const GroupDesc *groups,
                             const unsigned short *x0, const unsigned short *x1, const int32_t *kfinal, int64_t plane,
                             double *dst)
{
    if (ngroups <= 0) return hipSuccess;
    const int64_t tot = (int64_t)max_npad * max_npad;
    const dim3 grid((unsigned)std::min<int64_t>((tot + 2047) / 2048, 4096), (unsigned)ngroups);
    if (fmt == 0 && nw == 1) hipLaunchKernelGGL((words_to_f64_kernel<0, 1>), grid, dim3(256), 0, st, groups, x0, x1, kfinal, plane, dst);
    else if (fmt == 0 && nw == 2) hipLaunchKernelGGL((words_to_f64_kernel<0, 2>), grid, dim3(256), 0, st, groups, x0, x1, kfinal, plane, dst);
    else if (fmt == 1 && nw == 1) hipLaunchKernelGGL((words_to_f64_kernel<1, 1>), grid, dim3(256), 0, st, groups, x0, x1, kfinal, plane, dst);
    else if (fmt == 1 && nw == 3) hipLaunchKernelGGL((words_to_f64_kernel<1, 3>), grid, dim3(256), 0, st, groups, x0, x1, kfinal, plane, dst);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace smx
