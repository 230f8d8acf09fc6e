// FP64 Newton-Schulz products on the gfx950 matrix cores.
//
// One step of the second-order Newton-Schulz sign iteration (Sec. II-B),
// X_{k+1} = X_k (3I - X_k^2) / 2, is split into two batched products over
// all submatrices:
//   mode 0 ("square"): T = a^2 X_k X_k; the step-k residual max|T - I| over the
//                      true n_g x n_g part; W = 1.5 I - 0.5 T.
//   mode 1 ("update"): X_{k+1} = a X_k W, unless the step-k residual already
//                      meets the stopping rule (then X_k is the result).
// a = 1/s_g at k = 0 (Gershgorin prescaling folded into the first step), 1 after.
// The third-order Pade iteration X_{k+1} = X_k (15I - 10X_k^2 + 3X_k^4) / 8
// (Sec. VI-A) takes three products per step:
//   mode 5 ("Pade square"):  T = a^2 X_k X_k and its residual, as mode 0, T stored;
//   mode 6 ("Pade combine"): W = (15 I - 10 T + 3 T T) / 8 (T read at the output position);
//   mode 1 ("update") as above.
//
// Every iterate is a polynomial in the symmetric A_g, so X, T and W are
// symmetric and X W = W X.  Each workgroup therefore computes one
// lower-triangle 128 x 128 tile and writes it twice (tile and mirror); both
// operands are read as columns (A(i, k) = X(k, i)), which keeps every global
// load contiguous along k.
//
// Workgroup: 256 threads = 4 waves in a 2 x 2 arrangement, each wave owns a
// 64 x 64 sub-tile = 4 x 4 blocks of v_mfma_f64_16x16x4_f64.  K is staged
// through LDS in steps of 16 with double buffering.  Inside a 16-step the
// k index handed to the matrix core is permuted (lane group q, sub-step t ->
// k = 4q + t) so each lane's four operand values are contiguous in LDS; the
// same permutation is applied to both operands, so the sum is unchanged.
#include "smx_internal.h"

namespace smx {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int BM = kTile;      // 128
constexpr int BK = 16;
constexpr int SK = BK + 2;     // LDS row stride in doubles (breaks bank aliasing)

__device__ inline double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <int MODE>
__global__ __launch_bounds__(256, 2)
void ns_f64_kernel(const TileDesc *__restrict__ tiles, const GroupDesc *__restrict__ groups,
                   const double *__restrict__ xin, const double *__restrict__ bin,
                   double *__restrict__ out, IterState it, int k, double tol, int max_iter, int polish,
                   const double *__restrict__ aux)
{
    __shared__ double As[2][BM][SK];
    __shared__ double Bs[2][BM][SK];

    const TileDesc td = tiles[blockIdx.x];
    const int g = td.x;
    if (g < 0) return;                            // idle slot of the launch order
    if (it.kact >= 0 && it.kfix && it.kact >= it.kfix[g]) return;   // group not in this adjoint step
    if (!polish && (MODE <= 2 || MODE >= 5) && it.done[g]) return;  // finished at an earlier step
    const int ti = td.y >> 16, tj = td.y & 0xffff;
    const GroupDesc gd = groups[g];
    const int ld = gd.npad;

    // the prescaling enters the products that read X_0: squares and the update
    constexpr bool reads_x0 = MODE < 2 || MODE == 5;
    double a = 1.0;
    if (k == 0 && !polish && reads_x0) {
        const double s = __longlong_as_double((long long)it.scale_bits[g]);
        a = s > 0.0 ? 1.0 / s : 0.0;
    }
    if (MODE == 2 && it.done[g]) return;          // tangent only while the group iterates
    if (MODE == 1 && !polish) {
        const double rk = __longlong_as_double((long long)it.resid_bits[(int64_t)g * it.resid_stride + k]);
        const bool finite = rk <= 1.7976931348623157e308;
        const bool stop = it.kfix ? (k >= it.kfix[g]) : (rk <= tol || k >= max_iter);
        if (stop || !finite) {
            if (ti == 0 && tj == 0 && threadIdx.x == 0) {
                it.done[g] = 1;
                it.kfinal[g] = k;
                int fl = 0;
                if (!it.kfix && !(rk <= tol)) fl |= 1;
                if (!finite) fl |= 2;
                it.flags[g] = fl;
                atomicAdd(it.ndone, 1);
            }
            return;
        }
    }

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;

    // global -> LDS staging: a K step is 16 k = 128 B per tile column, i.e. eight
    // 16-B chunks.  Chunk q*256 + tid (q = 0..3) is column 32 q + tid/8, part
    // tid%8: eight consecutive lanes read one full cache line.
    const int part = tid & 7;
    const int col8 = tid >> 3;
    const double *pa = xin + gd.off + (int64_t)(ti * BM + col8) * ld + part * 2;
    const double *pb = bin + gd.off + (int64_t)(tj * BM + col8) * ld + part * 2;
    const int64_t col_stride = (int64_t)32 * ld;

    // waves whose 64 x 64 sub-tile lies wholly in the padding, or strictly
    // above the diagonal of a diagonal tile (never stored), skip the math
    const int row_w = ti * BM + wr * 64, col_w = tj * BM + wc * 64;
    const bool wave_live = (row_w < ld) && (col_w < ld) && (MODE == 4 || !(ti == tj && wr < wc));

    d4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    d2 ra[4], rb[4];
    const d2 z2 = {0.0, 0.0};
    auto gload = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; q++) {
            ra[q] = (ti * BM + 32 * q + col8 < ld) ? *reinterpret_cast<const d2 *>(pa + q * col_stride + k0) : z2;
            rb[q] = (tj * BM + 32 * q + col8 < ld) ? *reinterpret_cast<const d2 *>(pb + q * col_stride + k0) : z2;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; q++) {
            *reinterpret_cast<d2 *>(&As[buf][32 * q + col8][part * 2]) = ra[q];
            *reinterpret_cast<d2 *>(&Bs[buf][32 * q + col8][part * 2]) = rb[q];
        }
    };

    const int nk = ld / BK;
    gload(0);
    sstore(0);
    __syncthreads();

    const int li = lane & 15;
    const int lq = (lane >> 4) * 4;
    for (int kt = 0; kt < nk; kt++) {
        const int buf = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * BK);
        if (wave_live) {
            d4 av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const double *sa = &As[buf][wr * 64 + i * 16 + li][lq];
                const double *sb = &Bs[buf][wc * 64 + i * 16 + li][lq];
                const d2 a0 = *reinterpret_cast<const d2 *>(sa);
                const d2 a1 = *reinterpret_cast<const d2 *>(sa + 2);
                const d2 b0 = *reinterpret_cast<const d2 *>(sb);
                const d2 b1 = *reinterpret_cast<const d2 *>(sb + 2);
                av[i] = d4{a0.x, a0.y, a1.x, a1.y};
                bv[i] = d4{b0.x, b0.y, b1.x, b1.y};
            }
#pragma unroll
            for (int t = 0; t < 4; t++)
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][t], bv[j][t], acc[i][j], 0, 0, 0);
        }
        if (kt + 1 < nk) sstore(buf ^ 1);
        __syncthreads();
    }

    if (!wave_live) return;

    // Epilogue.  Block (i, j) of this wave, lane l, register v holds element
    // (row l/16 + 4 v, column l%16) of the 16 x 16 block (the f64 16x16x4
    // output layout; operands: lane l gives A[l%16][l/16] and B[l/16][l%16]).
    double *og = out + gd.off;
    const int n = gd.n;
    // The prescaling a = 1/s_g belongs to the true n_g x n_g block only: the
    // padded identity is a fixed point of the iteration and must stay exactly
    // I (a scaled padding entry 1/s_g would leave [-1, 1] when s_g < 1 and
    // grow without bound).  The padding never mixes with the true block, so
    // setting it after the product is exact.
    const bool pad_fix = (k == 0 && !polish && reads_x0);
    double rmax = 0.0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int c = col_w + j * 16 + li;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int r = row_w + i * 16 + (lane >> 4) + 4 * v;
                double val;
                if (MODE == 0 || MODE == 5) {
                    const double t = a * a * acc[i][j][v];
                    if (r < n && c < n) {
                        double d = fabs(t - (r == c ? 1.0 : 0.0));
                        if (!(d <= 1.7976931348623157e308)) d = __builtin_huge_val();
                        rmax = fmax(rmax, d);
                    }
                    val = MODE == 0 ? -0.5 * t + (r == c ? 1.5 : 0.0) : t;
                } else if (MODE == 6) {
                    // W = (15 I - 10 T + 3 T^2) / 8, T = x at this position
                    val = (r < ld && c < ld)
                              ? 0.125 * ((r == c ? 15.0 : 0.0) - 10.0 * xin[gd.off + r + (int64_t)c * ld] + 3.0 * acc[i][j][v])
                              : 0.0;
                } else if (MODE == 1) {
                    val = a * acc[i][j][v];
                } else if (MODE == 2) {
                    // tangent: 3 Xd W - 3 Xd (Xd and W commute, so the product is symmetric)
                    val = (r < ld && c < ld) ? 3.0 * acc[i][j][v] - 3.0 * xin[gd.off + r + (int64_t)c * ld] : 0.0;
                } else if (MODE == 3) {
                    // adjoint step: Xb_k = -1.5 Xb + Z + Z^T - 0.5 X (Xb X), Z = Xb W
                    val = 0.0;
                    if (r < ld && c < ld && r >= c)
                        val = -1.5 * og[r + (int64_t)c * ld] + aux[gd.off + r + (int64_t)c * ld] +
                              aux[gd.off + c + (int64_t)r * ld] - 0.5 * acc[i][j][v];
                } else {
                    val = acc[i][j][v];
                }
                if (pad_fix && (r >= n || c >= n)) val = (r == c) ? 1.0 : 0.0;
                if (MODE == 4) {
                    if (r < ld && c < ld) og[r + (int64_t)c * ld] = val;
                    continue;
                }
                if (r < ld && c < ld && r >= c) {
                    og[r + (int64_t)c * ld] = val;
                    if (r > c) og[c + (int64_t)r * ld] = val;
                }
            }
        }
    }
    if (MODE == 0 || MODE == 5) {
        rmax = wave_max(rmax);
        if (lane == 0) {
            unsigned long long *slot = it.resid_bits + (int64_t)g * it.resid_stride + k;
            atomicMax(slot, (unsigned long long)__double_as_longlong(rmax));
        }
    }
}

}  // namespace

hipError_t launch_ns_f64(hipStream_t st, int mode, int ntiles, const TileDesc *tiles,
                         const GroupDesc *groups, const double *x, const double *b, double *out,
                         const IterState &it, int k, double tol, int max_iter, int polish, const double *aux)
{
    if (ntiles <= 0) return hipSuccess;
#define SMX_NS_LAUNCH(M)                                                                                    \
    hipLaunchKernelGGL(ns_f64_kernel<M>, dim3(ntiles), dim3(256), 0, st, tiles, groups, x, b, out, it, k, tol, \
                       max_iter, polish, aux)
    switch (mode) {
    case 0: SMX_NS_LAUNCH(0); break;
    case 1: SMX_NS_LAUNCH(1); break;
    case 2: SMX_NS_LAUNCH(2); break;
    case 3: SMX_NS_LAUNCH(3); break;
    case 4: SMX_NS_LAUNCH(4); break;
    case 5: SMX_NS_LAUNCH(5); break;
    case 6: SMX_NS_LAUNCH(6); break;
    default: return hipErrorInvalidValue;
    }
#undef SMX_NS_LAUNCH
    return hipGetLastError();
}

}  // namespace smx
