// Memory-bound kernels of the reverse (adjoint) pass through the frozen
// Newton-Schulz iteration: seed of the adjoint at the own columns, in-place
// symmetrisation, prescaling of X_0, and the transposed gather that sums the
// per-group adjoints Abar_g = Xbar_0 / s_g into dK in a fixed order.
#include "smx_internal.h"

#include <algorithm>

namespace smx {

namespace {

__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wave per stored block of an own column: the derivative of
// L = gE E + gN N + <gD, D> with respect to D_IJ is gE K_IJ + gN I [I = J] + gD_IJ,
// and D_IJ = (delta_IJ I - S_g[I, J]) / 2, so the seed of S_g there is -1/2 of it.
__global__ __launch_bounds__(256)
void adj_seed_kernel(int64_t nblocks, const ScatterDesc *__restrict__ sd, const int64_t *__restrict__ valoff,
                     const GroupDesc *__restrict__ groups, const double *__restrict__ kvals,
                     const double *__restrict__ gdv, double ge, double gn, double *__restrict__ xb)
{
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= nblocks) return;
    const ScatterDesc d = sd[p];
    const GroupDesc gd = groups[d.g];
    const int bi = d.bij & 0xffff, bj = d.bij >> 16;
    const bool diag = (d.oi == d.oj);
    const int64_t vo = valoff[p];
    for (int t = lane; t < bi * bj; t += 64) {
        const int rr = t % bi, cc = t / bi;
        double gdval = ge * kvals[vo + t];
        if (diag && rr == cc) gdval += gn;
        if (gdv) gdval += gdv[vo + t];
        xb[gd.off + (int64_t)(d.oi + rr) + (int64_t)(d.oj + cc) * gd.npad] = -0.5 * gdval;
    }
}

__global__ __launch_bounds__(256)
void symmetrize_kernel(const GroupDesc *__restrict__ groups, double *__restrict__ xb)
{
    const GroupDesc gd = groups[blockIdx.y];
    const int64_t tot = (int64_t)gd.npad * gd.npad;
    double *x = xb + gd.off;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t r = e % gd.npad, c = e / gd.npad;
        if (r <= c) continue;                 // each pair once, by its lower element
        const double v = 0.5 * (x[r + c * gd.npad] + x[c + r * gd.npad]);
        x[r + c * gd.npad] = v;
        x[c + r * gd.npad] = v;
    }
}

__global__ __launch_bounds__(256)
void scale_slab_kernel(const GroupDesc *__restrict__ groups, const unsigned long long *__restrict__ scale_bits,
                       double *__restrict__ x)
{
    const GroupDesc gd = groups[blockIdx.y];
    const int64_t tot = (int64_t)gd.npad * gd.npad;
    const double s = __longlong_as_double((long long)scale_bits[blockIdx.y]);
    const double a = s > 0.0 ? 1.0 / s : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t r = e % gd.npad, c = e / gd.npad;
        // the padded identity is not part of A / s and stays 1 (a fixed point)
        x[gd.off + e] = (r < gd.n && c < gd.n) ? a * x[gd.off + e] : x[gd.off + e];
    }
}

// One wave per stored block p of K: its contributions (group, row offset,
// column offset) are listed in cptr[p] .. cptr[p+1]-1 in ascending group order.
__global__ __launch_bounds__(256)
void gather_t_kernel(int64_t nblocks, const int64_t *__restrict__ cptr, const int4 *__restrict__ contrib,
                     const int64_t *__restrict__ valoff, const int32_t *__restrict__ brow,
                     const int32_t *__restrict__ bcol, const GroupDesc *__restrict__ groups,
                     const unsigned long long *__restrict__ scale_bits, const double *__restrict__ xb,
                     const double *__restrict__ dvals, double ge, double *__restrict__ dk)
{
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= nblocks) return;
    const int bi = brow[p], bj = bcol[p];
    const int64_t vo = valoff[p];
    for (int t = lane; t < bi * bj; t += 64) {
        const int rr = t % bi, cc = t / bi;
        double acc = ge * dvals[vo + t];                         // explicit term of E = sum D K
        for (int64_t q = cptr[p]; q < cptr[p + 1]; q++) {
            const int4 cq = contrib[q];                          // (g, oi, oj, -)
            const GroupDesc gd = groups[cq.x];
            const double s = __longlong_as_double((long long)scale_bits[cq.x]);
            const double a = s > 0.0 ? 1.0 / s : 0.0;
            acc += a * xb[gd.off + (int64_t)(cq.y + rr) + (int64_t)(cq.z + cc) * gd.npad];
        }
        dk[vo + t] = acc;
    }
}

// part[g] = -tr(Abar_g) = -(1/s_g) sum_{i < n_g} Xbar_0[i, i]  (A_g = K_sub - mu I).
__global__ __launch_bounds__(64)
void diag_part_kernel(const GroupDesc *__restrict__ groups, const unsigned long long *__restrict__ scale_bits,
                      const double *__restrict__ xb, double *__restrict__ part)
{
    const int g = blockIdx.x;
    const GroupDesc gd = groups[g];
    const double s = __longlong_as_double((long long)scale_bits[g]);
    const double a = s > 0.0 ? 1.0 / s : 0.0;
    double acc = 0.0;
    for (int i = threadIdx.x; i < gd.n; i += 64) acc += xb[gd.off + (int64_t)i * (gd.npad + 1)];
    acc = wave_sum(acc);
    if (threadIdx.x == 0) part[g] = -a * acc;
}

dim3 slab_grid(int ngroups, int max_npad)
{
    const int64_t tot = (int64_t)max_npad * max_npad;
    return dim3((unsigned)std::min<int64_t>((tot + 2047) / 2048, 4096), (unsigned)ngroups);
}

}  // namespace

hipError_t launch_adj_seed(hipStream_t st, int64_t nblocks, const ScatterDesc *sd, const int64_t *valoff,
                           const GroupDesc *groups, const double *kvals, const double *gd, double ge, double gn,
                           double *xb)
{
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(adj_seed_kernel, dim3((unsigned)((nblocks + 3) / 4)), dim3(256), 0, st, nblocks, sd, valoff,
                       groups, kvals, gd, ge, gn, xb);
    return hipGetLastError();
}

hipError_t launch_symmetrize(hipStream_t st, int ngroups, int max_npad, const GroupDesc *groups, double *xb)
{
    if (ngroups <= 0) return hipSuccess;
    hipLaunchKernelGGL(symmetrize_kernel, slab_grid(ngroups, max_npad), dim3(256), 0, st, groups, xb);
    return hipGetLastError();
}

hipError_t launch_scale_slab(hipStream_t st, int ngroups, int max_npad, const GroupDesc *groups,
                             const unsigned long long *scale_bits, double *x)
{
    if (ngroups <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_slab_kernel, slab_grid(ngroups, max_npad), dim3(256), 0, st, groups, scale_bits, x);
    return hipGetLastError();
}

hipError_t launch_gather_t(hipStream_t st, int64_t nblocks, const int64_t *cptr, const int4 *contrib,
                           const int64_t *valoff, const int32_t *brow, const int32_t *bcol,
                           const GroupDesc *groups, const unsigned long long *scale_bits, const double *xb,
                           const double *dvals, double ge, double *dk)
{
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_t_kernel, dim3((unsigned)((nblocks + 3) / 4)), dim3(256), 0, st, nblocks, cptr, contrib,
                       valoff, brow, bcol, groups, scale_bits, xb, dvals, ge, dk);
    return hipGetLastError();
}

hipError_t launch_diag_part(hipStream_t st, int ngroups, const GroupDesc *groups,
                            const unsigned long long *scale_bits, const double *xb, double *part)
{
    if (ngroups <= 0) return hipSuccess;
    hipLaunchKernelGGL(diag_part_kernel, dim3(ngroups), dim3(64), 0, st, groups, scale_bits, xb, part);
    return hipGetLastError();
}

}  // namespace smx
