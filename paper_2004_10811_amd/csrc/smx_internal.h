// Internal declarations shared by the host side of libsmx and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace smx {

// Edge of the square output tile of the Newton-Schulz products, and the
// granularity to which every submatrix is padded.  Padding rows/columns hold
// the identity, which is a fixed point of the iteration (p(1) = 1), so the
// padded block never mixes with the true one.
constexpr int kTile = 128;
constexpr int kPad = 32;

// One submatrix (group) as the device sees it.
struct GroupDesc {
    int64_t off;        // element offset of the group's dense matrices in the work buffers
    int64_t map_off;    // offset of the m x m block map (int32 storage positions, -1 = not stored)
    int64_t rinfo_off;  // offset of the per-row table (npad entries)
    int32_t boff_off;   // offset of the m+1 block offsets inside the submatrix
    int32_t n;          // true dimension n_g
    int32_t npad;       // padded dimension = leading dimension (multiple of kPad)
    int32_t m;          // number of block rows |R(g)|
};

// Row table entry: x = local block index in R(g); y = (row inside block) | (block size << 16).
using RowInfo = int2;

// Output tile of a product: x = group, y = (tile row << 16) | tile column, tile row >= tile column.
using TileDesc = int2;

// Source of one stored block of D in the group matrices.
struct ScatterDesc {
    int32_t g;          // group owning the block column
    int32_t oi;         // row offset of block row I inside the submatrix
    int32_t oj;         // column offset of block column J inside the submatrix
    int32_t bij;        // b_I | (b_J << 16)
};

// Per-evaluation device state of the iteration.
struct IterState {
    unsigned long long *scale_bits;   // [ngroups] s_g = ||A_g||_inf as raw bits (atomic max)
    unsigned long long *resid_bits;   // [ngroups * resid_stride] max|X_k^2 - I| per step
    int32_t *done;                    // [ngroups] 1 once the group's result is fixed
    int32_t *kfinal;                  // [ngroups] step k whose X_k is the result
    int32_t *flags;                   // [ngroups] bit 0: not converged, bit 1: non-finite
    int32_t *ndone;                   // [1] number of finished groups
    int32_t resid_stride;             // max_iter + 2
};

// ---- launchers (stream-ordered, no synchronisation) -----------------------

hipError_t launch_gather(hipStream_t st, int nchunks, const int2 *chunks, const GroupDesc *groups,
                         const RowInfo *rinfo, const int32_t *bmap, const int32_t *boffs,
                         const int64_t *valoff, const double *kvals, double mu, double *x0,
                         unsigned long long *scale_bits);

// mode 0: T = a^2 X X, records max|T - I| for step k, writes W = 1.5 I - 0.5 T.
// mode 1: if the step-k residual meets the stopping rule the group is finished
//         at X_k; otherwise X_{k+1} = a X W.   a = 1/s_g at k = 0, else 1.
hipError_t launch_ns_f64(hipStream_t st, int mode, int ntiles, const TileDesc *tiles,
                         const GroupDesc *groups, const double *x, const double *b, double *out,
                         const IterState &it, int k, double tol, int max_iter);

hipError_t launch_scatter(hipStream_t st, int64_t nblocks, const ScatterDesc *sd,
                          const int64_t *valoff, const GroupDesc *groups, const double *x0,
                          const double *x1, const IterState &it, const double *kvals,
                          double *dvals, double *part_e, double *part_n);

hipError_t launch_reduce(hipStream_t st, int64_t n, const double *part_e, const double *part_n,
                         double *out2);

hipError_t launch_check_values(hipStream_t st, int64_t nblocks, const int64_t *valoff,
                               const int32_t *blk_rows, const int32_t *blk_cols,
                               const int64_t *mirror, const double *kvals, double *out2);

}  // namespace smx
