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
    int64_t thin_off;   // element offset of the group's npad x m_own own-column buffers
    int32_t boff_off;   // offset of the m+1 block offsets inside the submatrix
    int32_t n;          // true dimension n_g
    int32_t npad;       // padded dimension = leading dimension (multiple of kPad)
    int32_t m;          // number of block rows |R(g)|
    int32_t own_off;    // offset of the group's own-column list (submatrix column indices)
    int32_t m_own;      // number of own columns (sum of the member block sizes)
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
    int32_t ocol;       // position of block column J's first column in the own-column list
    int32_t pad;
};

// Per-evaluation device state of the iteration.
struct IterState {
    unsigned long long *scale_bits;   // [ngroups] s_g = ||A_g||_inf as raw bits (atomic max)
    unsigned long long *resid_bits;   // [ngroups * resid_stride] max|X_k^2 - I| per step
    int32_t *done;                    // [ngroups] 1 once the group's result is fixed
    int32_t *kfinal;                  // [ngroups] step k whose X_k is the result
    int32_t *flags;                   // [ngroups] bit 0: not converged, bit 1: non-finite
    int32_t *ndone;                   // [1] number of finished groups
    const int32_t *kfix;              // [ngroups] frozen step counts (nullptr: stopping rule)
    int32_t kact;                     // >= 0: only groups with kact < kfix[g] take part (adjoint passes)
    double *tdiag;                    // [sum of n_pad] 1 - T_ii of the last square, row i of group g
                                      // at GroupDesc::rinfo_off + i (reduced-precision bulk)
    double *tau_hist;                 // [ngroups * resid_stride] Tr(I - X_k^2) per step
    int32_t resid_stride;             // steps 0..max_iter, then one slot per polish step
};

// Row r of A_g = K[R(g), R(g)] - mu I over the columns c < n_g (Sec. III-A
// step 1), block column by block column: emit(c, v) for every column, zero
// for unstored blocks and padding rows.  Returns sum_c |v| for true rows (the
// row's term of the Gershgorin bound ||A_g||_inf), 0 for padding rows.
template <class Emit>
__device__ inline double gather_row(const GroupDesc &gd, int r, const RowInfo *__restrict__ rinfo,
                                    const int32_t *__restrict__ bmap, const int32_t *__restrict__ boffs,
                                    const int64_t *__restrict__ valoff, const double *__restrict__ kvals,
                                    double mu, Emit &&emit)
{
    const bool real = r < gd.n;
    int lb = 0, rr = 0, br = 0;
    if (real) {
        const RowInfo ri = rinfo[gd.rinfo_off + r];
        lb = ri.x;
        rr = ri.y & 0xffff;
        br = ri.y >> 16;
    }
    const int32_t *map_row = bmap + gd.map_off + lb;     // + m * column block
    const int32_t *bo = boffs + gd.boff_off;
    double rowsum = 0.0;
    for (int cb = 0; cb < gd.m; cb++) {
        const int c0 = bo[cb];
        const int bc = bo[cb + 1] - c0;
        const int32_t p = real ? map_row[(int64_t)gd.m * cb] : -1;
        // Every lane loads (an unstored block or a padding row reads K's first
        // value and uses zero), eight columns of the block row at a time, so
        // that the loads are in flight together rather than one by one.
        const double *src = kvals + ((p >= 0) ? valoff[p] + rr : 0);
        const int64_t stride = (p >= 0) ? br : 0;
        for (int cc0 = 0; cc0 < bc; cc0 += 8) {
            double vb[8];
#pragma unroll
            for (int u = 0; u < 8; u++) vb[u] = src[(int64_t)min(cc0 + u, bc - 1) * stride];
            // an empty statement that takes all eight values keeps the compiler
            // from sinking each load to its (conditional) use
#pragma unroll
            for (int u = 0; u < 8; u++) asm volatile("" ::"v"(vb[u]));
#pragma unroll
            for (int u = 0; u < 8; u++) {
                if (cc0 + u >= bc) break;
                const int c = c0 + cc0 + u;
                double v = (p >= 0) ? vb[u] : 0.0;
                if (r == c) v -= mu;
                rowsum += fabs(v);
                emit(c, v);
            }
        }
    }
    return real ? rowsum : 0.0;
}

// ---- launchers (stream-ordered, no synchronisation) -----------------------

hipError_t launch_gather(hipStream_t st, int nchunks, const int2 *chunks, const GroupDesc *groups,
                         const RowInfo *rinfo, const int32_t *bmap, const int32_t *boffs,
                         const int64_t *valoff, const double *kvals, double mu, double *x0,
                         unsigned long long *scale_bits);

// mode 0: T = a^2 X X, records max|T - I| for step k, writes W = 1.5 I - 0.5 T.
// mode 1: if the step-k residual meets the stopping rule the group is finished
//         at X_k; otherwise X_{k+1} = a X W.   a = 1/s_g at k = 0, else 1.
// mode 2: tangent of the step, Xd_{k+1} = 3 (W - I) Xd_k = 3 Xd_k W - 3 Xd_k, for groups
//         still iterating after step k (x = Xd_k, b = W).
// polish != 0: unconditional step on every group (a = 1, no skipping, no
// stopping); the square's residual goes to slot k of the residual history.
// With it.kfix set, a group stops exactly at step kfix[g] (frozen iteration).
// mode 3 (adjoint step, lower tiles): acc = X Y; out = Xb is updated in place to
//         -1.5 Xb + Z + Z^T - 0.5 acc with Z = aux (= Xb W).
// mode 4 (full tiles, plain product): out = x b with x symmetric (read by columns)
//         and b general; every tile of the group is listed.
// mode 5 (Pade square): T = a^2 X X stored, residual as mode 0.
// mode 6 (Pade combine): out = (15 I - 10 x + 3 x x) / 8 with x = b = T.
hipError_t launch_ns_f64(hipStream_t st, int mode, int ntiles, const TileDesc *tiles,
                         const GroupDesc *groups, const double *x, const double *b, double *out,
                         const IterState &it, int k, double tol, int max_iter, int polish,
                         const double *aux = nullptr);

// ---- adjoint helpers ------------------------------------------------------
// xb (zeroed) at the own-column stored positions: -1/2 (gE K + gN I_diag + gD).
hipError_t launch_adj_seed(hipStream_t st, int64_t nblocks, const ScatterDesc *sd, const int64_t *valoff,
                           const GroupDesc *groups, const double *kvals, const double *gd, double ge, double gn,
                           double *xb);
// in place: xb = (xb + xb^T) / 2 on each group's n_pad x n_pad slab.
hipError_t launch_symmetrize(hipStream_t st, int ngroups, int max_npad, const GroupDesc *groups, double *xb);
// in place: x = a x with a = 1/s_g (the Gershgorin prescaling of X_0).
hipError_t launch_scale_slab(hipStream_t st, int ngroups, int max_npad, const GroupDesc *groups,
                             const unsigned long long *scale_bits, double *x);
// dK[p] = ge D[p] + sum over the contributions (g, oi, oj) of block p of Xb_g[oi.., oj..] / s_g,
// in list order; part[g] = -sum_i Xb_g[i, i] / s_g (the mu derivative).
hipError_t launch_gather_t(hipStream_t st, int64_t nblocks, const int64_t *cptr, const int4 *contrib,
                           const int64_t *valoff, const int32_t *brow, const int32_t *bcol,
                           const GroupDesc *groups, const unsigned long long *scale_bits, const double *xb,
                           const double *dvals, double ge, double *dk);
hipError_t launch_diag_part(hipStream_t st, int ngroups, const GroupDesc *groups,
                            const unsigned long long *scale_bits, const double *xb, double *part);

// Word storage of the reduced-precision iterates (nw 16-bit words per value):
// group g's words start at element nw * off of an operand buffer; inside them
// column c holds its 32-row blocks one after another, and a block holds word 0
// of its 32 rows, then word 1, ...  So one K step of 32 of a product reads the
// nw words of a column as one contiguous nw * 64-B run (a whole 128-B line for
// two FP16 words).  Position of word 0 of element (r, c); word w is 32 w further.
__host__ __device__ inline int64_t word_pos(int nw, int ld, int r, int c)
{
    return (int64_t)c * ld * nw + (int64_t)(r >> 5) * (32 * nw) + (r & 31);
}

// Persistent form of the 128 x 128 word products (Newton-Schulz square and
// update; 2-word FP16 and 1-word BF16): nwg workgroups take the tiles from
// eight per-XCD lists tiles_x[xbeg[x] .. xbeg[x + 1]) through the counters
// cnt[0 .. 8), which must be zero at launch.
hipError_t launch_ns_words_persistent(hipStream_t st, int fmt, int nw, int mode, int nwg, const TileDesc *tiles_x,
                                      const int32_t *xbeg, int32_t *cnt, const GroupDesc *groups,
                                      const unsigned short *x, const unsigned short *b, unsigned short *out,
                                      const IterState &it, int k, double switch_tol, int kmax);
// Workgroups of the persistent word products one CU holds at once.
int words_persistent_blocks_per_cu(int fmt, int nw);

// Reduced-precision bulk products (fmt 0 = FP16, 1 = BF16; nw words per value;
// fmt 2 = one FP32 value per element, column-major like the FP64 slabs).
// mode 0: Newton-Schulz square (W = 1.5 I - 0.5 X^2, residual, 1 - T_ii);
// mode 1: update X_{k+1} = X W after the bulk stopping rule;
// mode 2: Pade square (T = X^2 stored, residual, 1 - T_ii);
// mode 3: Pade combine W = (15 I - 10 T + 3 T T) / 8 (x = b = T).
// variant: operand stream of the word products (0: global_load_lds into LDS one
// K step at a time; 1: next K step prefetched into registers); results are
// bitwise the same.
hipError_t launch_ns_words(hipStream_t st, int fmt, int nw, int mode, int variant, int ntiles, const TileDesc *tiles,
                           const GroupDesc *groups, const unsigned short *x, const unsigned short *b,
                           unsigned short *out, const IterState &it, int k, double switch_tol, int kmax);
// The same products on 256 x 256 output tiles (tiles list (group, tile row
// << 16 | tile column) in units of 256; fmt 0 / 1 with nw = 1 or 2 only).
// Results are bitwise those of the 128 x 128 tiles.
constexpr int kTile2 = 256;
// guard region of the debug checks (doubles after the arena, the polish pool and D)
constexpr size_t kGuardElems = 8192;
hipError_t launch_ns_words256(hipStream_t st, int fmt, int nw, int mode, int ntiles, const TileDesc *tiles,
                              const GroupDesc *groups, const unsigned short *x, const unsigned short *b,
                              unsigned short *out, const IterState &it, int k, double switch_tol, int kmax);
// Group-walking launchers take the first group g0 and the count ngroups (a wave).
// Gershgorin bounds only (atomic max of the row sums into scale_bits), no
// writes of A_g; then X_0 = A_g / s_g gathered straight into the word storage
// (fmt 0 / 1 with nw words, fmt 2 FP32 values) with the bounds in scale_bits.
hipError_t launch_gather_bound(hipStream_t st, int nchunks, const int2 *chunks, const GroupDesc *groups,
                               const RowInfo *rinfo, const int32_t *bmap, const int32_t *boffs,
                               const int64_t *valoff, const double *kvals, double mu,
                               unsigned long long *scale_bits);
hipError_t launch_gather_words(hipStream_t st, int fmt, int nw, int nchunks, const int2 *chunks,
                               const GroupDesc *groups, const RowInfo *rinfo, const int32_t *bmap,
                               const int32_t *boffs, const int64_t *valoff, const double *kvals, double mu,
                               const unsigned long long *scale_bits, unsigned short *dst);
hipError_t launch_from_words(hipStream_t st, int fmt, int nw, int g0, int ngroups, int max_npad, const GroupDesc *groups,
                             const unsigned short *x0, const unsigned short *x1, const int32_t *kfinal, double *dst);

// Last polish step restricted to the own columns (FP64, vector ALU):
//   O = P[:, own];  Y = P O (residual of P^2 on the own columns -> slot);  F = 1.5 O - 0.5 P Y.
// Where the own-column polish reads the bulk result X of each group: an FP64
// slab (fmt < 0), or the storage of the reduced-precision bulk (fmt 0 FP16 /
// 1 BF16 words, nw of them; fmt 2 one FP32 value) in the buffer of the group's
// final step: w1 when kfinal[g] is odd, else w0.
struct XSource {
    const double *f64;
    const unsigned short *w0, *w1;
    const int32_t *kfinal;
    int fmt, nw;
};

// Own-column polish: out = X[:, own]; y = X z (mode 0) or 1.5 o - 0.5 X z (mode 1);
// c = 1.5 a - 0.5 c; max |b - E| into the residual slot.
hipError_t launch_own_gather(hipStream_t st, int g0, int ngroups, int max_npad, const GroupDesc *groups,
                             const int32_t *own_list, const XSource &xs, double *out);
hipError_t launch_thin_mul(hipStream_t st, int mode, int g0, int ngroups, int max_npad, int max_own,
                           const GroupDesc *groups, const XSource &xs, const double *z, const double *o, double *y);
hipError_t launch_thin_combine(hipStream_t st, int g0, int ngroups, int max_npad, int max_own,
                               const GroupDesc *groups, const double *a, double *c);
hipError_t launch_thin_resid(hipStream_t st, int g0, int ngroups, int max_npad, int max_own,
                             const GroupDesc *groups, const int32_t *own_list, const double *b,
                             const IterState &it, int slot);

// from_thin = 0: S_g = a X_kfinal (full matrices x0 / x1 by step parity);
// from_thin = 1: S_g own columns from the npad x m_own buffer x0.
// plist (nullable): the stored-block positions to scatter (one wave's own columns).
hipError_t launch_scatter(hipStream_t st, int64_t nblocks, const int64_t *plist, const ScatterDesc *sd,
                          const int64_t *valoff, const GroupDesc *groups, const double *x0,
                          const double *x1, const IterState &it, const double *kvals,
                          double *dvals, double *part_e, double *part_n, int from_thin);

// flags[g] |= 1 unless 3 r^2 / 4 <= tol for the polish residual r in `slot`
// (|= 2 if r is not finite), for the groups g0 .. g0 + ngroups - 1.
hipError_t launch_polish_flags(hipStream_t st, int g0, int ngroups, const IterState &it, int slot, double tol);

hipError_t launch_reduce(hipStream_t st, int64_t n, const double *part_e, const double *part_n,
                         double *out2);
// out2[0] / out2[1] = number of groups with flag bit 0 / bit 1 set.
hipError_t launch_count_flags(hipStream_t st, int ngroups, const int32_t *flags, int32_t *out2);
// dst[0 .. n_dst) = 0, then dst[idx[q]] = src[q] for q < n_src (idx checked on the host).
hipError_t launch_expand_values(hipStream_t st, int64_t n_src, const int64_t *idx, const double *src, int64_t n_dst,
                                double *dst);

// Xd_0 = -a I on the true n_g x n_g block (a = 1/s_g), zero elsewhere: the mu tangent
// of X_0 = (K_sub - mu I) / s_g with s_g frozen.
hipError_t launch_tangent_init(hipStream_t st, int g0, int ngroups, int max_npad, const GroupDesc *groups,
                               const unsigned long long *scale_bits, double *xd);

// part[g] = sum over the own columns c of Xd_{kfinal}[c, c] (Xd in xd0 / xd1 by step parity).
hipError_t launch_own_trace(hipStream_t st, int g0, int ngroups, const GroupDesc *groups, const int32_t *own_list,
                            const double *xd0, const double *xd1, const int32_t *kfinal, double *part);

hipError_t launch_check_values(hipStream_t st, int64_t nblocks, const int64_t *valoff,
                               const int32_t *blk_rows, const int32_t *blk_cols,
                               const int64_t *mirror, const double *kvals, double *out2);

// ---- batched symmetric eigensolver (finite temperature, Algorithm 1) --------
// Largest submatrix dimension of the eigensolver path (its workgroups keep
// two vectors of this length in LDS and 64-row column strips in registers).
constexpr int kEigMaxN = 3072;

// Per-row arrays of the eigensolver, indexed like the row tables
// (GroupDesc::rinfo_off + i): T's diagonal d and off-diagonal e (e_i couples
// rows i and i + 1; 0 where T splits), the reflector scalars tau, the
// eigenvalues of A_g - mu0 I (ascending within each unreduced block of T)
// and of A_g + 0 (lam_abs = lam + mu0), Algorithm 1's weights
// w_l = sum_{c in own} Q_cl^2, and each row's unreduced block [bs, be).
struct EigVecs {
    double *d, *e, *tau, *lam, *lam_abs, *w;
    int32_t *bs, *be;
};

// Householder reduction of each group's slab (A_g - mu0 I, column-major) to
// tridiagonal form, reflectors left below the subdiagonal; then the split.
// wpanel: a second slab (n_pad x 16 of each group's place used as panel work).
hipError_t launch_eig_tridiag(hipStream_t st, int g0, int ngroups, const GroupDesc *groups, double *a,
                              double *wpanel, const EigVecs &ev);
// Eigenvalues (bisection) and eigenvectors (twisted factorisations, then
// Gram-Schmidt inside tight clusters) of T: s[i * n_pad + l] = component i of
// eigenvector l; scratch: one more slab.
hipError_t launch_eig_values_vectors(hipStream_t st, int g0, int ngroups, int max_npad, const GroupDesc *groups,
                                     const EigVecs &ev, double *s, double *scratch);
// y = the own-column selector (n_pad x m_own blocks at thin_off).
hipError_t launch_eig_own_select(hipStream_t st, int g0, int ngroups, int max_npad, int max_own,
                                 const GroupDesc *groups, const int32_t *own_list, double *y);
// y <- Q^T y (forward != 0) or Q y, with Q from the reflectors in a.
hipError_t launch_eig_reflect(hipStream_t st, int forward, int g0, int ngroups, int max_own, const GroupDesc *groups,
                              const double *a, const EigVecs &ev, double *y);
// mode 0: out = S^T in, with weights and lam_abs = lam + mu0;
// mode 1: out = S diag(g(lam - dmu)) in, g = tanh(x / 2kT) (signum at T = 0).
hipError_t launch_eig_thin(hipStream_t st, int mode, int g0, int ngroups, int max_npad, int max_own,
                           const GroupDesc *groups, const EigVecs &ev, const double *s, const double *in, double *out,
                           double mu0, double dmu, double kT, const unsigned long long *scale_bits);
// out[m] = N(mus[m]) = sum_g sum_l w_gl (1 - g(lam_abs_gl - mus[m])) / 2 over all groups
// (part: ngroups * nmu scratch).
hipError_t launch_n_of_mu(hipStream_t st, int ngroups, const GroupDesc *groups, const EigVecs &ev, const double *mus,
                          int nmu, double kT, const unsigned long long *scale_bits, double *part, double *out);

}  // namespace smx
