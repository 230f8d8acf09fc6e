// Batched symmetric eigensolver of the submatrices (Sec. IV-F: the paper's
// production path diagonalises every submatrix, A_g = Q Lambda Q^T, and takes
// D_g = Q f(Lambda) Q^T with f the Fermi function at finite temperature, or
// the signum of Eq. signev at T = 0; Algorithm 1 of Sec. IV-G then finds mu
// from the stored decompositions without solving again).
//
// Four stages, each one launch over all groups of a wave:
//   1. Householder reduction A_g = Q T Q^T to symmetric tridiagonal form, one
//      512-lane workgroup per group (the reflectors stay in the slab, below
//      the subdiagonal, as in LAPACK's sytrd), then splitting of T where an
//      off-diagonal entry is negligible;
//   2. eigenvalues of T by bisection on Sturm counts, one lane per eigenvalue
//      (each unreduced block on its own);
//   3. eigenvectors of T by twisted factorisations, one lane per eigenvalue;
//      clusters of nearly equal eigenvalues by inverse iteration with
//      orthogonalisation;
//   4. the group's own columns only (that is all D needs): Y = Q^T E (E the
//      own-column selector; reflectors applied to a thin block), C = S^T Y
//      (S the eigenvectors of T; C's rows give Algorithm 1's weights
//      w_l = sum_c C_lc^2 = sum_{c in own} Q_cl^2), Z = S diag(g) C and
//      G = Q Z = Q diag(g) Q^T E with g = 1 - 2 f = tanh(lambda / 2kT) (signum
//      at T = 0, 0 for |lambda| <= 1e-14 ||A_g||_inf).  D's own columns are
//      (E - G) / 2, which the scatter of the sign path forms.
#include "smx_internal.h"

namespace smx {

namespace {

// lanes of the reduction workgroups: two waves per SIMD, so that the
// compiler may hold 256 registers and keep eight loads per lane in flight in
// the row dots of A_s v (at 1024 lanes and 128 registers it issued them one
// at a time)
constexpr int kEigBlock = 512;
constexpr int kReflBlock = 512;     // lanes of the reflector workgroups (two waves per SIMD: 256 registers)

// Sum over a kEigBlock-lane workgroup in a fixed order (lanes by a xor tree, lane
// 0's value per wave, then the waves in order); every lane gets the same bits.
__device__ inline double block_sum(double v, double *red)
{
    const int tid = threadIdx.x;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kEigBlock / 64; w++) s += red[w];
    __syncthreads();
    return s;
}

__device__ inline double wave_sum0(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return __shfl(v, 0, 64);
}

// ---- 1. Householder tridiagonalisation --------------------------------------
// Step k (0 <= k < n - 2): x = A[k+1:, k]; the reflector H_k = I - tau v v^T
// (v_0 = 1) maps x to beta e_1 (beta = -sign(x_0) ||x||, tau = (beta - x_0) /
// beta); with p = tau A22 v and w = p - (tau / 2)(p^T v) v the trailing block
// becomes A22 - v w^T - w v^T.  d_k = A_kk, e_k = beta; v is stored in
// A[k+1:, k].  A is column-major with leading dimension n_pad (full storage).
//
// Blocked as in LAPACK's sytrd: the steps of a panel of kPanel columns leave
// the trailing block as it was at the panel's start (A_s) and keep their
// vectors V (in A's columns) and W (n_pad x kPanel, in the second slab); a
// step first brings its own column up to date, A[:, k] -= V W[k, :]^T + W
// V[k, :]^T, and forms p = tau (A_s v - V (W^T v) - W (V^T v)); after the
// panel one pass applies A22 -= V W^T + W V^T to the trailing block.  Each
// step then reads the trailing block once instead of reading it twice and
// writing it once.
// sum over columns jj in [jb, je) of row[jj * ld] * v[jj], with eight partial
// sums in flight (eight independent loads per lane) added in a fixed order
__device__ inline double row_dot(const double *__restrict__ row, int ld, const double *v, int jb, int je)
{
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int jj = jb;
    for (; jj + 7 < je; jj += 8) {
#pragma unroll
        for (int u = 0; u < 8; u++) a[u] += row[(int64_t)(jj + u) * ld] * v[jj + u];
    }
    for (; jj < je; jj++) a[0] += row[(int64_t)jj * ld] * v[jj];
    return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

constexpr int kPanel = 16;
constexpr int kTrailCols = 64;      // columns of V and W rows staged per trailing-update pass

__global__ __launch_bounds__(kEigBlock)
void tridiag_kernel(const GroupDesc *__restrict__ groups, int g0, double *__restrict__ abase,
                    double *__restrict__ wbase, EigVecs ev)
{
    __shared__ double vs[kEigMaxN];
    __shared__ double ws[kEigMaxN];
    __shared__ double red[kEigBlock / 64];
    __shared__ double rowk[2 * kPanel];               // V[k, t], W[k, t] of the panel's earlier steps
    __shared__ double dots[2 * kPanel];               // W[:, t]^T v, V[:, t]^T v
    __shared__ double vwc[kTrailCols][2 * kPanel];    // V[c, t], W[c, t] of a run of trailing columns
    __shared__ double psum[kEigBlock];                // column-part sums of A_s v
    const int g = g0 + blockIdx.x;
    const GroupDesc gd = groups[g];
    const int n = gd.n, ld = gd.npad, tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    double *A = abase + gd.off;
    double *W = wbase + gd.off;                       // W[:, t] at W + t * ld (kPanel <= 32 <= n_pad)
    double *d = ev.d + gd.rinfo_off, *e = ev.e + gd.rinfo_off, *tau = ev.tau + gd.rinfo_off;
    for (int kp = 0; kp + 2 < n; kp += kPanel) {
        const int nb = min(kPanel, n - 2 - kp);
        const double *V = A + (int64_t)kp * ld;       // V[:, t] = A[:, kp + t] below its subdiagonal
        bool any = false;                             // a reflector of the panel is not the identity
        for (int j = 0; j < nb; j++) {
            const int k = kp + j;
            double *col = A + (int64_t)k * ld;
            // column k (rows k ..) up to date with the panel's steps 0 .. j - 1
            if (tid < j) {
                rowk[tid] = V[k + (int64_t)tid * ld];
                rowk[kPanel + tid] = W[k + (int64_t)tid * ld];
            }
            __syncthreads();
            if (j > 0)
                for (int i = k + tid; i < n; i += kEigBlock) {
                    double s = col[i];
                    for (int q = 0; q < j; q++)
                        s -= V[i + (int64_t)q * ld] * rowk[kPanel + q] + W[i + (int64_t)q * ld] * rowk[q];
                    col[i] = s;
                }
            __syncthreads();
            const double x0 = col[k + 1];             // read by every lane before the barrier in
            double part = 0.0;                        // block_sum; lane 0 overwrites it with v_0 below
            for (int i = k + 2 + tid; i < n; i += kEigBlock) part += col[i] * col[i];
            const double sigma = block_sum(part, red);
            double beta = x0, tk = 0.0, sc = 0.0;
            if (sigma > 0.0) {
                const double nrm = sqrt(x0 * x0 + sigma);
                beta = x0 >= 0.0 ? -nrm : nrm;
                tk = (beta - x0) / beta;
                sc = 1.0 / (x0 - beta);
            }
            for (int i = k + 1 + tid; i < n; i += kEigBlock) {
                const double vi = (i == k + 1) ? 1.0 : col[i] * sc;
                vs[i] = vi;
                col[i] = vi;
            }
            if (tid == 0) {
                d[k] = col[k];
                e[k] = beta;
                tau[k] = tk;
            }
            __syncthreads();
            double *wj = W + (int64_t)j * ld;
            any = any || tk != 0.0;                   // the same in every lane
            if (tk != 0.0) {
                // W[:, q]^T v and V[:, q]^T v over rows k + 1 .., one wave per product
                for (int q = wave; q < 2 * j; q += kEigBlock / 64) {
                    const double *src = q < j ? W + (int64_t)q * ld : V + (int64_t)(q - j) * ld;
                    double s = 0.0;
                    for (int i = k + 1 + lane; i < n; i += 64) s += src[i] * vs[i];
                    s = wave_sum0(s);
                    if (lane == 0) dots[q] = s;
                }
                __syncthreads();
                // p = tau (A_s v - V (W^T v) - W (V^T v)).  A_s v: the lanes of a
                // row slot read consecutive rows of a column (coalesced); while the
                // trailing block has at most kEigBlock rows, the columns are split into
                // kEigBlock / (rows rounded up to 64) parts so every lane streams,
                // and the parts' sums are added in order
                const int R = n - k - 1;
                if (R <= kEigBlock) {
                    const int RS = (R + 63) & ~63, P = kEigBlock / RS;
                    const int sl = tid % RS, part = tid / RS;
                    if (part < P) {
                        double acc = 0.0;
                        if (sl < R) {
                            const int i = k + 1 + sl, cl = (R + P - 1) / P;
                            const int jb = k + 1 + part * cl, je = min(n, jb + cl);
                            acc = row_dot(A + i, ld, vs, jb, je);
                        }
                        psum[part * RS + sl] = acc;
                    }
                    __syncthreads();
                    for (int sl2 = tid; sl2 < R; sl2 += kEigBlock) {
                        double s = 0.0;
                        for (int pp = 0; pp < P; pp++) s += psum[pp * RS + sl2];
                        const int i = k + 1 + sl2;
                        for (int q = 0; q < j; q++)
                            s -= V[i + (int64_t)q * ld] * dots[q] + W[i + (int64_t)q * ld] * dots[j + q];
                        ws[i] = tk * s;
                    }
                } else {
                    for (int i = k + 1 + tid; i < n; i += kEigBlock) {
                        double s = row_dot(A + i, ld, vs, k + 1, n);
                        for (int q = 0; q < j; q++)
                            s -= V[i + (int64_t)q * ld] * dots[q] + W[i + (int64_t)q * ld] * dots[j + q];
                        ws[i] = tk * s;
                    }
                }
                __syncthreads();
                double pv = 0.0;
                for (int i = k + 1 + tid; i < n; i += kEigBlock) pv += ws[i] * vs[i];
                const double kk = -0.5 * tk * block_sum(pv, red);
                for (int i = k + 1 + tid; i < n; i += kEigBlock) wj[i] = ws[i] + kk * vs[i];
            } else {
                for (int i = k + 1 + tid; i < n; i += kEigBlock) wj[i] = 0.0;
            }
            __syncthreads();
        }
        // trailing block (rows and columns from k1 on): A -= V W^T + W V^T over the panel
        const int k1 = kp + nb;
        for (int c0 = k1; any && c0 < n; c0 += kTrailCols) {
            const int ncol = min(kTrailCols, n - c0);
            __syncthreads();
            for (int u = tid; u < kTrailCols * 2 * kPanel; u += kEigBlock) {
                const int cl = u / (2 * kPanel), q = u % (2 * kPanel);
                const int qq = q % kPanel;
                double v = 0.0;
                if (cl < ncol && qq < nb) v = (q < kPanel ? V : W)[c0 + cl + (int64_t)qq * ld];
                vwc[cl][q] = v;
            }
            __syncthreads();
            for (int r = k1 + tid; r < n; r += kEigBlock) {
                double vr[kPanel], wr[kPanel];
#pragma unroll
                for (int q = 0; q < kPanel; q++) {
                    vr[q] = q < nb ? V[r + (int64_t)q * ld] : 0.0;
                    wr[q] = q < nb ? W[r + (int64_t)q * ld] : 0.0;
                }
                // Eight columns' entries of the row at a time (the row is this
                // lane's alone, and V's columns lie left of k1); the next eight
                // are loaded, unconditionally (columns past the chunk read its last
                // one), before this batch is updated and stored, into two
                // register sets in turn, so no load waits behind the stores.
                auto load8 = [&](int cb, double (&dst)[8]) {
#pragma unroll
                    for (int u = 0; u < 8; u++) dst[u] = A[r + (int64_t)(c0 + min(cb + u, ncol - 1)) * ld];
                };
                auto update8 = [&](int cb, const double (&src)[8]) {
#pragma unroll
                    for (int u = 0; u < 8; u++) {
                        if (cb + u >= ncol) break;
                        const int cl = cb + u;
                        double s = src[u];
#pragma unroll
                        for (int q = 0; q < kPanel; q++) s -= vr[q] * vwc[cl][kPanel + q] + wr[q] * vwc[cl][q];
                        A[r + (int64_t)(c0 + cl) * ld] = s;
                    }
                };
                double ba[8], bb[8];
                load8(0, ba);
                for (int cb = 0; cb < ncol; cb += 16) {
                    load8(cb + 8, bb);
                    update8(cb, ba);
                    if (cb + 8 >= ncol) break;
                    load8(cb + 16, ba);
                    update8(cb + 8, bb);
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (n >= 2) {
            d[n - 2] = A[(n - 2) + (int64_t)(n - 2) * ld];
            e[n - 2] = A[(n - 1) + (int64_t)(n - 2) * ld];
            tau[n - 2] = 0.0;
            d[n - 1] = A[(n - 1) + (int64_t)(n - 1) * ld];
        } else {
            d[0] = A[0];
        }
        e[n - 1] = 0.0;
        if (n >= 1) tau[n - 1] = 0.0;
    }
}

// Split T into unreduced blocks: e_i is set to 0 where |e_i| <= 2u ||T||_inf
// (u the FP64 unit roundoff; a change of T of the size of the reduction's own
// rounding) or |e_i| <= u (|d_i| + |d_{i+1}|); bs[i] / be[i] are the first row
// and one past the last row of the block holding row i.  One lane per group.
__global__ void split_kernel(const GroupDesc *__restrict__ groups, int g0, int ng, EigVecs ev)
{
    const int q = blockIdx.x * 64 + threadIdx.x;
    if (q >= ng) return;
    const GroupDesc gd = groups[g0 + q];
    const int n = gd.n;
    double *d = ev.d + gd.rinfo_off, *e = ev.e + gd.rinfo_off;
    int32_t *bs = ev.bs + gd.rinfo_off, *be = ev.be + gd.rinfo_off;
    double tn = 0.0;
    for (int i = 0; i < n; i++)
        tn = fmax(tn, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0));
    int s = 0;
    for (int i = 0; i < n; i++) {
        bool end = (i == n - 1);
        if (!end && (fabs(e[i]) <= 2.220446049250313e-16 * tn ||
                     fabs(e[i]) <= 1.1102230246251565e-16 * (fabs(d[i]) + fabs(d[i + 1])))) {
            e[i] = 0.0;
            end = true;
        }
        if (end) {
            for (int r = s; r < i + 1; r++) {
                bs[r] = s;
                be[r] = i + 1;
            }
            s = i + 1;
        }
    }
}

// Number of eigenvalues of the block T[s:t, s:t] below x (Sylvester inertia of
// T - x I from its LDL^T pivots); pivots smaller than pivmin are replaced by
// -pivmin.  e2[i] = e[i]^2 (d and e2 staged in LDS by the caller).
__device__ inline int sturm_count(const double *d, const double *e2, int s, int t, double x, double pivmin)
{
    double q = d[s] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0;
    for (int i = s + 1; i < t; i++) {
        q = (d[i] - x) - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
    }
    return cnt;
}

// ---- 2. eigenvalues by bisection --------------------------------------------
// Lane l of group g finds the (l - s)-th smallest eigenvalue of its block
// [s, t) (ascending within each block), inside the block's Gershgorin
// interval, to the width of a few units in the last place.  The workgroup
// first stages d and e^2 of its group in LDS: every Sturm count then reads
// them there (the lanes of a wave mostly at the same index: broadcasts)
// instead of waiting on a global load per recurrence step.
__global__ __launch_bounds__(256)
void bisect_kernel(const GroupDesc *__restrict__ groups, int g0, EigVecs ev)
{
    __shared__ double ds[kEigMaxN], e2s[kEigMaxN];
    const int g = g0 + blockIdx.y;
    const GroupDesc gd = groups[g];
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (blockIdx.x * 256 >= gd.n) return;             // whole workgroup beyond this group
    const double *d = ev.d + gd.rinfo_off, *e = ev.e + gd.rinfo_off;
    for (int i = threadIdx.x; i < gd.n; i += 256) {
        ds[i] = d[i];
        e2s[i] = e[i] * e[i];
    }
    __syncthreads();
    if (l >= gd.n) return;
    const int s = ev.bs[gd.rinfo_off + l], t = ev.be[gd.rinfo_off + l], m = l - s;
    double lo = 1.7976931348623157e308, hi = -1.7976931348623157e308, tn = 0.0, emax = 0.0;
    for (int i = s; i < t; i++) {
        const double r = (i > s ? fabs(e[i - 1]) : 0.0) + (i + 1 < t ? fabs(e[i]) : 0.0);
        lo = fmin(lo, d[i] - r);
        hi = fmax(hi, d[i] + r);
        tn = fmax(tn, fabs(d[i]) + r);
        if (i + 1 < t) emax = fmax(emax, fabs(e[i]));
    }
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax * emax) * 1e10;
    const double pad = 4.440892098500626e-16 * fmax(tn, 1e-300) + pivmin;
    lo -= pad;
    hi += pad;
    // count(lo) <= m < count(hi)
    for (int it = 0; it < 400; it++) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (hi - lo <= 4.440892098500626e-16 * fmax(fabs(lo), fabs(hi)) + 2.220446049250313e-16 * tn + pivmin) break;
        if (sturm_count(ds, e2s, s, t, mid, pivmin) > m) hi = mid;
        else lo = mid;
    }
    ev.lam[gd.rinfo_off + l] = 0.5 * (lo + hi);
}

// ---- 3. eigenvectors by twisted factorisations ------------------------------
// For lambda of block [s, t): the stationary factorisation T - lambda I =
// L+ D+ L+^T from the top (D+_s = d_s - lambda, L+_i = e_i / D+_i,
// D+_{i+1} = d_{i+1} - lambda - L+_i e_i) and the progressive one from the
// bottom (D-_{t-1} = d_{t-1} - lambda, U-_i = e_i / D-_{i+1},
// D-_i = d_i - lambda - U-_i e_i) meet at the twist r minimising |gamma_r|,
// gamma_r = D+_r + D-_r - (d_r - lambda); the eigenvector then follows from
// z_r = 1, z_i = -L+_i z_{i+1} (i < r), z_{i+1} = -U-_i z_i (i >= r).
// S[i * n_pad + l] holds component i of eigenvector l (U-_i is parked there
// at row i + 1 until z overwrites it); lbuf holds D- and then L+.
__global__ __launch_bounds__(256)
void tvec_kernel(const GroupDesc *__restrict__ groups, int g0, EigVecs ev, double *__restrict__ sbase,
                 double *__restrict__ lbase)
{
    const int g = g0 + blockIdx.y;
    const GroupDesc gd = groups[g];
    const int l = blockIdx.x * 256 + threadIdx.x;
    const int ld = gd.npad;
    if (l >= ld) return;
    double *S = sbase + gd.off;
    double *Lb = lbase + gd.off;
    if (l >= gd.n) {                       // padding: the identity's columns
        for (int i = 0; i < ld; i++) S[(int64_t)i * ld + l] = (i == l) ? 1.0 : 0.0;
        return;
    }
    const double *d = ev.d + gd.rinfo_off, *e = ev.e + gd.rinfo_off;
    const int s = ev.bs[gd.rinfo_off + l], t = ev.be[gd.rinfo_off + l];
    const double lam = ev.lam[gd.rinfo_off + l];
    double emax = 0.0;
    for (int i = s; i + 1 < t; i++) emax = fmax(emax, fabs(e[i]));
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax * emax) * 1e10;
    auto guard = [&](double q) { return fabs(q) < pivmin ? (q < 0.0 ? -pivmin : pivmin) : q; };
    for (int i = 0; i < s; i++) S[(int64_t)i * ld + l] = 0.0;
    for (int i = t; i < ld; i++) S[(int64_t)i * ld + l] = 0.0;
    if (t - s == 1) {
        S[(int64_t)s * ld + l] = 1.0;
        return;
    }
    // progressive (bottom-up): D- into lbuf, U- into S one row down
    double dm = guard(d[t - 1] - lam);
    Lb[(int64_t)(t - 1) * ld + l] = dm;
    for (int i = t - 2; i >= s; i--) {
        const double u = e[i] / dm;
        S[(int64_t)(i + 1) * ld + l] = u;
        dm = guard(d[i] - lam - u * e[i]);
        Lb[(int64_t)i * ld + l] = dm;
    }
    // stationary (top-down): gamma at every row, L+ replaces D- in lbuf
    double dp = guard(d[s] - lam);
    int r = s;
    double gbest = 1.7976931348623157e308;
    for (int i = s; i < t; i++) {
        const double dmi = Lb[(int64_t)i * ld + l];
        const double gam = dp + dmi - (d[i] - lam);
        if (fabs(gam) < gbest) {
            gbest = fabs(gam);
            r = i;
        }
        if (i + 1 < t) {
            const double lp = e[i] / dp;
            Lb[(int64_t)i * ld + l] = lp;
            dp = guard(d[i + 1] - lam - lp * e[i]);
        }
    }
    double nrm = 1.0;
    double z = 1.0;
    S[(int64_t)r * ld + l] = 1.0;
    for (int i = r - 1; i >= s; i--) {
        z = -Lb[(int64_t)i * ld + l] * z;
        S[(int64_t)i * ld + l] = z;
        nrm += z * z;
    }
    z = 1.0;
    for (int i = r; i + 1 < t; i++) {
        z = -S[(int64_t)(i + 1) * ld + l] * z;
        S[(int64_t)(i + 1) * ld + l] = z;
        nrm += z * z;
    }
    const double inv = 1.0 / sqrt(nrm);
    for (int i = s; i < t; i++) S[(int64_t)i * ld + l] *= inv;
}

// Clusters: consecutive eigenvalues of one block closer than 1e-8 ||T|| (for
// instance the pairs of a degenerate spectrum when the reduction leaves them
// in one block) need not get independent vectors from twisted
// factorisations.  The lane of a cluster's first member recomputes all its
// vectors by inverse iteration with orthogonalisation against the members
// already done (as LAPACK's stein does): three steps of
// (T - lambda I) y = x by the LDL^T factorisation (pivots smaller than
// 1e-14 ||T|| raised to that size), each followed by modified Gram-Schmidt and
// normalisation, from deterministic start vectors that differ per member.
// Clusters are rare and small; everything else keeps its twisted vector.
__global__ __launch_bounds__(256)
void cluster_kernel(const GroupDesc *__restrict__ groups, int g0, EigVecs ev, double *__restrict__ sbase,
                    double *__restrict__ lbase)
{
    const int g = g0 + blockIdx.y;
    const GroupDesc gd = groups[g];
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= gd.n) return;
    const int ro = gd.rinfo_off, ld = gd.npad;
    const int s = ev.bs[ro + l], t = ev.be[ro + l];
    const double *lam = ev.lam + ro, *d = ev.d + ro, *e = ev.e + ro;
    double tn = 0.0;
    for (int i = s; i < t; i++)
        tn = fmax(tn, fabs(d[i]) + (i > s ? fabs(e[i - 1]) : 0.0) + (i + 1 < t ? fabs(e[i]) : 0.0));
    const double delta = 1e-8 * fmax(tn, 1e-300);
    auto close = [&](int a, int b) { return lam[b] - lam[a] <= delta; };
    if (l > s && close(l - 1, l)) return;            // not the first member
    if (l + 1 >= t || !close(l, l + 1)) return;      // a single eigenvalue
    int last = l + 1;
    while (last + 1 < t && close(last, last + 1)) last++;
    double *S = sbase + gd.off;
    double *Lb = lbase + gd.off;
    const double piv = 1e-14 * fmax(tn, 1e-300);
    for (int m = l; m <= last; m++) {
        double *x = S + m;                       // column m: x[i * ld]
        double *lm = Lb + m;
        for (int i = s; i < t; i++) x[(int64_t)i * ld] = 1.0 + 0.5 * sin(0.7 * (i - s + 1) * (m - l + 1) + m - l);
        for (int iter = 0; iter < 3; iter++) {
            // forward: LDL^T of T - lambda I with the solve of L z = x, w = D^-1 z
            double dd = d[s] - lam[m];
            if (fabs(dd) < piv) dd = dd < 0.0 ? -piv : piv;
            double z = x[(int64_t)s * ld];
            x[(int64_t)s * ld] = z / dd;
            for (int i = s; i + 1 < t; i++) {
                const double li = e[i] / dd;
                lm[(int64_t)i * ld] = li;
                dd = d[i + 1] - lam[m] - li * e[i];
                if (fabs(dd) < piv) dd = dd < 0.0 ? -piv : piv;
                z = x[(int64_t)(i + 1) * ld] - li * z;
                x[(int64_t)(i + 1) * ld] = z / dd;
            }
            // backward: L^T y = w
            for (int i = t - 2; i >= s; i--) x[(int64_t)i * ld] -= lm[(int64_t)i * ld] * x[(int64_t)(i + 1) * ld];
            // against the members already done, then normalise
            for (int p = l; p < m; p++) {
                double dot = 0.0;
                for (int i = s; i < t; i++) dot += S[(int64_t)i * ld + p] * x[(int64_t)i * ld];
                for (int i = s; i < t; i++) x[(int64_t)i * ld] -= dot * S[(int64_t)i * ld + p];
            }
            double nrm = 0.0;
            for (int i = s; i < t; i++) nrm += x[(int64_t)i * ld] * x[(int64_t)i * ld];
            const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
            for (int i = s; i < t; i++) x[(int64_t)i * ld] *= inv;
        }
    }
}

// ---- 4. own columns ---------------------------------------------------------
// y (n_pad x m_own, column-major at thin_off) = the own-column selector E.
__global__ __launch_bounds__(256)
void own_select_kernel(const GroupDesc *__restrict__ groups, const int32_t *__restrict__ own_list, int g0,
                       double *__restrict__ y)
{
    const GroupDesc gd = groups[g0 + blockIdx.y];
    const int64_t tot = (int64_t)gd.npad * gd.m_own;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < tot; q += (int64_t)gridDim.x * 256) {
        const int r = (int)(q % gd.npad), c = (int)(q / gd.npad);
        y[gd.thin_off + q] = (r == own_list[gd.own_off + c]) ? 1.0 : 0.0;
    }
}

// The reflectors applied to a thin block: forward (H_0 first: Y <- Q^T Y) or
// backward (H_{n-3} first: Y <- Q Y).  One 512-lane workgroup per group and
// chunk of 8 columns keeps its part of the block in registers (rows tid +
// 512 q); per reflector the 8 dot products are reduced in a fixed order (xor
// trees inside the waves, then the 8 waves in order), then every lane updates
// its rows.
constexpr int kReflCols = 8;
template <bool FORWARD>
__global__ __launch_bounds__(kReflBlock)
void reflect_kernel(const GroupDesc *__restrict__ groups, int g0, const double *__restrict__ abase,
                    EigVecs ev, double *__restrict__ y)
{
    constexpr int R = kEigMaxN / kReflBlock;
    constexpr int NWV = kReflBlock / 64;
    __shared__ double red[NWV][kReflCols];
    const GroupDesc gd = groups[g0 + blockIdx.y];
    const int c0 = blockIdx.x * kReflCols;
    if (c0 >= gd.m_own) return;
    const int nc = min(kReflCols, gd.m_own - c0);
    const int n = gd.n, ld = gd.npad, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double *A = abase + gd.off;
    const double *tau = ev.tau + gd.rinfo_off;
    double *yb = y + gd.thin_off + (int64_t)c0 * ld;
    double yr[R][kReflCols];
#pragma unroll
    for (int q = 0; q < R; q++) {
        const int i = tid + kReflBlock * q;
#pragma unroll
        for (int c = 0; c < kReflCols; c++) yr[q][c] = (i < n && c < nc) ? yb[i + (int64_t)c * ld] : 0.0;
    }
    // The next step's reflector and tau are loaded while this step's dot
    // products are reduced (the reflectors do not change); two register sets
    // take turns, so that no step waits on a memory round trip before its
    // products (the barriers of a step wait for LDS accesses, not for these
    // loads).  Every lane loads, rows beyond n reading row n - 1, so that the
    // loads sit outside any branch; rows outside the reflector are masked to
    // zero where they are used.
    auto load_v = [&](int step, double (&dst)[R], double &tdst) {
        const int k = FORWARD ? step : n - 3 - step;
        const double *v = A + (int64_t)k * ld;
        tdst = tau[k];
#pragma unroll
        for (int q = 0; q < R; q++) dst[q] = v[min(tid + kReflBlock * q, n - 1)];
    };
    auto apply = [&](int step, const double (&vl)[R], double t) {
        if (t == 0.0) return;
        const int k = FORWARD ? step : n - 3 - step;
        double vr[R];
#pragma unroll
        for (int q = 0; q < R; q++) {
            const int i = tid + kReflBlock * q;
            vr[q] = (i > k && i < n) ? vl[q] : 0.0;
        }
        double part[kReflCols];
#pragma unroll
        for (int c = 0; c < kReflCols; c++) part[c] = 0.0;
#pragma unroll
        for (int q = 0; q < R; q++)
#pragma unroll
            for (int c = 0; c < kReflCols; c++) part[c] += vr[q] * yr[q][c];
#pragma unroll
        for (int c = 0; c < kReflCols; c++) {
            double s = part[c];
            for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
            if (lane == 0) red[wave][c] = s;
        }
        __syncthreads();
        double sv[kReflCols];
#pragma unroll
        for (int c = 0; c < kReflCols; c++) {
            double s = 0.0;
            for (int w = 0; w < NWV; w++) s += red[w][c];
            sv[c] = t * s;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < R; q++)
#pragma unroll
            for (int c = 0; c < kReflCols; c++) yr[q][c] -= sv[c] * vr[q];
    };
    const int nsteps = n - 2;
    double va[R], vb[R], ta = 0.0, tb = 0.0;
    if (nsteps > 0) load_v(0, va, ta);
    // (the loads are unconditional, the last step's reflector read again at
    // the end: loads issued under a branch made the compiler wait for every
    // outstanding load where the paths join)
    for (int st = 0; st < nsteps; st += 2) {
        load_v(min(st + 1, nsteps - 1), vb, tb);
        apply(st, va, ta);
        if (st + 1 >= nsteps) break;
        load_v(min(st + 2, nsteps - 1), va, ta);
        apply(st + 1, vb, tb);
    }
#pragma unroll
    for (int q = 0; q < R; q++) {
        const int i = tid + kReflBlock * q;
#pragma unroll
        for (int c = 0; c < kReflCols; c++)
            if (i < ld && c < nc) yb[i + (int64_t)c * ld] = i < n ? yr[q][c] : 0.0;
    }
}

// g(lambda) = 1 - 2 f(lambda): tanh(lambda / 2kT) for kT > 0; at T = 0 the
// signum, 0 for |lambda| <= tau0 (Eq. signevext).
__device__ inline double occ_sign(double x, double kT, double tau0)
{
    if (kT > 0.0) return tanh(x / (2.0 * kT));
    if (fabs(x) <= tau0) return 0.0;
    return x < 0.0 ? -1.0 : 1.0;
}

// Thin products with S on 64 x 64 LDS tiles (one workgroup of 256 lanes per
// 64 output rows and chunk of 128 columns of a group; lane (r, j) accumulates
// output row r, columns j, j + 4, ... of the chunk):
//   MODE 0: C = S^T Y (rows l);
//   MODE 1: Z = S diag(g) C (rows i), g at lambda_l - dmu.
constexpr int kThinMax = 128;
template <int MODE>
__global__ __launch_bounds__(256)
void eig_thin_kernel(const GroupDesc *__restrict__ groups, int g0, EigVecs ev, const double *__restrict__ sbase,
                     const double *__restrict__ in, double *__restrict__ out, double mu0, double dmu, double kT,
                     const unsigned long long *__restrict__ scale_bits)
{
    __shared__ double Ssh[64][65];
    __shared__ double Bsh[64][kThinMax + 1];
    const int g = g0 + blockIdx.y;
    const GroupDesc gd = groups[g];
    const int ld = gd.npad, n = gd.n;
    const int r0 = blockIdx.x * 64, cb0 = blockIdx.z * kThinMax;
    if (r0 >= ld || cb0 >= gd.m_own) return;
    const int mo = min(kThinMax, gd.m_own - cb0);      // columns of this chunk
    const int tid = threadIdx.x, rr = tid & 63, jj = tid >> 6;
    const double *S = sbase + gd.off;
    const double *lam = ev.lam + gd.rinfo_off;
    const double sg = __longlong_as_double((long long)scale_bits[g]);
    const double tau0 = 1e-14 * sg;
    double acc[kThinMax / 4];
#pragma unroll
    for (int q = 0; q < kThinMax / 4; q++) acc[q] = 0.0;
    for (int k0 = 0; k0 < n; k0 += 64) {
        // S tile: MODE 0 rows k (sum index) x columns r (output rows l);
        // MODE 1 rows r (output rows i) x columns k (sum index l)
        for (int q = tid; q < 64 * 64; q += 256) {
            const int a = q >> 6, b = q & 63;          // b fastest: consecutive l in memory
            double v = 0.0;
            if (MODE == 0) {
                const int k = k0 + a, l = r0 + b;
                if (k < n && l < ld) v = S[(int64_t)k * ld + l];
                Ssh[a][b] = v;                          // [k][l]
            } else {
                const int i = r0 + a, l = k0 + b;
                if (i < ld && l < n) v = S[(int64_t)i * ld + l];
                Ssh[a][b] = v;                          // [i][l]
            }
        }
        for (int q = tid; q < 64 * mo; q += 256) {
            const int c = q / 64, a = q % 64;           // a fastest: consecutive rows of a column
            const int k = k0 + a;
            double v = 0.0;
            if (k < n) {
                v = in[gd.thin_off + k + (int64_t)(cb0 + c) * ld];
                if (MODE == 1) v *= occ_sign(lam[k] - dmu, kT, tau0);
            }
            Bsh[a][c] = v;
        }
        __syncthreads();
        const int kend = min(64, n - k0);
        for (int a = 0; a < kend; a++) {
            const double sv = MODE == 0 ? Ssh[a][rr] : Ssh[rr][a];
#pragma unroll
            for (int q = 0; q < kThinMax / 4; q++) {
                const int c = jj + 4 * q;
                if (c < mo) acc[q] += sv * Bsh[a][c];
            }
        }
        __syncthreads();
    }
    const int r = r0 + rr;
#pragma unroll
    for (int q = 0; q < kThinMax / 4; q++) {
        const int c = jj + 4 * q;
        if (c < mo && r < ld) out[gd.thin_off + r + (int64_t)(cb0 + c) * ld] = r < n ? acc[q] : 0.0;
    }
}

// Algorithm 1's weights w_l = sum over the own columns of C_lc^2 (= sum_{c in
// own} Q_cl^2), in column order, and the unshifted eigenvalues lambda_l + mu0.
__global__ __launch_bounds__(256)
void weights_kernel(const GroupDesc *__restrict__ groups, int g0, EigVecs ev, const double *__restrict__ cbuf,
                    double mu0)
{
    const GroupDesc gd = groups[g0 + blockIdx.y];
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= gd.n) return;
    double w = 0.0;
    for (int c = 0; c < gd.m_own; c++) {
        const double v = cbuf[gd.thin_off + l + (int64_t)c * gd.npad];
        w += v * v;
    }
    ev.w[gd.rinfo_off + l] = w;
    ev.lam_abs[gd.rinfo_off + l] = ev.lam[gd.rinfo_off + l] + mu0;
}

// N(mu_m) = sum_g sum_l w_gl (1 - g(lambda_gl - mu_m)) / 2 for nmu trial values
// (Algorithm 1): part[q * nmu + m] over the eigenvalues of group g0 + q in
// order, one lane per (group, trial).
__global__ __launch_bounds__(256)
void n_of_mu_kernel(const GroupDesc *__restrict__ groups, int g0, int ng, EigVecs ev, const double *__restrict__ mus,
                    int nmu, double kT, const unsigned long long *__restrict__ scale_bits, double *__restrict__ part)
{
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (u >= (int64_t)ng * nmu) return;
    const int q = (int)(u / nmu), m = (int)(u % nmu);
    const GroupDesc gd = groups[g0 + q];
    const double mu = mus[m];
    const double tau0 = 1e-14 * __longlong_as_double((long long)scale_bits[g0 + q]);
    double s = 0.0;
    for (int l = 0; l < gd.n; l++)
        s += ev.w[gd.rinfo_off + l] * 0.5 * (1.0 - occ_sign(ev.lam_abs[gd.rinfo_off + l] - mu, kT, tau0));
    part[u] = s;
}

// out[m] = sum over the groups in order of part[q * nmu + m].
__global__ __launch_bounds__(256)
void n_reduce_kernel(int ng, int nmu, const double *__restrict__ part, double *__restrict__ out)
{
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= nmu) return;
    double s = 0.0;
    for (int q = 0; q < ng; q++) s += part[(int64_t)q * nmu + m];
    out[m] = s;
}

}  // namespace

hipError_t launch_eig_tridiag(hipStream_t st, int g0, int ngroups, const GroupDesc *groups, double *a,
                              double *wpanel, const EigVecs &ev)
{
    if (ngroups <= 0) return hipSuccess;
    hipLaunchKernelGGL(tridiag_kernel, dim3((unsigned)ngroups), dim3(kEigBlock), 0, st, groups, g0, a, wpanel, ev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(split_kernel, dim3((unsigned)((ngroups + 63) / 64)), dim3(64), 0, st, groups, g0, ngroups, ev);
    return hipGetLastError();
}

hipError_t launch_eig_values_vectors(hipStream_t st, int g0, int ngroups, int max_npad, const GroupDesc *groups,
                                     const EigVecs &ev, double *s, double *scratch)
{
    if (ngroups <= 0) return hipSuccess;
    const dim3 grid((unsigned)((max_npad + 255) / 256), (unsigned)ngroups);
    hipLaunchKernelGGL(bisect_kernel, grid, dim3(256), 0, st, groups, g0, ev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(tvec_kernel, grid, dim3(256), 0, st, groups, g0, ev, s, scratch);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cluster_kernel, grid, dim3(256), 0, st, groups, g0, ev, s, scratch);
    return hipGetLastError();
}

hipError_t launch_eig_own_select(hipStream_t st, int g0, int ngroups, int max_npad, int max_own,
                                 const GroupDesc *groups, const int32_t *own_list, double *y)
{
    if (ngroups <= 0) return hipSuccess;
    const int64_t tot = (int64_t)max_npad * max_own;
    const dim3 grid((unsigned)std::min<int64_t>((tot + 255) / 256, 1024), (unsigned)ngroups);
    hipLaunchKernelGGL(own_select_kernel, grid, dim3(256), 0, st, groups, own_list, g0, y);
    return hipGetLastError();
}

hipError_t launch_eig_reflect(hipStream_t st, int forward, int g0, int ngroups, int max_own, const GroupDesc *groups,
                              const double *a, const EigVecs &ev, double *y)
{
    if (ngroups <= 0 || max_own <= 0) return hipSuccess;
    const dim3 grid((unsigned)((max_own + kReflCols - 1) / kReflCols), (unsigned)ngroups);
    if (forward)
        hipLaunchKernelGGL(reflect_kernel<true>, grid, dim3(kReflBlock), 0, st, groups, g0, a, ev, y);
    else
        hipLaunchKernelGGL(reflect_kernel<false>, grid, dim3(kReflBlock), 0, st, groups, g0, a, ev, y);
    return hipGetLastError();
}

hipError_t launch_eig_thin(hipStream_t st, int mode, int g0, int ngroups, int max_npad, int max_own,
                           const GroupDesc *groups, const EigVecs &ev, const double *s, const double *in, double *out,
                           double mu0, double dmu, double kT, const unsigned long long *scale_bits)
{
    if (ngroups <= 0 || max_own <= 0) return hipSuccess;
    const dim3 grid((unsigned)((max_npad + 63) / 64), (unsigned)ngroups, (unsigned)((max_own + kThinMax - 1) / kThinMax));
    if (mode == 0) {
        hipLaunchKernelGGL(eig_thin_kernel<0>, grid, dim3(256), 0, st, groups, g0, ev, s, in, out, mu0, dmu, kT,
                           scale_bits);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(weights_kernel, dim3((unsigned)((max_npad + 255) / 256), (unsigned)ngroups), dim3(256), 0,
                           st, groups, g0, ev, out, mu0);
    } else {
        hipLaunchKernelGGL(eig_thin_kernel<1>, grid, dim3(256), 0, st, groups, g0, ev, s, in, out, mu0, dmu, kT,
                           scale_bits);
    }
    return hipGetLastError();
}

hipError_t launch_n_of_mu(hipStream_t st, int ngroups, const GroupDesc *groups, const EigVecs &ev, const double *mus,
                          int nmu, double kT, const unsigned long long *scale_bits, double *part, double *out)
{
    if (ngroups <= 0 || nmu <= 0) return hipSuccess;
    const int64_t tot = (int64_t)ngroups * nmu;
    hipLaunchKernelGGL(n_of_mu_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, groups, 0, ngroups, ev,
                       mus, nmu, kT, scale_bits, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(n_reduce_kernel, dim3((unsigned)((nmu + 255) / 256)), dim3(256), 0, st, ngroups, nmu, part, out);
    return hipGetLastError();
}

}  // namespace smx
