// Shapes of the submatrices (Sec. IV-C, "Minimization of Floating-Point
// Operations"), host code that acts on the sparsity pattern, the values'
// magnitudes and coordinates before any submatrix exists:
//  * group selection ("Generating Submatrices From Multiple Block Columns"):
//    the estimated additional speedup S of combining block columns into
//    submatrices (Eq. estimatedspeedup), and a k-means clustering of the block
//    columns' positions in space that proposes such combinations;
//  * splitting ("Splitting up submatrices"): the problem of the
//    sub-submatrices, one per single column, each holding the rows where that
//    column is non-zero element by element.
#include "smx.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <random>
#include <string>
#include <thread>
#include <vector>

namespace smx_groups {

std::string g_err;

int32_t fail(int32_t code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int32_t check_pattern(int32_t nblk, const int32_t *blk_size, const int64_t *col_ptr, const int32_t *row_idx)
{
    if (nblk <= 0 || !blk_size || !col_ptr || !row_idx) return fail(SMX_E_INVALID, "need nblk > 0 and the pattern");
    if (col_ptr[0] != 0) return fail(SMX_E_INVALID, "col_ptr[0] must be 0");
    for (int32_t j = 0; j < nblk; j++) {
        if (blk_size[j] < 1) return fail(SMX_E_INVALID, "block sizes must be positive");
        if (col_ptr[j + 1] < col_ptr[j]) return fail(SMX_E_INVALID, "col_ptr must be non-decreasing");
        for (int64_t p = col_ptr[j]; p < col_ptr[j + 1]; p++)
            if (row_idx[p] < 0 || row_idx[p] >= nblk) return fail(SMX_E_INVALID, "row index out of range");
    }
    return SMX_OK;
}

int32_t check_groups(int32_t nblk, int32_t ngroups, const int32_t *grp_ptr, const int32_t *grp_blocks)
{
    if (ngroups <= 0 || !grp_ptr || !grp_blocks) return fail(SMX_E_INVALID, "need ngroups > 0 and the groups");
    if (grp_ptr[0] != 0 || grp_ptr[ngroups] != nblk)
        return fail(SMX_E_INVALID, "groups must cover every block column exactly once");
    std::vector<char> seen((size_t)nblk, 0);
    for (int32_t g = 0; g < ngroups; g++) {
        if (grp_ptr[g + 1] <= grp_ptr[g]) return fail(SMX_E_INVALID, "empty group");
        for (int32_t q = grp_ptr[g]; q < grp_ptr[g + 1]; q++) {
            const int32_t j = grp_blocks[q];
            if (j < 0 || j >= nblk || seen[j]) return fail(SMX_E_INVALID, "block column listed twice or out of range");
            seen[j] = 1;
        }
    }
    return SMX_OK;
}

// n of the submatrix of a set of block columns: the sum of the block sizes of
// the union of their stored block rows (Sec. III-A step 1, Sec. IV-C).
double submatrix_dim(const int32_t *blk_size, const int64_t *col_ptr, const int32_t *row_idx, const int32_t *cols,
                     int32_t ncols, std::vector<int32_t> &mark, int32_t stamp)
{
    double n = 0.0;
    for (int32_t q = 0; q < ncols; q++) {
        const int32_t j = cols[q];
        for (int64_t p = col_ptr[j]; p < col_ptr[j + 1]; p++) {
            const int32_t i = row_idx[p];
            if (mark[i] != stamp) {
                mark[i] = stamp;
                n += blk_size[i];
            }
        }
    }
    return n;
}

// Squared distance of two points, plain or under the minimum-image
// convention of a cubic periodic box of edge `box` (box <= 0: plain).
inline double dist2(const double *a, const double *b, double box)
{
    double s = 0.0;
    for (int x = 0; x < 3; x++) {
        double d = a[x] - b[x];
        if (box > 0.0) d -= box * std::nearbyint(d / box);
        s += d * d;
    }
    return s;
}

}  // namespace smx_groups

using namespace smx_groups;

extern "C" {

int32_t smx_group_speedup(int32_t nblk, const int32_t *blk_size, const int64_t *col_ptr, const int32_t *row_idx,
                          int32_t ngroups, const int32_t *grp_ptr, const int32_t *grp_blocks, double *s_out,
                          double *work_out)
{
    if (int32_t st = check_pattern(nblk, blk_size, col_ptr, row_idx)) return st;
    if (int32_t st = check_groups(nblk, ngroups, grp_ptr, grp_blocks)) return st;
    if (!s_out && !work_out) return fail(SMX_E_INVALID, "s_out and work_out are both NULL");
    std::vector<int32_t> mark((size_t)nblk, -1);
    int32_t stamp = 0;
    double single = 0.0, grouped = 0.0;
    for (int32_t j = 0; j < nblk; j++) {
        const double n = submatrix_dim(blk_size, col_ptr, row_idx, &j, 1, mark, stamp++);
        single += n * n * n;
    }
    for (int32_t g = 0; g < ngroups; g++) {
        const double n = submatrix_dim(blk_size, col_ptr, row_idx, grp_blocks + grp_ptr[g], grp_ptr[g + 1] - grp_ptr[g],
                                       mark, stamp++);
        grouped += n * n * n;
    }
    if (s_out) *s_out = single / grouped;
    if (work_out) *work_out = grouped;
    return SMX_OK;
}

int32_t smx_group_kmeans(int32_t nblk, const double *coords, double box, int32_t nclusters, int32_t seed,
                         int32_t max_iter, int32_t *ngroups_out, int32_t *grp_ptr_out, int32_t *grp_blocks_out)
{
    if (nblk <= 0 || !coords || !ngroups_out || !grp_ptr_out || !grp_blocks_out)
        return fail(SMX_E_INVALID, "need nblk > 0, coords and the outputs");
    if (nclusters < 1 || nclusters > nblk) return fail(SMX_E_INVALID, "need 1 <= nclusters <= nblk");
    if (max_iter < 1) return fail(SMX_E_INVALID, "need max_iter >= 1");
    if (!(box >= 0.0) || !std::isfinite(box)) return fail(SMX_E_INVALID, "box must be finite and >= 0");
    for (int64_t i = 0; i < 3 * (int64_t)nblk; i++)
        if (!std::isfinite(coords[i])) return fail(SMX_E_NONFINITE, "coordinates must be finite");
    const int32_t k = nclusters;
    std::vector<double> cen((size_t)k * 3);
    std::mt19937_64 rng((uint64_t)(uint32_t)seed * 0x9E3779B97F4A7C15ull + 1);
    // k-means++ seeding: the first centre uniformly, then each next one with
    // probability proportional to the squared distance to the nearest centre
    std::vector<double> dmin((size_t)nblk, std::numeric_limits<double>::infinity());
    {
        const int32_t i0 = (int32_t)(rng() % (uint64_t)nblk);
        std::copy(coords + 3 * (int64_t)i0, coords + 3 * (int64_t)i0 + 3, cen.begin());
    }
    for (int32_t c = 1; c < k; c++) {
        double tot = 0.0;
        for (int32_t i = 0; i < nblk; i++) {
            dmin[i] = std::min(dmin[i], dist2(coords + 3 * (int64_t)i, &cen[3 * (size_t)(c - 1)], box));
            tot += dmin[i];
        }
        int32_t pick = nblk - 1;
        if (tot > 0.0) {
            const double r = std::uniform_real_distribution<double>(0.0, tot)(rng);
            double acc = 0.0;
            for (int32_t i = 0; i < nblk; i++) {
                acc += dmin[i];
                if (acc > r) {
                    pick = i;
                    break;
                }
            }
        } else {
            pick = (int32_t)(rng() % (uint64_t)nblk);
        }
        std::copy(coords + 3 * (int64_t)pick, coords + 3 * (int64_t)pick + 3, &cen[3 * (size_t)c]);
    }
    // Lloyd iterations: nearest centre (lowest index on ties), then the means
    // (circular means per axis in a periodic box)
    std::vector<int32_t> asg((size_t)nblk, -1);
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    for (int32_t it = 0; it < max_iter; it++) {
        std::vector<char> changed(nth, 0);
        auto work = [&](unsigned w) {
            for (int32_t i = (int32_t)w; i < nblk; i += (int32_t)nth) {
                int32_t best = 0;
                double bd = std::numeric_limits<double>::infinity();
                for (int32_t c = 0; c < k; c++) {
                    const double d = dist2(coords + 3 * (int64_t)i, &cen[3 * (size_t)c], box);
                    if (d < bd) {
                        bd = d;
                        best = c;
                    }
                }
                if (asg[i] != best) {
                    asg[i] = best;
                    changed[w] = 1;
                }
            }
        };
        std::vector<std::thread> pool;
        for (unsigned w = 1; w < nth; w++) pool.emplace_back(work, w);
        work(0);
        for (auto &th : pool) th.join();
        bool any = false;
        for (char ch : changed) any = any || ch;
        if (!any && it > 0) break;
        std::vector<double> s((size_t)k * 6, 0.0);
        std::vector<int32_t> cnt((size_t)k, 0);
        const double w2 = box > 0.0 ? 2.0 * M_PI / box : 0.0;
        for (int32_t i = 0; i < nblk; i++) {
            const int32_t c = asg[i];
            cnt[c]++;
            for (int x = 0; x < 3; x++) {
                const double v = coords[3 * (int64_t)i + x];
                if (box > 0.0) {
                    s[6 * (size_t)c + 2 * x] += std::cos(w2 * v);
                    s[6 * (size_t)c + 2 * x + 1] += std::sin(w2 * v);
                } else {
                    s[6 * (size_t)c + 2 * x] += v;
                }
            }
        }
        for (int32_t c = 0; c < k; c++) {
            if (!cnt[c]) continue;                    // an empty cluster keeps its centre
            for (int x = 0; x < 3; x++) {
                if (box > 0.0) {
                    double a = std::atan2(s[6 * (size_t)c + 2 * x + 1], s[6 * (size_t)c + 2 * x]) / w2;
                    if (a < 0.0) a += box;
                    cen[3 * (size_t)c + x] = a;
                } else {
                    cen[3 * (size_t)c + x] = s[6 * (size_t)c + 2 * x] / cnt[c];
                }
            }
        }
    }
    // groups: the non-empty clusters in the order of their first block column,
    // block columns ascending inside each
    std::vector<int32_t> order((size_t)k, -1);
    int32_t ng = 0;
    for (int32_t i = 0; i < nblk; i++)
        if (order[asg[i]] < 0) order[asg[i]] = ng++;
    std::vector<int32_t> cnt((size_t)ng + 1, 0);
    for (int32_t i = 0; i < nblk; i++) cnt[order[asg[i]] + 1]++;
    for (int32_t g = 0; g < ng; g++) cnt[g + 1] += cnt[g];
    std::copy(cnt.begin(), cnt.end(), grp_ptr_out);
    std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
    for (int32_t i = 0; i < nblk; i++) grp_blocks_out[pos[order[asg[i]]]++] = i;
    *ngroups_out = ng;
    return SMX_OK;
}

// The element-level problem: block sizes 1, column c keeps row r where r = c
// or where r lies in a stored block of c's block column and |K_rc| > eps.  For
// every own column c of a block-column submatrix A_g (c's block column in g)
// the rows of A_g that are non-zero in column c are exactly these rows, so the
// submatrix of element column c is the sub-submatrix of c (whatever group c's
// block column was in), and D's column c comes out of it.  Groups: single
// columns, or (merge != 0) runs of consecutive columns of one block column
// that keep the same rows, which share one sub-submatrix.
int32_t smx_split_columns(int32_t nblk, const int32_t *blk_size, const int64_t *col_ptr, const int32_t *row_idx,
                          const double *values, double eps, int32_t merge, int32_t *n_out, int64_t *nnz_out,
                          int32_t *ngroups_out, int64_t *e_col_ptr, int32_t *e_row_idx, double *e_values,
                          int64_t *e_src, int32_t *e_grp_ptr, int32_t *e_grp_cols)
{
    if (int32_t st = check_pattern(nblk, blk_size, col_ptr, row_idx)) return st;
    if (!values || !n_out || !nnz_out || !ngroups_out) return fail(SMX_E_INVALID, "need values and the size outputs");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(SMX_E_INVALID, "eps must be finite and >= 0");
    const bool fill = e_col_ptr != nullptr;
    if (fill && (!e_row_idx || !e_values || !e_src || !e_grp_ptr || !e_grp_cols))
        return fail(SMX_E_INVALID, "the fill call needs every output array");
    std::vector<int64_t> boff((size_t)nblk + 1, 0), voff((size_t)col_ptr[nblk] + 1, 0);
    for (int32_t j = 0; j < nblk; j++) boff[j + 1] = boff[j] + blk_size[j];
    for (int32_t j = 0; j < nblk; j++)
        for (int64_t p = col_ptr[j]; p < col_ptr[j + 1]; p++)
            voff[p + 1] = voff[p] + (int64_t)blk_size[row_idx[p]] * blk_size[j];
    for (int32_t j = 0; j < nblk; j++)
        for (int64_t p = col_ptr[j] + 1; p < col_ptr[j + 1]; p++)
            if (row_idx[p] <= row_idx[p - 1]) return fail(SMX_E_INVALID, "row_idx must ascend within a column");
    const int64_t n = boff[nblk];
    if (n > INT32_MAX) return fail(SMX_E_INVALID, "more than 2^31 - 1 columns");
    int64_t nnz = 0;
    int32_t ngroups = 0;
    std::vector<int32_t> rows, prev_rows;
    for (int32_t j = 0; j < nblk; j++) {
        const int32_t bj = blk_size[j];
        for (int32_t cc = 0; cc < bj; cc++) {
            const int64_t c = boff[j] + cc;
            rows.clear();
            if (fill) e_col_ptr[c] = nnz;
            for (int64_t p = col_ptr[j]; p < col_ptr[j + 1]; p++) {
                const int32_t i = row_idx[p];
                const int32_t bi = blk_size[i];
                const double *col = values + voff[p] + (int64_t)cc * bi;
                for (int32_t a = 0; a < bi; a++) {
                    const int64_t r = boff[i] + a;
                    if (r != c && !(std::fabs(col[a]) > eps)) continue;
                    if (fill) {
                        e_row_idx[nnz] = (int32_t)r;
                        e_values[nnz] = col[a];
                        e_src[nnz] = voff[p] + (int64_t)cc * bi + a;
                    }
                    rows.push_back((int32_t)r);
                    nnz++;
                }
            }
            const bool same = merge && cc > 0 && rows == prev_rows;
            if (!same) {
                if (fill) e_grp_ptr[ngroups] = (int32_t)c;
                ngroups++;
            }
            if (fill) e_grp_cols[c] = (int32_t)c;
            prev_rows.swap(rows);
        }
    }
    if (fill) {
        e_col_ptr[n] = nnz;
        e_grp_ptr[ngroups] = (int32_t)n;
    }
    *n_out = (int32_t)n;
    *nnz_out = nnz;
    *ngroups_out = ngroups;
    return SMX_OK;
}

const char *smx_group_last_error(void)
{
    return g_err.c_str();
}

}  // extern "C"
