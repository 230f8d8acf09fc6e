// Host-code driver for the AddressSanitizer / UndefinedBehaviorSanitizer
// build: the host-only parts of libsmx (group selection and splitting) and
// the plain C oracle, called on a small seeded problem and on bad arguments.
// Built with g++/gcc (no device code) by tests/test_sanitize.py; prints "ok".
#include "smx.h"

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
struct OracleInfo {
    int32_t n, nrow_blk, sweeps, n_neg, n_zero, pad;
    double min_abs_lambda, max_abs_lambda, inf_norm, eig_residual, orth_residual;
};
int32_t oracle_jacobi(int32_t n, double *a, double *lam, double *q, int32_t max_sweeps);
int32_t oracle_dense_map(int32_t n, const double *a, int32_t mode, double kT, double *out, double *lam_out,
                         double *q_out);
int32_t oracle_submatrix(int32_t nblk, const int32_t *blk_size, const int64_t *col_ptr, const int32_t *row_idx,
                         const double *values, int32_t ngroups, const int32_t *grp_ptr, const int32_t *grp_blocks,
                         double mu, double kT, const int32_t *which, int32_t nwhich, int32_t nthreads,
                         double *d_values, double *n_out, double *e_out, OracleInfo *info);
}

static int fails = 0;
#define CHECK(cond)                                                  \
    do {                                                             \
        if (!(cond)) {                                               \
            std::printf("check failed: %s (line %d)\n", #cond, __LINE__); \
            fails++;                                                 \
        }                                                            \
    } while (0)

int main()
{
    std::mt19937_64 rng(7);
    std::normal_distribution<double> nd(0.0, 0.05);
    const std::vector<int32_t> bs = {3, 5, 2, 4, 6, 1, 3, 5};
    const int32_t nb = (int32_t)bs.size();
    // symmetric pattern: |I - J| <= 1, plus (0, 5) and (2, 7)
    std::vector<std::vector<char>> m(nb, std::vector<char>(nb, 0));
    for (int i = 0; i < nb; i++)
        for (int j = 0; j < nb; j++) m[i][j] = std::abs(i - j) <= 1;
    m[0][5] = m[5][0] = m[2][7] = m[7][2] = 1;
    std::vector<int64_t> boff(nb + 1, 0);
    for (int j = 0; j < nb; j++) boff[j + 1] = boff[j] + bs[j];
    const int64_t n = boff[nb];
    std::vector<double> kd((size_t)(n * n), 0.0);
    for (int64_t c = 0; c < n; c++)
        for (int64_t r = c; r < n; r++) {
            double v = (r == c) ? ((r % 2) ? 0.5 : -0.5) + nd(rng) : nd(rng);
            kd[r + c * n] = kd[c + r * n] = v;
        }
    std::vector<int64_t> cp(nb + 1, 0);
    std::vector<int32_t> ri;
    std::vector<double> vals;
    for (int j = 0; j < nb; j++) {
        for (int i = 0; i < nb; i++) {
            if (!m[i][j]) continue;
            ri.push_back(i);
            for (int b = 0; b < bs[j]; b++)
                for (int a = 0; a < bs[i]; a++) {
                    double v = kd[(boff[i] + a) + (boff[j] + b) * n];
                    if (std::fabs(v) < 0.02 && boff[i] + a != boff[j] + b) v = 0.0;   // element zeros
                    vals.push_back(v);
                }
        }
        cp[j + 1] = (int64_t)ri.size();
    }
    // symmetric element zeros: the mirror of a zeroed element is zeroed above too (same |v|)
    const std::vector<int32_t> gp = {0, 2, 4, 6, 8}, gb = {0, 1, 2, 3, 4, 5, 6, 7};

    // oracle
    std::vector<double> d(vals.size(), 0.0);
    double ne = 0, ee = 0;
    std::vector<OracleInfo> info(4);
    CHECK(oracle_submatrix(nb, bs.data(), cp.data(), ri.data(), vals.data(), 4, gp.data(), gb.data(), 0.0, 0.0,
                           nullptr, 4, 2, d.data(), &ne, &ee, info.data()) == 0);
    CHECK(std::fabs(ne) > 0 && std::isfinite(ee));
    std::vector<double> a((size_t)(n * n)), lam(n), q((size_t)(n * n)), out((size_t)(n * n));
    a = kd;
    CHECK(oracle_jacobi((int32_t)n, a.data(), lam.data(), q.data(), 60) > 0);
    CHECK(oracle_dense_map((int32_t)n, kd.data(), 1, 0.05, out.data(), nullptr, nullptr) == 0);
    CHECK(oracle_dense_map(-1, kd.data(), 1, 0.0, out.data(), nullptr, nullptr) != 0);

    // group selection
    double s = 0, work = 0;
    CHECK(smx_group_speedup(nb, bs.data(), cp.data(), ri.data(), 4, gp.data(), gb.data(), &s, &work) == SMX_OK);
    CHECK(s > 0 && work > 0);
    const std::vector<int32_t> bad_gp = {0, 2, 4, 6, 7};
    CHECK(smx_group_speedup(nb, bs.data(), cp.data(), ri.data(), 4, bad_gp.data(), gb.data(), &s, &work) ==
          SMX_E_INVALID);
    std::uniform_real_distribution<double> ud(0.0, 10.0);
    std::vector<double> xyz(3 * nb);
    for (auto &x : xyz) x = ud(rng);
    std::vector<int32_t> kp(nb + 1), kb(nb);
    int32_t ng = 0;
    CHECK(smx_group_kmeans(nb, xyz.data(), 10.0, 3, 1, 50, &ng, kp.data(), kb.data()) == SMX_OK);
    CHECK(ng >= 1 && ng <= 3 && kp[ng] == nb);
    CHECK(smx_group_kmeans(nb, xyz.data(), 0.0, nb + 1, 1, 50, &ng, kp.data(), kb.data()) == SMX_E_INVALID);

    // splitting
    int32_t en = 0, eng = 0;
    int64_t ennz = 0;
    CHECK(smx_split_columns(nb, bs.data(), cp.data(), ri.data(), vals.data(), 0.0, 1, &en, &ennz, &eng, nullptr,
                            nullptr, nullptr, nullptr, nullptr, nullptr) == SMX_OK);
    std::vector<int64_t> ecp(en + 1), esrc(ennz);
    std::vector<int32_t> eri(ennz), egp(eng + 1), egc(en);
    std::vector<double> ev(ennz);
    CHECK(smx_split_columns(nb, bs.data(), cp.data(), ri.data(), vals.data(), 0.0, 1, &en, &ennz, &eng, ecp.data(),
                            eri.data(), ev.data(), esrc.data(), egp.data(), egc.data()) == SMX_OK);
    CHECK(en == n && ecp[en] == ennz && egp[eng] == en);
    for (int64_t t = 0; t < ennz; t++) CHECK(ev[t] == vals[esrc[t]]);
    CHECK(smx_split_columns(nb, bs.data(), cp.data(), ri.data(), vals.data(), -1.0, 1, &en, &ennz, &eng, nullptr,
                            nullptr, nullptr, nullptr, nullptr, nullptr) == SMX_E_INVALID);
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}
