"""Pins of the oracle's frozen-iteration quantities (electron count and dN/dmu)."""

import numpy as np

from waterbox import water_system, random_block_system


def test_ns_poly_fixed_points_and_derivative():
    import oracle
    # +-1 and 0 are fixed points of p(x) = x(3 - x^2)/2; p'(0) = 3/2 per step
    assert np.allclose(oracle.ns_poly([-1.0, 0.0, 1.0], 7), [-1.0, 0.0, 1.0])
    assert np.isclose(oracle.ns_poly_deriv(0.0, 5), 1.5 ** 5)
    x = np.linspace(-0.9, 0.9, 13)
    h = 1e-6
    fd = (oracle.ns_poly(x + h, 6) - oracle.ns_poly(x - h, 6)) / (2 * h)
    assert np.allclose(oracle.ns_poly_deriv(x, 6), fd, rtol=1e-6, atol=1e-8)


def test_frozen_count_converges_to_the_submatrix_count(oracle_lib):
    """Many steps: p_k -> sign, so N_k(mu) -> Tr D of the submatrix method."""
    s = water_system(n_mol=6, box=6.0, r_cut=3.5, seed=41)
    spec = oracle_lib.GroupSpectra(s)
    mu = 0.02
    ref = oracle_lib.submatrix(s, mu=mu)
    scale = [np.abs(np.linalg.eigvalsh(np.diag(l) - mu * np.eye(len(l)))).max() * 1.3 for l in spec.lam]
    k = [80] * s.ngroups
    assert abs(spec.n_frozen(mu, k, scale) - ref.n_elec) < 1e-10
    # dN/dmu of the converged map vanishes inside the gap
    assert abs(spec.dn_dmu_frozen(mu, k, scale)) < 1e-8


def test_frozen_dn_dmu_matches_finite_differences(oracle_lib):
    s = random_block_system(43, [4, 3, 5, 2, 6], density=0.6, coupling=0.05, groups="column")
    spec = oracle_lib.GroupSpectra(s)
    k = [3, 4, 5, 2, 6]
    scale = [2.0, 1.5, 2.5, 1.8, 2.2]
    mu, h = 0.05, 1e-6
    fd = (spec.n_frozen(mu + h, k, scale) - spec.n_frozen(mu - h, k, scale)) / (2 * h)
    assert abs(spec.dn_dmu_frozen(mu, k, scale) - fd) <= 1e-6 * max(1.0, abs(fd))


def test_weights_sum_to_own_column_count(oracle_lib):
    s = water_system(n_mol=4, box=5.0, r_cut=3.0, seed=42)
    spec = oracle_lib.GroupSpectra(s)
    for t, g in enumerate(spec.groups):
        own = s.blk_size[s.grp_blocks[s.grp_ptr[g]:s.grp_ptr[g + 1]]].sum()
        assert abs(spec.w[t].sum() - own) < 1e-12


def _sym_direction(s, rng, i, j):
    """Random symmetric change of K on the block pair (I, J) and (J, I)."""
    voff = s.val_off()
    v = np.zeros_like(s.values)
    where = {}
    for jj in range(s.nblk):
        for p in range(s.col_ptr[jj], s.col_ptr[jj + 1]):
            where[(int(s.row_idx[p]), jj)] = p
    bi, bj = s.blk_size[i], s.blk_size[j]
    m = rng.normal(size=(bi, bj))
    if i == j:
        m = m + m.T
    p = where[(i, j)]
    v[voff[p]:voff[p + 1]] = m.reshape(-1, order="F")
    if i != j:
        q = where[(j, i)]
        v[voff[q]:voff[q + 1]] = m.T.reshape(-1, order="F")
    return v


def test_frozen_gradient_matches_finite_differences(oracle_lib):
    """Daleckii-Krein gradient of L = gE E + gN N + <gD, D> vs central differences."""
    s = random_block_system(47, [3, 4, 2, 5, 3], density=0.6, coupling=0.06, groups=[[0, 1], [2], [3, 4]])
    k = [4, 3, 5]
    scale = [2.0, 2.5, 1.7]
    mu = 0.03
    rng = np.random.default_rng(5)
    gd = rng.normal(size=s.values.shape)
    ge, gn = 0.7, -1.3

    def loss(vals, m):
        r = oracle_lib.frozen_gradient(s, k, scale, m, values=vals)
        return ge * r["energy"] + gn * r["n_elec"] + float(np.dot(gd, r["d_values"]))

    r0 = oracle_lib.frozen_gradient(s, k, scale, mu, ge, gn, gd)
    h = 1e-6
    for (i, j) in [(0, 0), (1, 0), (3, 4), (2, 2), (4, 3)]:
        try:
            v = _sym_direction(s, rng, i, j)
        except KeyError:
            continue
        fd = (loss(s.values + h * v, mu) - loss(s.values - h * v, mu)) / (2 * h)
        ad = float(np.dot(r0["dk"], v))
        assert abs(fd - ad) <= 1e-6 * max(1.0, abs(ad)), (i, j, fd, ad)
    fd_mu = (loss(s.values, mu + h) - loss(s.values, mu - h)) / (2 * h)
    assert abs(fd_mu - r0["dmu"]) <= 1e-6 * max(1.0, abs(fd_mu))


def test_frozen_gradient_dmu_equals_tangent_form(oracle_lib):
    """dN/dmu from the reverse form equals the closed form sum w p_k'/(2s)."""
    s = water_system(n_mol=4, box=5.0, r_cut=3.0, seed=44)
    spec = oracle_lib.GroupSpectra(s)
    k = [5] * s.ngroups
    scale = [4.0] * s.ngroups
    r = oracle_lib.frozen_gradient(s, k, scale, 0.02, gN=1.0)
    assert abs(r["dmu"] - spec.dn_dmu_frozen(0.02, k, scale)) <= 1e-10 * max(1.0, abs(r["dmu"]))


def test_frozen_forward_equals_submatrix_at_large_k(oracle_lib):
    """frozen_gradient's forward outputs (D, N, E) are the k-step map
    D = (I - p_k(A_g / s_g)) / 2; with k = 80 steps every eigenvalue with
    |lambda| / s_g >= 1e-3 has reached +-1 to rounding (1.5^80 >> 1e3), so the
    map must equal the oracle's Jacobi submatrix D (signum of the eigenvalues)."""
    from waterbox import water_config, random_block_system
    for s in (water_config("water16"),
              random_block_system(23, [5, 3, 8, 2, 6, 4, 7, 5], density=0.5, coupling=0.05,
                                  groups=[[0, 1], [2], [3, 4, 5], [6, 7]], mu=0.02)):
        k = np.full(s.ngroups, 80)
        scale = np.zeros(s.ngroups)
        ref = oracle_lib.submatrix(s)
        # a bound on each group's spectral radius, so that every |lambda / s| <= 1
        for g in range(s.ngroups):
            _, lam, _, _ = oracle_lib.group_eig(s, g)
            scale[g] = 1.05 * np.abs(lam).max()
            assert np.abs(lam).min() / scale[g] > 1e-3
        fz = oracle_lib.frozen_gradient(s, k, scale, s.mu)
        assert np.abs(fz["d_values"] - ref.d_values).max() <= 1e-12
        assert abs(fz["n_elec"] - ref.n_elec) <= 1e-11
        assert abs(fz["energy"] - ref.energy) <= 1e-11
