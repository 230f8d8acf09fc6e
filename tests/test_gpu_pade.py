"""GPU: the third-order Pade sign iteration (Sec. VI-A) against the oracle.

The iteration changes the path to sign(A_g), not the result: D must meet the
same bars (1e-10 FP64, 1e-6 reduced precision) against the Jacobi oracle.  The
FP64 residual history max|X_k^2 - I| must follow the oracle's eigenpairs
through the scalar Pade map, X_k = Q p_k(Lambda / s) Q^T (which pins the
iteration itself, not only its limit).  Size buckets stay bitwise equal, and
the maps that differentiate the Newton-Schulz polynomial refuse a Pade
evaluation.
"""

import numpy as np
import pytest

from waterbox import water_config, random_block_system

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp16x2": 1e-6, "bf16x3": 1e-6, "fp32": 1e-6}


@pytest.fixture(scope="module")
def smx():
    import paper_2004_10811_amd as smx
    smx.load_library()
    return smx


def run(smx, s, precision, iteration, shape=0, **kw):
    ctx = smx.Context(0).load(s).configure(precision=precision, iteration=iteration, tile_shape=shape, **kw)
    res = ctx.evaluate()
    out = dict(d=res.d_values.copy(), n=res.n_elec, e=res.energy, info=ctx.group_info(), stats=ctx.stats())
    ctx.close()
    return out


def ragged():
    return random_block_system(91, [13, 5, 5, 17, 9, 31, 22, 13, 27, 11, 5, 25] * 3, density=0.45,
                               coupling=0.02, groups="pairs", mu=0.01)


@pytest.mark.parametrize("precision", ["fp64", "fp16x2", "bf16x3", "fp32"])
@pytest.mark.parametrize("case", ["water16", "ragged"])
def test_pade_matches_oracle(smx, oracle_lib, precision, case):
    s = water_config("water16") if case == "water16" else ragged()
    ref = oracle_lib.submatrix(s)
    pd = run(smx, s, precision, "pade3")
    ns = run(smx, s, precision, "ns2")
    err = float(np.abs(pd["d"] - ref.d_values).max())
    print(f"{case} {precision}: Pade max|dD| = {err:.2e}, steps {pd['stats']['iters_min']}-{pd['stats']['iters_max']} "
          f"(Newton-Schulz {ns['stats']['iters_min']}-{ns['stats']['iters_max']}), dN = {pd['n'] - ref.n_elec:.1e}")
    assert err <= TOL[precision]
    assert abs(pd["n"] - ref.n_elec) <= TOL[precision] * s.n
    assert pd["stats"]["n_not_converged"] == 0
    assert pd["stats"]["iters_max"] < ns["stats"]["iters_max"]


def test_pade_fp64_history_follows_the_scalar_map(smx, oracle_lib):
    s = water_config("water16")
    ctx = smx.Context(0).load(s).configure(precision="fp64", iteration="pade3")
    ctx.evaluate()
    info = ctx.group_info()
    h = smx.smx_get_history(ctx.handle, 64)
    ctx.close()
    np.testing.assert_array_equal(h["nsteps"], info["iters"] + 1)
    for g in (0, 5, s.ngroups - 1):
        n = int(h["nsteps"][g])
        _, lam, q, _ = oracle_lib.group_eig(s, g)
        r_or = []
        for k in range(n):
            x = oracle_lib.pade_poly(lam / info["scale"][g], k)
            r_or.append(float(np.abs((q * (1.0 - x * x)) @ q.T).max()))
        r_or = np.array(r_or)
        r = h["resid"][g, :n]
        print(f"group {g}: {n} Pade steps, resid {r[0]:.3e} -> {r[-1]:.3e}")
        assert np.all(np.abs(r - r_or) <= 1e-11 + 1e-10 * r_or)
        assert r[-1] <= 1e-12 < r[-2]


@pytest.mark.parametrize("precision", ["fp16x2", "bf16"])
def test_pade_buckets_bitwise_equal(smx, precision):
    s = ragged()
    a = run(smx, s, precision, "pade3", 0, max_iter=100, n_polish=4 if precision == "bf16" else 2)
    b = run(smx, s, precision, "pade3", 32, max_iter=100, n_polish=4 if precision == "bf16" else 2)
    assert np.array_equal(a["d"], b["d"]) and a["n"] == b["n"] and a["e"] == b["e"]
    assert np.array_equal(a["info"]["iters"], b["info"]["iters"])


def test_pade_large_single_submatrix(smx):
    """n = 2600 dimerized chain (gap [-0.4, 0.4]): exact D from LAPACK."""
    from waterbox import dense_to_bsc
    n, blk = 2600, 26
    h = np.zeros((n, n))
    hop = np.where(np.arange(n - 1) % 2 == 0, -1.0, -0.6)
    h[np.arange(n - 1), np.arange(1, n)] = hop
    h[np.arange(1, n), np.arange(n - 1)] = hop
    nb = n // blk
    s = dense_to_bsc(h, [blk] * nb, np.ones((nb, nb), dtype=bool), groups=[list(range(nb))], mu=0.0)
    lam, q = np.linalg.eigh(h)
    d_exact = q[:, lam < 0] @ q[:, lam < 0].T
    voff = s.val_off()
    for precision in ("fp64", "fp16x2"):
        r = run(smx, s, precision, "pade3", 256)
        err = 0.0
        for j in range(nb):
            for p in range(int(s.col_ptr[j]), int(s.col_ptr[j + 1])):
                i = int(s.row_idx[p])
                ref = d_exact[i * blk:(i + 1) * blk, j * blk:(j + 1) * blk].T.reshape(-1)
                err = max(err, float(np.abs(r["d"][voff[p]:voff[p + 1]] - ref).max()))
        print(f"n = 2600 Pade {precision}: max|dD| = {err:.2e}, {r['stats']['iters_max']} steps")
        assert err <= TOL[precision]


def test_water1024_pade_sampled_groups(smx, oracle_lib):
    s = water_config("water1024")
    pd = run(smx, s, "fp16x2", "pade3")
    ns = run(smx, s, "fp16x2", "ns2")
    n_g = pd["info"]["n"]
    rng = np.random.default_rng(4321)
    pick = {int(np.argmax(n_g)), int(np.argmin(n_g))}
    while len(pick) < 6:
        pick.add(int(rng.integers(s.ngroups)))
    ref = oracle_lib.submatrix(s, which=sorted(pick))
    ok = ~np.isnan(ref.d_values)
    err = float(np.abs(pd["d"][ok] - ref.d_values[ok]).max())
    print(f"water1024 fp16x2: Pade {pd['stats']['time_total_ms']:.1f} ms ({pd['stats']['iters_mean']:.2f} steps), "
          f"Newton-Schulz {ns['stats']['time_total_ms']:.1f} ms ({ns['stats']['iters_mean']:.2f} steps); "
          f"max|dD| vs oracle {err:.2e}, vs Newton-Schulz {float(np.abs(pd['d'] - ns['d']).max()):.2e}")
    assert err <= 1e-6


def test_derivative_maps_refuse_pade(smx):
    s = water_config("water16")
    ctx = smx.Context(0).load(s).configure(precision="fp64", iteration="pade3")
    ctx.evaluate()
    for call in (lambda: smx.smx_set_frozen(ctx.handle, 1),
                 lambda: smx.smx_backward(ctx.handle, 1.0, 0.0, None, np.empty(ctx.nvalues))):
        with pytest.raises(smx.SmxError) as ei:
            call()
        assert ei.value.code == smx.SMX_E_UNSUPPORTED
    with pytest.raises(smx.SmxError) as ei:
        smx.smx_find_mu(ctx.handle, s.n / 2)
    assert ei.value.code == smx.SMX_E_UNSUPPORTED
    ctx.close()
