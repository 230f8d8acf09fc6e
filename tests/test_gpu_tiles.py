"""GPU: size buckets of the word products (128 x 128 and 256 x 256 tiles).

The 256 x 256 kernel performs, for every output element, the same sequence of
matrix-core operations as the 128 x 128 kernel (K steps in order, word pairs
least significant first) and the same epilogue conversions, so D, N, E, step
counts and residuals must be bitwise equal whatever the bucket boundary
(smx_set_tile_shape).  Cases: every group on 256 x 256 tiles, a boundary that
splits the batch, ragged sizes from one 32-row block up to several 256-tiles
with ragged last tiles, one submatrix of n = 2600, and the sampled water1024
groups against the oracle in the configuration the benchmark times.
"""

import numpy as np
import pytest

from waterbox import water_config, random_block_system

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-6


@pytest.fixture(scope="module")
def smx():
    import paper_2004_10811_amd as smx
    smx.load_library()
    return smx


def run(smx, s, precision, shape, **kw):
    ctx = smx.Context(0).load(s).configure(precision=precision, **kw)
    smx.smx_set_tile_shape(ctx.handle, shape)
    res = ctx.evaluate(allow_not_converged=True)
    out = dict(d=res.d_values.copy(), n=res.n_elec, e=res.energy, status=res.status, info=ctx.group_info(),
               stats=ctx.stats(), prof=ctx.launch_profile())
    ctx.close()
    return out


def same(a, b):
    return (np.array_equal(a["d"], b["d"]) and a["n"] == b["n"] and a["e"] == b["e"] and a["status"] == b["status"]
            and np.array_equal(a["info"]["iters"], b["info"]["iters"])
            and np.array_equal(a["info"]["resid"], b["info"]["resid"]))


def ragged_system(seed):
    # groups of 1 .. 6 block columns with blocks of 5 .. 31: n_g from ~30 to ~700
    sizes = [13, 5, 5, 17, 9, 31, 22, 13, 27, 11, 5, 25, 7, 30, 19, 3, 28, 16] * 3
    nb = len(sizes)
    groups, j, w = [], 0, 1
    while j < nb:
        groups.append(list(range(j, min(j + w, nb))))
        j += w
        w = w % 6 + 1
    return random_block_system(seed, sizes, density=0.5, coupling=0.02, groups=groups, mu=0.0)


@pytest.mark.parametrize("precision", ["fp16x2", "bf16"])
@pytest.mark.parametrize("case", ["water16", "ragged"])
def test_tile_shapes_bitwise_equal(smx, oracle_lib, precision, case):
    s = water_config("water16") if case == "water16" else ragged_system(81)
    base = run(smx, s, precision, 0)
    all256 = run(smx, s, precision, 32)
    split = run(smx, s, precision, 160)
    kinds = {k: set(r["prof"][2].tolist()) for k, r in (("base", base), ("all", all256), ("split", split))}
    print(f"{case} {precision}: n_g {base['info']['n'].min()}-{base['info']['n'].max()}, launch kinds {kinds}")
    assert kinds["base"] <= {2, 3} and kinds["all"] <= {7, 8} and {7, 8} <= kinds["all"]
    assert same(base, all256) and same(base, split)
    if precision == "fp16x2":
        ref = oracle_lib.submatrix(s)
        err = float(np.abs(all256["d"] - ref.d_values).max())
        print(f"  max|dD| vs oracle {err:.2e}")
        assert err <= TOL_MIXED and base["status"] == smx.SMX_OK


def test_large_single_submatrix_on_256_tiles(smx):
    """n = 2600: eleven 256-tile rows with a ragged last one (40 rows)."""
    from waterbox import dense_to_bsc
    n, blk = 2600, 26
    h = np.zeros((n, n))
    hop = np.where(np.arange(n - 1) % 2 == 0, -1.0, -0.6)
    h[np.arange(n - 1), np.arange(1, n)] = hop
    h[np.arange(1, n), np.arange(n - 1)] = hop
    nb = n // blk
    s = dense_to_bsc(h, [blk] * nb, np.ones((nb, nb), dtype=bool), groups=[list(range(nb))], mu=0.0)
    a = run(smx, s, "fp16x2", 0)
    b = run(smx, s, "fp16x2", 256)
    lam, q = np.linalg.eigh(h)
    d_exact = q[:, lam < 0] @ q[:, lam < 0].T
    voff = s.val_off()
    err = 0.0
    for j in range(nb):
        for p in range(int(s.col_ptr[j]), int(s.col_ptr[j + 1])):
            i = int(s.row_idx[p])
            ref = d_exact[i * blk:(i + 1) * blk, j * blk:(j + 1) * blk].T.reshape(-1)
            err = max(err, float(np.abs(b["d"][voff[p]:voff[p + 1]] - ref).max()))
    print(f"n = 2600 on 256 x 256 tiles: max|dD| = {err:.2e}")
    assert same(a, b)
    assert err <= TOL_MIXED


def test_water1024_buckets_match_oracle(smx, oracle_lib):
    """The full water1024 batch with the bucket boundary splitting it, against
    every group on 128 x 128 tiles (bitwise) and the oracle on sampled groups."""
    s = water_config("water1024")
    a = run(smx, s, "fp16x2", 0)
    b = run(smx, s, "fp16x2", 864)
    n_g = a["info"]["n"]
    rng = np.random.default_rng(4321)
    pick = {int(np.argmax(n_g)), int(np.argmin(n_g))}
    while len(pick) < 6:
        pick.add(int(rng.integers(s.ngroups)))
    ref = oracle_lib.submatrix(s, which=sorted(pick))
    ok = ~np.isnan(ref.d_values)
    err = float(np.abs(b["d"][ok] - ref.d_values[ok]).max())
    ms_a, ms_b = a["stats"]["time_total_ms"], b["stats"]["time_total_ms"]
    print(f"water1024 fp16x2: {ms_a:.1f} ms (128 x 128) / {ms_b:.1f} ms (buckets at n_pad >= 864); "
          f"max|dD| vs oracle on {sorted(pick)}: {err:.2e}")
    assert same(a, b)
    assert err <= TOL_MIXED


def test_autotune_word_buckets(smx, oracle_lib, tmp_path, monkeypatch):
    """The autotuner's choice for 2-word FP16 (launch order x step graphs x size
    bucket boundary) gives bitwise the default result, and its cache record
    carries the bucket boundary."""
    cache = tmp_path / "smx_tune.txt"
    monkeypatch.setenv("SMX_TUNE_CACHE", str(cache))
    s = ragged_system(83)
    ref = run(smx, s, "fp16x2", 0)
    ctx = smx.Context(0).load(s).configure(precision="fp16x2")
    g, o, ms = smx.smx_autotune(ctx.handle, reps=1, use_cache=False)
    cfg = smx.smx_get_launch_config(ctx.handle)
    print(f"ragged fp16x2 autotune: {cfg}, {ms:.3f} ms")
    assert cfg["graph_steps"] == g and cfg["tile_order"] == o and cfg["big_min_npad"] in (0, 384, 640, 896)
    fields = cache.read_text().split()
    assert len(fields) == 5 and fields[1:4] == [str(g), str(o), str(cfg["big_min_npad"])]
    res = ctx.evaluate()
    assert np.array_equal(res.d_values, ref["d"]) and res.n_elec == ref["n"] and res.energy == ref["e"]
    ctx2 = smx.Context(0).load(s).configure(precision="fp16x2")
    assert smx.smx_autotune(ctx2.handle, reps=1, use_cache=True)[:2] == (g, o)
    assert smx.smx_get_launch_config(ctx2.handle) == cfg
    res2 = ctx2.evaluate()
    assert np.array_equal(res2.d_values, ref["d"])
    ctx.close()
    ctx2.close()
    refo = oracle_lib.submatrix(s)
    assert float(np.abs(res.d_values - refo.d_values).max()) <= TOL_MIXED


@pytest.mark.parametrize("precision", ["fp16x2", "bf16"])
@pytest.mark.parametrize("variant", [1, 2])
def test_kernel_variants_bitwise_equal(smx, precision, variant):
    """smx_set_kernel_variant: the register-prefetch operand stream (1) and the
    persistent launch over per-XCD work lists (2) give bitwise the results of
    the default launch, with direct launches and with step graphs."""
    s = ragged_system(85)
    ref = run(smx, s, precision, 0)
    for graph_steps in (0, 2):
        ctx = smx.Context(0).load(s).configure(precision=precision, graph_steps=graph_steps)
        smx.smx_set_kernel_variant(ctx.handle, variant)
        for _ in range(2):                        # a second evaluation reuses counters / graphs
            r = ctx.evaluate(allow_not_converged=True)
            assert np.array_equal(r.d_values, ref["d"]) and r.n_elec == ref["n"] and r.energy == ref["e"]
        assert np.array_equal(ctx.group_info()["iters"], ref["info"]["iters"])
        ctx.close()
