"""Step graphs: the Newton-Schulz step launches replayed from captured HIP graphs.

Every replay must give bitwise the result of direct launches.  Each test
replays several times with the library's own eager work (gather, word
conversion, polish, scatter, reductions) and host synchronisation between the
replays, and checks every replay.
"""

import numpy as np
import pytest

from waterbox import water_config, random_block_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smx():
    import paper_2004_10811_amd as smx
    smx.load_library()
    return smx


def evaluate(ctx):
    res = ctx.evaluate()
    return res, ctx.group_info()


def same(a, b):
    (ra, ia), (rb, ib) = a, b
    np.testing.assert_array_equal(ra.d_values, rb.d_values)
    assert ra.n_elec == rb.n_elec and ra.energy == rb.energy
    np.testing.assert_array_equal(ia["iters"], ib["iters"])
    np.testing.assert_array_equal(ia["resid"], ib["resid"])


@pytest.mark.parametrize("precision,steps", [("fp64", 1), ("fp64", 4), ("fp16x2", 3), ("bf16x3", 5), ("fp32", 2)])
def test_graph_replays_equal_direct_launches(smx, oracle_lib, precision, steps):
    s = water_config("water16")
    direct = smx.Context(0).load(s).configure(precision=precision)
    ref = evaluate(direct)
    direct.close()
    ctx = smx.Context(0).load(s).configure(precision=precision, graph_steps=steps)
    for rep in range(3):
        got = evaluate(ctx)
        same(got, ref)
        # no per-launch profile for graph replays
        assert ctx.launch_profile()[0].size == 0
    ctx.close()
    o = oracle_lib.submatrix(s)
    ok = ~np.isnan(o.d_values)
    tol = 1e-10 if precision == "fp64" else 1e-6
    assert float(np.abs(ref[0].d_values[ok] - o.d_values[ok]).max()) <= tol


def test_graph_recaptures_when_settings_change(smx):
    s = random_block_system(12, [13, 5, 5] * 6, density=0.5, coupling=0.04, groups="pairs", mu=0.01)
    ctx = smx.Context(0).load(s).configure(precision="fp64", graph_steps=2)
    for tol, mu in [(1e-12, 0.01), (1e-9, 0.01), (1e-12, 0.03)]:
        ctx.configure(precision="fp64", tol=tol, mu=mu, graph_steps=2)
        got = evaluate(ctx)
        d = smx.Context(0).load(s).configure(precision="fp64", tol=tol, mu=mu)
        same(got, evaluate(d))
        d.close()
    # switching graphs off gives the direct path again
    ctx.configure(precision="fp64", graph_steps=0)
    evaluate(ctx)
    assert ctx.launch_profile()[0].size > 0
    ctx.close()


def test_graph_with_waves_and_mu_search(smx):
    s = water_config("water16")
    res = []
    for g in (0, 3):
        ctx = smx.Context(0).load(s).configure(precision="fp16x2", graph_steps=g, workspace_limit=8 << 20)
        r = evaluate(ctx)
        assert ctx.stats()["nwaves"] >= 2
        ctx.configure(precision="fp64", graph_steps=g)
        mu = smx.smx_find_mu(ctx.handle, round(r[0].n_elec) + 0.5, 1e-8, 30)
        res.append((r, mu))
        ctx.close()
    same(res[0][0], res[1][0])
    assert res[0][1] == res[1][1]


def test_tile_order_does_not_change_results(smx):
    s = random_block_system(14, [17, 9, 31, 4, 22, 13, 8, 27, 19, 11, 6, 25, 14], density=0.6,
                            coupling=0.04, groups="pairs", mu=0.01)
    out = []
    for order in (0, 1):
        ctx = smx.Context(0).load(s).configure(precision="fp16x2")
        smx.smx_set_tile_order(ctx.handle, order)
        out.append(evaluate(ctx))
        ctx.close()
    same(out[0], out[1])


def test_autotune_picks_a_configuration_and_caches_it(smx, tmp_path, monkeypatch):
    cache = tmp_path / "smx_tune.txt"
    monkeypatch.setenv("SMX_TUNE_CACHE", str(cache))
    s = water_config("water16")
    ref_ctx = smx.Context(0).load(s).configure(precision="fp64")
    ref = evaluate(ref_ctx)
    ref_ctx.close()
    ctx = smx.Context(0).load(s).configure(precision="fp64")
    g, o, ms = smx.smx_autotune(ctx.handle, reps=2, use_cache=False)
    print(f"water16 fp64 autotune: graph_steps {g}, tile order {o}, {ms:.3f} ms")
    assert g in (0, 2, 8) and o in (0, 1) and ms > 0
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split()[1:3] == [str(g), str(o)]
    same(evaluate(ctx), ref)
    # a second context reads the record instead of timing again
    ctx2 = smx.Context(0).load(s).configure(precision="fp64")
    assert smx.smx_autotune(ctx2.handle, reps=2, use_cache=True)[:2] == (g, o)
    assert len(cache.read_text().splitlines()) == 1
    same(evaluate(ctx2), ref)
    ctx.close()
    ctx2.close()
