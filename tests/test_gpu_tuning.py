"""Launch tuning, graph-captured iterations and the autotuner.

None of these may change what is computed: the grid caps and the graph/eager
issue mode leave every result bit-identical (each tile writes its own FP64
partials, summed in a fixed order whatever the grid); the stencil tile height
regroups those partials, so results move only by rounding.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2203_13675_amd import synth  # noqa: E402

SHAPES = [(128, 256), (256, 128), (96, 77), (200, 64), (1, 90)]


@pytest.fixture()
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_13675_amd.binding import Context
    c = Context(0)
    yield c
    c.close()


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def demeaned_diff(a, b):
    return float(np.abs((a - a.mean()) - (b - b.mean())).max())


def run_batch(ctx, maps, pc="dct", precision="mixed", **kw):
    psis = [dev(p) for p, _ in maps]
    phis, rc, stats = ctx.batch(psis, p=0.0, preconditioner=pc, precision=precision, k_max=3,
                                outer_tol=0.0, **kw)
    return [host(x) for x in phis], stats


@pytest.mark.parametrize("pc,precision", [("dct", "mixed"), ("jacobi", "mixed"), ("dct", "fp64"),
                                          ("none", "fp64")])
def test_graph_and_eager_are_bit_identical(ctx, pc, precision):
    maps = synth.batch_maps(sides=SHAPES, seed=5)
    ctx.set_tuning(use_graph=1)
    a, sa = run_batch(ctx, maps, pc, precision)
    ctx.set_tuning(use_graph=0)
    b, sb = run_batch(ctx, maps, pc, precision)
    for k in range(len(maps)):
        assert np.array_equal(a[k], b[k]), SHAPES[k]
        assert sa[k]["inner_iters_total"] == sb[k]["inner_iters_total"]
        assert sa[k]["final_relres"] <= 1e-6


def test_grid_caps_do_not_change_results(ctx):
    """Tiny grids force many grid-stride passes over the tile lists."""
    maps = synth.batch_maps(sides=SHAPES, seed=6)
    ref, _ = run_batch(ctx, maps)
    ctx.set_tuning(grid=64, dct_grid=64, max_batch_iters=3)
    small, _ = run_batch(ctx, maps)
    for k in range(len(maps)):
        assert np.array_equal(ref[k], small[k]), SHAPES[k]


@pytest.mark.parametrize("rows", [4, 8, 32, 64])
def test_tile_rows_change_only_rounding(ctx, rows):
    """Other stencil tile heights (including a ragged last tile row and the
    run-time-length loop of 64) reach the same solution up to the tolerance."""
    maps = synth.batch_maps(sides=SHAPES, seed=7)
    ref, _ = run_batch(ctx, maps)
    ctx.set_tuning(tile_rows=rows)
    assert ctx.tuning()["tile_rows"] == rows
    got, st = run_batch(ctx, maps)
    for k in range(len(maps)):
        assert st[k]["final_relres"] <= 1e-6
        assert demeaned_diff(ref[k], got[k]) <= 1e-4, (SHAPES[k], rows)


def test_graph_replays_reuse_across_shrinking_sets(ctx):
    """Maps of very different sizes finish at different times, so the active
    set shrinks between host checks; repeated calls reuse nothing stale."""
    shapes = [(32, 32), (256, 384), (64, 48), (384, 256)]
    maps = synth.batch_maps(sides=shapes, seed=8)
    first, s1 = run_batch(ctx, maps)
    second, s2 = run_batch(ctx, maps)
    ctx.set_tuning(use_graph=0)
    eager, s3 = run_batch(ctx, maps)
    for k in range(len(shapes)):
        assert np.array_equal(first[k], second[k])
        assert np.array_equal(first[k], eager[k])


def test_graphs_kept_across_calls_follow_layout_and_parameters(ctx):
    """Captured graphs outlive a call (they are dropped only when the work
    buffers are reallocated): a later call with another map layout that fits
    the same buffers, another tile height or another SSOR omega must replay
    graphs that match it.  Every call is compared with a fresh context's
    eager run of the same call, bit for bit."""
    from paper_2203_13675_amd.binding import Context
    big = synth.batch_maps(sides=[(256, 384), (384, 256), (128, 128)], seed=11)
    small = synth.batch_maps(sides=[(128, 256), (256, 128)], seed=12)
    calls = [(big, "dct", {}, 16), (small, "dct", {}, 16), (small, "dct", {}, 32),
             (big, "ssor_rb", {"ssor_omega": 1.0}, 16), (big, "ssor_rb", {"ssor_omega": 1.6}, 16),
             (small, "ssor", {"ssor_omega": 1.3}, 16), (small, "ssor", {"ssor_omega": 1.0}, 16)]
    ctx.set_tuning(use_graph=1)
    for maps, pc, kw, rows in calls:
        ctx.set_tuning(tile_rows=rows)
        got, sg = run_batch(ctx, maps, pc, **kw)
        ref_ctx = Context(0)
        try:
            ref_ctx.set_tuning(use_graph=0, tile_rows=rows)
            ref, sr = run_batch(ref_ctx, maps, pc, **kw)
        finally:
            ref_ctx.close()
        for k in range(len(maps)):
            assert np.array_equal(got[k], ref[k]), (pc, kw, rows, k)
            assert sg[k]["inner_iters_total"] == sr[k]["inner_iters_total"]


def test_set_tuning_rejects_bad_values(ctx):
    from paper_2203_13675_amd.binding import LpuError
    before = ctx.tuning()
    for kw in ({"tile_rows": 12}, {"grid": 8}, {"dct_grid": 1 << 20}, {"use_graph": 2},
               {"max_batch_iters": 1}):
        with pytest.raises(LpuError):
            ctx.set_tuning(**kw)
        assert ctx.tuning() == before
    assert ctx.set_tuning(default=True) == before


def test_autotune_installs_and_caches(ctx, tmp_path):
    maps = synth.batch_maps(sides=[(128, 128), (256, 128), (64, 96)], seed=9)
    psis = [dev(p) for p, _ in maps]
    cache = tmp_path / "tune.txt"
    best, ms = ctx.autotune(psis, p=0.0, preconditioner="dct", precision="mixed",
                            probe_iters=8, cache_path=cache)
    assert ms > 0.0
    assert best == ctx.tuning()
    assert best["tile_rows"] in (4, 8, 16, 32) and best["use_graph"] in (0, 1)
    line = cache.read_text().strip().split("\n")[-1].split()
    assert [int(x) for x in line[1:]] == [best["tile_rows"], best["grid"], best["dct_grid"],
                                          best["use_graph"], best["max_batch_iters"]]
    # a cache hit installs the stored tuning without timing anything
    ctx.set_tuning(default=True)
    again, ms2 = ctx.autotune(psis, p=0.0, preconditioner="dct", precision="mixed",
                              probe_iters=8, cache_path=cache)
    assert ms2 == 0.0 and again == best == ctx.tuning()
    # the tuned context still solves to the tolerance
    phis, rc, stats = ctx.batch(psis, p=0.0, preconditioner="dct", precision="mixed", k_max=2,
                                outer_tol=0.0)
    assert all(s["final_relres"] <= 1e-6 for s in stats)
