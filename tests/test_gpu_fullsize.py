"""Parity at the workloads' full sizes: the 1024 x 1024 peaks map, the
2048 x 2048 Gaussian map with a zero-quality hole, the 256-map uneven batch
and the 4096 x 4096 ramp, where the oracle cannot run Algorithm 1 end to end
in seconds.  Checked instead, through the C ABI:

* the linear-system property of the returned phase: after one outer step from
  phi0 = 0 the FP64 residual ||b - A phi|| / ||b|| of Eq. (7), with A and b
  assembled by the oracle from its own FP64 weights, meets the tolerance;
* exact recovery (up to a constant) of noise-free phase whose neighbour
  differences stay below pi, after one outer step;
* the DCT preconditioner against the oracle's FP64 transform at full size;
* sampled maps of the full batch against the oracle run on those maps alone.

Residual bounds: the FP64 path is held to the tolerance itself.  The mixed
path solves the system with FP32-rounded weights (b and A from the same
rounded weights, so the system is consistent); against the FP64-weight system
the residual moves by about u32 times the relative size of the weighted
misfit, well below 1e-7, so the bound is tol + 2e-7.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2203_13675_amd import synth  # noqa: E402

TOL = 1e-6
TARGET_RAD = 1e-4


@pytest.fixture(scope="module")
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


def demean(a, valid=None):
    if valid is None:
        return a - a.mean()
    out = a - a[valid].mean()
    out[~valid] = 0.0
    return out


def maxdiff(a, b, valid=None):
    return float(np.abs(demean(a, valid) - demean(b, valid)).max())


def relres_bound(precision):
    return TOL * (1 + 1e-9) if precision == "fp64" else TOL + 2e-7


# ---------------------------------------------------------------------------
# 1024 x 1024 peaks (+-60 rad, noise 0.5 rad): every preconditioner, p = 0, 1
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("pc", ["none", "jacobi", "ilu0", "ssor", "dct", "ilu0_rb", "ssor_rb"])
@pytest.mark.parametrize("p", [0.0, 1.0])
def test_peaks1024_system_residual(ctx, oracle, p, pc, precision):
    psi, mask, _ = synth.workload("peaks1024")
    res = ctx.solve(dev(psi), p=p, preconditioner=pc, tol=TOL, precision=precision, k_max=1,
                    outer_tol=0.0)
    phi = host(res.phi)
    rel = oracle.true_relres(psi, None, np.zeros_like(psi), phi, p=p, tau=0.01)
    print("peaks1024 p=%g %s %s: inner iterations %d, relres gpu %.3e oracle-assembled %.3e"
          % (p, pc, precision, res.stats["inner_iters_total"], res.stats["final_relres"], rel))
    assert res.stats["final_relres"] <= TOL
    assert rel <= relres_bound(precision)


@pytest.mark.parametrize("precision,mode,tol", [("fp64", "fp32", 1e-10),
                                                ("mixed", "split_bf16", 1e-7),
                                                ("mixed", "fp16_scaled", 1e-7)])
def test_peaks1024_exact_recovery(ctx, precision, mode, tol):
    """Noise-free 1024^2 peaks at +-60 rad (neighbour differences <= 0.52 rad):
    one outer step returns the field up to a constant."""
    psi, phi_true = synth.peaks_map(1024, 1024, amplitude=60.0, sigma=0.0)
    res = ctx.solve(dev(psi), p=0.0, preconditioner="dct", tol=tol, precision=precision,
                    dct_mode=mode, k_max=1, outer_tol=0.0)
    d = maxdiff(host(res.phi), phi_true)
    print("peaks1024 exact recovery", precision, mode, "max |error|", d)
    assert d <= (1e-6 if precision == "fp64" else TARGET_RAD)


# ---------------------------------------------------------------------------
# 2048 x 2048 Gaussians with a 10 % zero-quality hole, split-bf16 DCT
# ---------------------------------------------------------------------------
def test_gauss2048_hole(ctx, oracle):
    psi, mask, _ = synth.workload("gauss2048_hole")
    res = ctx.solve(dev(psi), dev(mask, torch.float32), p=0.0, preconditioner="dct", tol=TOL,
                    precision="mixed", dct_mode="split_bf16", k_max=1, outer_tol=0.0)
    phi = host(res.phi)
    rel = oracle.true_relres(psi, mask, np.zeros_like(psi), phi, p=0.0, tau=0.01)
    print("gauss2048 hole: inner %d relres %.3e oracle-assembled %.3e"
          % (res.stats["inner_iters_total"], res.stats["final_relres"], rel))
    assert rel <= relres_bound("mixed")
    # pixels inside the hole have no weighted edge: they keep phi0 = 0
    dx, dy = oracle.wrapped_differences(psi)
    wx, wy = oracle.edge_quality(mask, *psi.shape)
    U, V = oracle.irls_weights(np.zeros_like(psi), dx, dy, wx, wy, 0.0, 0.01)
    iso = oracle.isolated_pixels(U, V)
    assert iso.sum() > 0.09 * psi.size
    assert np.all(phi[iso] == 0.0)


def test_gauss2048_hole_exact_recovery(ctx, oracle):
    """Noise-free Gaussians (differences well below pi): recovered up to a
    constant on every pixel with a weighted edge."""
    _, mask, _ = synth.workload("gauss2048_hole")
    psi, phi_true = synth.gaussians_map(2048, 2048, sigma=0.0, seed=2000)
    res = ctx.solve(dev(psi), dev(mask, torch.float32), p=0.0, preconditioner="dct", tol=1e-7,
                    precision="mixed", dct_mode="split_bf16", k_max=1, outer_tol=0.0)
    dx, dy = oracle.wrapped_differences(psi)
    wx, wy = oracle.edge_quality(mask, *psi.shape)
    U, V = oracle.irls_weights(np.zeros_like(psi), dx, dy, wx, wy, 0.0, 0.01)
    valid = ~oracle.isolated_pixels(U, V)
    d = maxdiff(host(res.phi), phi_true, valid)
    print("gauss2048 hole exact recovery: max |error| on valid pixels", d)
    assert d <= TARGET_RAD


# ---------------------------------------------------------------------------
# The 256-map uneven batch: every map converged, sampled maps vs the oracle
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["split_bf16", "fp16_scaled"])
def test_batch256_sampled_maps(ctx, oracle, mode):
    shapes = synth.batch_sizes(256, seed=3000)
    maps = synth.batch_maps(256, seed=3000)
    psis = [dev(p) for p, _ in maps]
    phis, rc, stats = ctx.batch(psis, p=0.0, eps=0.01, preconditioner="dct", tol=TOL,
                                precision="mixed", dct_mode=mode, k_max=10, outer_tol=0.0)
    assert rc in (0, 1)
    assert max(s["final_relres"] for s in stats) <= TOL
    assert all(s["outer_iters"] == 10 for s in stats)
    # the three smallest maps, each against the oracle on that map alone
    order = sorted(range(256), key=lambda k: (shapes[k][0] * shapes[k][1], k))[:3]
    for k in order:
        p = maps[k][0]
        ex = oracle.unwrap_exact(p, p=0.0, outer=10)
        same_tol = oracle.unwrap(p, p=0.0, precond="dct", tol=TOL, k_max=10, outer_tol=0.0)
        d = maxdiff(host(phis[k]), ex.phi)
        d_orc = maxdiff(same_tol.phi, ex.phi)
        print("batch256", mode, "map", k, shapes[k], "maxdiff vs exact", d, "oracle", d_orc)
        assert d <= max(3.0 * d_orc, TARGET_RAD)


# ---------------------------------------------------------------------------
# 4096 x 4096 peaks + ramp, fp16-scaled DCT
# ---------------------------------------------------------------------------
def test_ramp4096_system_residual(ctx, oracle):
    psi, _, _ = synth.workload("ramp4096")
    res = ctx.solve(dev(psi), p=0.0, preconditioner="dct", tol=TOL, precision="mixed",
                    dct_mode="fp16_scaled", k_max=1, outer_tol=0.0)
    phi = host(res.phi)
    rel = oracle.true_relres(psi, None, np.zeros_like(psi), phi, p=0.0, tau=0.01)
    print("ramp4096: inner %d refinements %d relres %.3e oracle-assembled %.3e"
          % (res.stats["inner_iters_total"], res.stats["refinements"], res.stats["final_relres"], rel))
    assert rel <= relres_bound("mixed")


def test_ramp4096_exact_recovery(ctx):
    psi, phi_true = synth.ramp_peaks_map(4096, 4096, sigma=0.0, seed=4000)
    res = ctx.solve(dev(psi), p=0.0, preconditioner="dct", tol=1e-7, precision="mixed",
                    dct_mode="fp16_scaled", k_max=1, outer_tol=0.0)
    d = maxdiff(host(res.phi), phi_true)
    print("ramp4096 exact recovery: max |error|", d)
    assert d <= TARGET_RAD


# ---------------------------------------------------------------------------
# DCT preconditioner at full size (even/odd MFMA kernels) vs the FP64 transform
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,mode,rel", [(1024, "split_bf16", 2e-4), (1024, "fp16_scaled", 1e-2),
                                        (4096, "fp16_scaled", 1e-2)])
def test_dct_fullsize(ctx, oracle, n, mode, rel):
    rng = np.random.default_rng(n)
    U = np.ones((n, n))
    V = np.ones((n, n))
    U[:, -1] = 0.0
    V[-1, :] = 0.0
    r = rng.standard_normal((n, n)).astype(np.float32).astype(np.float64)
    r -= r.mean()
    ref = oracle.Preconditioner("dct", U, V).apply(r)
    s = host(ctx.precond_apply(dev(U, torch.float32), dev(V, torch.float32), dev(r, torch.float32),
                               "dct", precision="mixed", dct_mode=mode))
    err = np.abs(s - ref).max() / np.abs(ref).max()
    print("dct", n, mode, "max rel error", err)
    assert err <= rel
