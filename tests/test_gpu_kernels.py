"""Kernel-level parity: each HIP step against the oracle's same step, element by
element, through the C ABI.  Sizes span several 64x4 stencil tiles, several
64x64 DCT tiles and ragged tails.

Tolerances (derived from the arithmetic):
* wrapped differences: bit-exact (both sides evaluate the same FP64 formula,
  no contraction).
* FP64 elementwise results: |gpu - oracle| <= 16 u64 S, S the same sum taken
  over absolute values (rounding order differs, fused multiply-adds).
* FP32 results against the oracle evaluated in FP64 on the same FP32 inputs:
  |gpu - oracle| <= 16 u32 S.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U64 = 2.0 ** -53
U32 = 2.0 ** -24
SIZES = [(64, 64), (37, 53), (130, 77), (1, 40), (40, 1), (5, 300)]


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


def weights_case(O, M, N, seed, p=0.0, mask=None):
    rng = np.random.default_rng(seed)
    psi = rng.uniform(-np.pi, np.pi, (M, N))
    phi = rng.normal(0, 2.0, (M, N))
    dx, dy = O.wrapped_differences(psi)
    wx, wy = O.edge_quality(mask, M, N)
    U, V = O.irls_weights(phi, dx, dy, wx, wy, p, 0.01)
    return psi, phi, dx, dy, U, V


def abs_stencil(O, U, V, x):
    """|A| |x| -- the scale of each entry of A x."""
    sh = O._shift
    ax = np.abs(x)
    return (O.diag_A(U, V) * ax + sh(ax, 0, 1) * U + sh(ax, 1, 0) * V
            + sh(ax, 0, -1) * sh(U, 0, -1) + sh(ax, -1, 0) * sh(V, -1, 0))


@pytest.mark.parametrize("M,N", SIZES)
def test_wrapped_differences_bit_exact(ctx, oracle, M, N):
    rng = np.random.default_rng(M * 1000 + N)
    psi = rng.uniform(-np.pi, np.pi, (M, N))
    # plant exact ties W(+-pi) and differences near the boundary
    if N > 3:
        psi[0, 0], psi[0, 1] = 0.0, np.pi
        psi[0, 2] = -np.pi + 1e-15
    dx, dy = ctx.wrapped_differences(dev(psi))
    ex, ey = oracle.wrapped_differences(psi)
    assert np.array_equal(host(dx), ex)
    assert np.array_equal(host(dy), ey)


@pytest.mark.parametrize("M,N", SIZES)
@pytest.mark.parametrize("p", [0.0, 1.0, 1.3, 2.0])
def test_weights(ctx, oracle, M, N, p):
    psi, phi, dx, dy, U, V = weights_case(oracle, M, N, 7, p)
    mask = (np.random.default_rng(8).uniform(size=(M, N)) > 0.2).astype(np.float32)
    mask *= np.random.default_rng(9).uniform(0.2, 1.0, size=(M, N)).astype(np.float32)
    wx, wy = oracle.edge_quality(mask, M, N)
    Um, Vm = oracle.irls_weights(phi, dx, dy, wx, wy, p, 0.01)
    for prec, tol in (("fp64", 8 * U64), ("mixed", 2 * U32)):
        Ug, Vg = ctx.weights(dev(phi), dev(dx), dev(dy), None, p=p, tau=0.01, precision=prec)
        assert np.allclose(host(Ug), U, rtol=tol, atol=0)
        assert np.allclose(host(Vg), V, rtol=tol, atol=0)
        Ug, Vg = ctx.weights(dev(phi), dev(dx), dev(dy), dev(mask, torch.float32), p=p, tau=0.01,
                             precision=prec)
        assert np.allclose(host(Ug), Um, rtol=tol, atol=0)
        assert np.allclose(host(Vg), Vm, rtol=tol, atol=0)


@pytest.mark.parametrize("M,N", SIZES)
def test_apply_A(ctx, oracle, M, N):
    psi, phi, dx, dy, U, V = weights_case(oracle, M, N, 11)
    x = np.random.default_rng(12).normal(size=(M, N))
    ref = oracle.apply_A(U, V, x)
    S = abs_stencil(oracle, U, V, x)
    y = host(ctx.apply_A(dev(U), dev(V), dev(x), "fp64"))
    assert np.all(np.abs(y - ref) <= 16 * U64 * S)
    U32_, V32_, x32 = (a.astype(np.float32) for a in (U, V, x))
    ref32 = oracle.apply_A(U32_.astype(np.float64), V32_.astype(np.float64), x32.astype(np.float64))
    y32 = host(ctx.apply_A(dev(U32_, torch.float32), dev(V32_, torch.float32),
                           dev(x32, torch.float32), "mixed"))
    assert np.all(np.abs(y32 - ref32) <= 16 * U32 * S + 1e-30)


@pytest.mark.parametrize("M,N", SIZES)
def test_rhs(ctx, oracle, M, N):
    psi, phi, dx, dy, U, V = weights_case(oracle, M, N, 13)
    ref = oracle.rhs(U, V, dx, dy)
    S = abs_stencil(oracle, U, V, np.maximum(np.abs(dx), np.abs(dy)))
    b = host(ctx.rhs(dev(U), dev(V), dev(dx), dev(dy), "fp64"))
    assert np.all(np.abs(b - ref) <= 16 * U64 * S)


@pytest.mark.parametrize("M,N", [(64, 64), (37, 53), (130, 77), (1, 40), (40, 1), (200, 150)])
def test_ilu_pivots(ctx, oracle, M, N):
    psi, phi, dx, dy, U, V = weights_case(oracle, M, N, 17)
    ref = oracle.Preconditioner("ilu0", U, V).pivots()
    piv = host(ctx.ilu_pivots(dev(U), dev(V), "fp64"))
    assert np.allclose(piv, ref, rtol=1e-12, atol=0)
    # FP32: a one-dimensional chain's pivots shrink towards zero (the exact
    # factorization of a path graph is singular), which amplifies rounding; 2-D
    # pivots stay well away from zero.
    piv32 = host(ctx.ilu_pivots(dev(U, torch.float32), dev(V, torch.float32), "mixed"))
    assert np.allclose(piv32, ref, rtol=1e-4 if min(M, N) > 1 else 2e-3, atol=0)


def _precond_case(oracle, M, N, seed, hole):
    psi, phi, dx, dy, U, V = weights_case(oracle, M, N, seed)
    if hole and M > 8 and N > 8:
        mask = np.ones((M, N), dtype=np.float32)
        mask[M // 4:M // 2, N // 3:N // 2] = 0
        wx, wy = oracle.edge_quality(mask, M, N)
        U, V = oracle.irls_weights(phi, dx, dy, wx, wy, 0.0, 0.01)
    r = np.random.default_rng(seed + 1).normal(size=(M, N))
    r[oracle.isolated_pixels(U, V)] = 0.0
    return U, V, r


PC_SIZES = [(64, 64), (37, 53), (130, 77), (1, 40), (40, 1), (96, 160)]


@pytest.mark.parametrize("pc", ["none", "jacobi", "ilu0", "ic0", "ssor", "dct",
                                "ilu0_rb", "ic0_rb", "ssor_rb"])
@pytest.mark.parametrize("M,N", PC_SIZES)
@pytest.mark.parametrize("hole", [False, True])
def test_precond_fp64(ctx, oracle, pc, M, N, hole):
    U, V, r = _precond_case(oracle, M, N, 21, hole)
    for omega in ((1.0, 1.5) if pc in ("ssor", "ssor_rb") else (1.0,)):
        ref = oracle.Preconditioner(pc, U, V, omega=omega).apply(r)
        s = host(ctx.precond_apply(dev(U), dev(V), dev(r), pc, precision="fp64", omega=omega))
        scale = np.abs(ref).max() + 1e-300
        assert np.abs(s - ref).max() <= 1e-10 * scale, (pc, omega, np.abs(s - ref).max() / scale)


@pytest.mark.parametrize("pc,mode,rel", [("none", "fp32", 0.0), ("jacobi", "fp32", 4 * U32),
                                         ("ilu0", "fp32", 2e-4), ("ic0", "fp32", 2e-4),
                                         ("ssor", "fp32", 2e-4), ("dct", "fp32", 1e-4),
                                         ("dct", "split_bf16", 2e-4),
                                         ("dct", "fp16_scaled", 1e-2),
                                         # two explicit passes of a few FP32 terms each
                                         ("ilu0_rb", "fp32", 2e-5), ("ic0_rb", "fp32", 2e-5),
                                         ("ssor_rb", "fp32", 2e-5)])
@pytest.mark.parametrize("M,N", PC_SIZES)
@pytest.mark.parametrize("hole", [False, True])
def test_precond_mixed(ctx, oracle, pc, mode, rel, M, N, hole):
    U, V, r = _precond_case(oracle, M, N, 31, hole)
    U32_, V32_, r32 = (a.astype(np.float32).astype(np.float64) for a in (U, V, r))
    ref = oracle.Preconditioner(pc, U32_, V32_).apply(r32)
    s = host(ctx.precond_apply(dev(U32_, torch.float32), dev(V32_, torch.float32),
                               dev(r32, torch.float32), pc, precision="mixed", dct_mode=mode))
    scale = np.abs(ref).max() + 1e-300
    err = np.abs(s - ref).max() / scale
    assert err <= rel, (pc, mode, err)


@pytest.mark.parametrize("mode,rel", [("split_bf16", 2e-4), ("fp16_scaled", 1e-2)])
@pytest.mark.parametrize("M,N", [(128, 128), (128, 384), (256, 128), (384, 256)])
@pytest.mark.parametrize("hole", [False, True])
def test_precond_dct_even_odd(ctx, oracle, mode, rel, M, N, hole):
    """Sides that are multiples of 128 take the even/odd MFMA kernels (spectra
    in split order): same result as the dense definition."""
    U, V, r = _precond_case(oracle, M, N, 41, hole)
    U32_, V32_, r32 = (a.astype(np.float32).astype(np.float64) for a in (U, V, r))
    ref = oracle.Preconditioner("dct", U32_, V32_).apply(r32)
    s = host(ctx.precond_apply(dev(U32_, torch.float32), dev(V32_, torch.float32),
                               dev(r32, torch.float32), "dct", precision="mixed", dct_mode=mode))
    err = np.abs(s - ref).max() / np.abs(ref).max()
    assert err <= rel, (mode, M, N, err)


def test_mfma_operand_layout(ctx, oracle):
    """A DCT stage contraction on a structured input whose every output element
    depends on a distinct (row, column) pair: a wrong MFMA lane mapping would
    permute rows or columns and fail the comparison at split-bf16 accuracy."""
    M, N = 64, 96
    U = np.ones((M, N))
    V = np.ones((M, N))
    U[:, -1] = 0
    V[-1, :] = 0
    i = np.arange(M)[:, None]
    j = np.arange(N)[None, :]
    r = np.sin(0.37 * i + 0.11 * j * j) + 0.01 * i - 0.02 * j
    r -= r.mean()
    ref = oracle.Preconditioner("dct", U, V).apply(r)
    s = host(ctx.precond_apply(dev(U, torch.float32), dev(V, torch.float32), dev(r, torch.float32),
                               "dct", precision="mixed", dct_mode="split_bf16"))
    assert np.abs(s - ref).max() <= 2e-4 * np.abs(ref).max()
