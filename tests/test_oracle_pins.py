"""Pins for the FP64 oracle: each check ties it to something other than itself
(values the paper prints, closed forms, library routines, brute force on tiny
inputs, invariants).  CPU only.

Each pin is a function returning True/False so that the mutation tests at the
bottom can plant a plausible mistake in the oracle and show that some pin
catches it.
"""
import math

import numpy as np
import pytest
import scipy.fft
import scipy.sparse
import scipy.sparse.linalg

from conftest import read_golden
from paper_2203_13675_amd import synth

TAU = 0.01


# ---------------------------------------------------------------------------
# helpers written independently of the oracle
# ---------------------------------------------------------------------------
def edge_list(M, N):
    """Every in-grid neighbour pair: ('x', i, j) joins (i,j)-(i,j+1); ('y', i, j) joins (i,j)-(i+1,j)."""
    e = [("x", i, j) for i in range(M) for j in range(N - 1)]
    e += [("y", i, j) for i in range(M - 1) for j in range(N)]
    return e


def incidence(M, N):
    """Forward-difference matrix D (edges x pixels): (D phi)_e = phi_head - phi_tail."""
    E = edge_list(M, N)
    D = np.zeros((len(E), M * N))
    for k, (ax, i, j) in enumerate(E):
        a = i * N + j
        b = a + 1 if ax == "x" else a + N
        D[k, a] = -1.0
        D[k, b] = 1.0
    return D, E


def edge_values(E, X, Y):
    return np.array([X[i, j] if ax == "x" else Y[i, j] for ax, i, j in E])


def random_weights(M, N, rng, lo=0.05, hi=1.0):
    U = rng.uniform(lo, hi, (M, N))
    V = rng.uniform(lo, hi, (M, N))
    U[:, N - 1] = 0.0
    V[M - 1, :] = 0.0
    return U, V


def noisy_peaks(M, N, scale, sigma, seed):
    psi, phi = synth.peaks_map(M, N, scale=scale, sigma=sigma, seed=seed)
    return psi, phi


# ---------------------------------------------------------------------------
# pins as predicates
# ---------------------------------------------------------------------------
def pin_wrap_range_and_ties(O):
    """Eq. (1): W(x) - x is a multiple of 2 pi and W(x) lies in (-pi, pi]; ties go to +pi."""
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-2 * np.pi + 1e-9, 2 * np.pi - 1e-9, 10000),
                        [np.pi, -np.pi, 0.0, 3.0, -3.0]])
    w = O.wrap(x)
    k = (w - x) / (2 * np.pi)
    ok = np.all(np.abs(k - np.round(k)) < 1e-12)
    ok &= np.all(w > -np.pi) and np.all(w <= np.pi)
    ok &= O.wrap(np.pi) == np.pi and O.wrap(-np.pi) == np.pi
    # inside the principal range W is the identity
    y = rng.uniform(-3.1, 3.1, 1000)
    ok &= np.array_equal(O.wrap(y), y)
    # agrees with the complex-argument definition away from the tie
    ok &= np.allclose(O.wrap(x[:10000]), np.angle(np.exp(1j * x[:10000])), atol=1e-12)
    return bool(ok)


def pin_wrapped_differences(O):
    """Delta^x, Delta^y of Section 2.1 against the complex-argument wrap of each difference."""
    rng = np.random.default_rng(2)
    psi = rng.uniform(-np.pi, np.pi, (9, 11))
    dx, dy = O.wrapped_differences(psi)
    ex = np.angle(np.exp(1j * (psi[:, 1:] - psi[:, :-1])))
    ey = np.angle(np.exp(1j * (psi[1:, :] - psi[:-1, :])))
    return bool(np.allclose(dx[:, :-1], ex, atol=1e-12) and np.allclose(dy[:-1, :], ey, atol=1e-12)
                and dx.shape == psi.shape and dy.shape == psi.shape)


def pin_weights_hand_values(O):
    """Eq. (6) at hand-computed points (tau = 0.01)."""
    M, N = 2, 2
    dx = np.zeros((M, N))
    dy = np.zeros((M, N))
    wx, wy = O.edge_quality(None, M, N)
    # phi with horizontal differences 0.1 (row 0) and 0 (row 1); vertical 0.3, 0.2
    phi = np.array([[0.0, 0.1], [0.3, 0.3 + 0.0 - 0.1 + 0.1]])
    phi[1, 1] = phi[0, 1] + 0.2  # vertical difference at column 1 is 0.2
    rx0 = 0.1
    rx1 = phi[1, 1] - phi[1, 0]
    ok = True
    # p = 0: tau / (r^2 + tau)
    U, V = O.irls_weights(phi, dx, dy, wx, wy, 0.0, TAU)
    ok &= math.isclose(U[0, 0], 0.5, rel_tol=1e-12)                       # 0.01/(0.01+0.01)
    ok &= math.isclose(U[1, 0], TAU / (rx1 * rx1 + TAU), rel_tol=1e-12)
    ok &= math.isclose(V[0, 0], 0.01 / (0.09 + 0.01), rel_tol=1e-12)      # 0.1
    ok &= math.isclose(V[0, 1], 0.01 / (0.04 + 0.01), rel_tol=1e-12)      # 0.2
    # p = 1: tau / (|r| + tau); r = 0.3 -> 1/31
    U1, V1 = O.irls_weights(phi, dx, dy, wx, wy, 1.0, TAU)
    ok &= math.isclose(V1[0, 0], 1.0 / 31.0, rel_tol=1e-12)
    ok &= math.isclose(U1[0, 0], 0.01 / 0.11, rel_tol=1e-12)
    # p = 2: constant tau / (1 + tau)
    U2, V2 = O.irls_weights(phi, dx, dy, wx, wy, 2.0, TAU)
    ok &= math.isclose(U2[0, 0], TAU / (1 + TAU), rel_tol=1e-14)
    # p = 1.5 at r = 0.25: |r|^0.5 = 0.5 -> 0.01/0.51
    phi15 = np.array([[0.0, 0.25], [0.0, 0.25]])
    U15, _ = O.irls_weights(phi15, dx, dy, wx, wy, 1.5, TAU)
    ok &= math.isclose(U15[0, 0], 0.01 / 0.51, rel_tol=1e-12)
    # zero residual -> weight 1 for p < 2
    Uz, Vz = O.irls_weights(np.zeros((M, N)), dx, dy, wx, wy, 0.0, TAU)
    ok &= Uz[0, 0] == 1.0 and Vz[0, 0] == 1.0
    # zero-flux boundary
    ok &= np.all(U[:, -1] == 0) and np.all(V[-1, :] == 0)
    _ = rx0
    return bool(ok)


def pin_normal_equations(O):
    """Eq. (7) is the normal equation of the weighted least-squares problem
    min sum_e w_e (phi_head - phi_tail - Delta_e)^2: A = D^T W D, b = D^T W Delta."""
    rng = np.random.default_rng(3)
    M, N = 6, 7
    U, V = random_weights(M, N, rng)
    dx = rng.uniform(-np.pi, np.pi, (M, N))
    dy = rng.uniform(-np.pi, np.pi, (M, N))
    D, E = incidence(M, N)
    w = edge_values(E, U, V)
    delta = edge_values(E, dx, dy)
    A_ref = D.T @ (w[:, None] * D)
    b_ref = D.T @ (w * delta)
    x = rng.normal(size=(M, N))
    ok = np.allclose(O.apply_A(U, V, x).ravel(), A_ref @ x.ravel(), atol=1e-12)
    ok &= np.allclose(O.rhs(U, V, dx, dy).ravel(), b_ref, atol=1e-12)
    rowptr, col, a = O.assemble_csr(U, V)
    A_csr = scipy.sparse.csr_matrix((a, col, rowptr), shape=(M * N, M * N)).toarray()
    ok &= np.allclose(A_csr, A_ref, atol=1e-14)
    ok &= np.allclose(O.diag_A(U, V).ravel(), np.diag(A_ref), atol=1e-14)
    return bool(ok)


def pin_gradient_of_energy(O):
    """A phi - b is half the gradient of the quadratic energy sum_e w_e (D phi - Delta)_e^2
    (central differences are exact for a quadratic up to rounding)."""
    rng = np.random.default_rng(4)
    M, N = 4, 5
    U, V = random_weights(M, N, rng)
    dx = rng.uniform(-3, 3, (M, N))
    dy = rng.uniform(-3, 3, (M, N))
    phi = rng.normal(size=(M, N))

    def energy(f):
        rx = f[:, 1:] - f[:, :-1] - dx[:, :-1]
        ry = f[1:, :] - f[:-1, :] - dy[:-1, :]
        return np.sum(U[:, :-1] * rx * rx) + np.sum(V[:-1, :] * ry * ry)

    g = np.zeros((M, N))
    h = 1e-3
    for i in range(M):
        for j in range(N):
            e = np.zeros((M, N))
            e[i, j] = h
            g[i, j] = (energy(phi + e) - energy(phi - e)) / (2 * h)
    lhs = O.apply_A(U, V, phi) - O.rhs(U, V, dx, dy)
    return bool(np.allclose(lhs, 0.5 * g, atol=1e-9))


def pin_table1_structure(O):
    """Table 1: the nonzero count of A for every image size, and its density."""
    ok = True
    for scale, w, h, nnz, dens in read_golden("table1_matrix_sizes.txt"):
        N, M = int(w), int(h)
        rng = np.random.default_rng(5)
        U, V = random_weights(M, N, rng)
        rowptr, col, a = O.assemble_csr(U, V)
        ok &= int(rowptr[-1]) == int(nnz)
        d = int(nnz) / float(M * N) ** 2 * 100
        if scale != "0.25":                      # the first row's density is a misprint
            ok &= math.floor(d * 1e4) / 1e4 == float(dens)
    return bool(ok)


def pin_laplacian_properties(O):
    """A symmetric, A 1 = 0, A positive semidefinite (so -A, the discrete
    divergence of the weighted gradient, is negative semidefinite)."""
    rng = np.random.default_rng(6)
    M, N = 7, 6
    U, V = random_weights(M, N, rng)
    rowptr, col, a = O.assemble_csr(U, V)
    A = scipy.sparse.csr_matrix((a, col, rowptr), shape=(M * N, M * N)).toarray()
    ok = np.allclose(A, A.T, atol=0)
    ok &= np.allclose(O.apply_A(U, V, np.ones((M, N))), 0.0, atol=1e-14)
    ev = np.linalg.eigvalsh(A)
    ok &= ev.min() > -1e-12 and np.sum(ev < 1e-10) == 1     # connected grid: one zero mode
    ok &= np.linalg.eigvalsh(-A).max() < 1e-12
    return bool(ok)


def pin_dense_lstsq(O):
    """One inner system solved by PCG equals the dense weighted least-squares solution."""
    M, N = 12, 10
    psi, _ = noisy_peaks(M, N, 4.0, 0.3, 7)
    dx, dy = O.wrapped_differences(psi)
    wx, wy = O.edge_quality(None, M, N)
    rng = np.random.default_rng(7)
    phi_k = rng.normal(size=(M, N))
    U, V = O.irls_weights(phi_k, dx, dy, wx, wy, 0.0, TAU)
    D, E = incidence(M, N)
    sw = np.sqrt(edge_values(E, U, V))
    ref = np.linalg.lstsq(sw[:, None] * D, sw * edge_values(E, dx, dy), rcond=None)[0]
    ok = True
    for pc in ("none", "jacobi", "ilu0", "ic0", "ssor", "dct"):
        P = O.Preconditioner(pc, U, V)
        b = O.rhs(U, V, dx, dy)
        res = O.pcg(U, V, b, phi_k, P, tol=1e-13)
        x = res.x.ravel()
        ok &= np.allclose(x - x.mean(), ref - ref.mean(), atol=1e-9)
    return bool(ok)


def pin_scipy_cg(O):
    """Plain CG (M = I) reaches the same solution as scipy's CG on the assembled matrix."""
    M, N = 24, 20
    psi, _ = noisy_peaks(M, N, 4.0, 0.3, 8)
    dx, dy = O.wrapped_differences(psi)
    wx, wy = O.edge_quality(None, M, N)
    U, V = O.irls_weights(np.zeros((M, N)), dx, dy, wx, wy, 1.0, TAU)
    b = O.rhs(U, V, dx, dy)
    rowptr, col, a = O.assemble_csr(U, V)
    A = scipy.sparse.csr_matrix((a, col, rowptr), shape=(M * N, M * N))
    xs, info = scipy.sparse.linalg.cg(A, b.ravel(), rtol=1e-13, atol=0.0, maxiter=20000)
    res = O.pcg(U, V, b, np.zeros((M, N)), O.Preconditioner("none", U, V), tol=1e-13)
    x = res.x.ravel()
    return bool(info == 0 and np.allclose(x - x.mean(), xs - xs.mean(), atol=1e-8))


def pin_exact_recovery(O):
    """Noise-free phase whose neighbour differences stay below pi: Delta = D phi exactly,
    so one outer step with an exact inner solve returns phi + const for any p
    (with a mask: on the connected valid region; isolated pixels keep phi0 = 0)."""
    M, N = 40, 48
    phi = synth.peaks(M, N) * 0.8 + np.linspace(0, 6, N)[None, :]
    assert np.abs(np.diff(phi, axis=0)).max() < np.pi and np.abs(np.diff(phi, axis=1)).max() < np.pi
    psi = synth.wrap_measurement(phi)
    ok = True
    for p in (0.0, 1.0, 1.5, 2.0):
        for pc in ("none", "ilu0", "dct"):
            r = O.unwrap(psi, p=p, precond=pc, tol=1e-12, k_max=1, outer_tol=0.0)
            e = r.phi - phi
            ok &= np.ptp(e) < 1e-7
    mask = np.ones((M, N), dtype=np.float32)
    mask[10:20, 15:30] = 0.0
    r = O.unwrap(psi, mask, p=0.0, precond="ilu0", tol=1e-12, k_max=1, outer_tol=0.0)
    valid = mask > 0
    e = r.phi - phi
    ok &= np.ptp(e[valid]) < 1e-7
    ok &= np.all(r.phi[~valid] == 0.0)
    return bool(ok)


def pin_p2_dct_one_step(O):
    """p = 2: U = V = tau/(1+tau) everywhere, so A is a multiple of the unit Neumann
    Laplacian and the DCT-preconditioned CG finishes in one iteration."""
    M, N = 32, 24
    psi, _ = noisy_peaks(M, N, 4.0, 0.3, 9)
    dx, dy = O.wrapped_differences(psi)
    wx, wy = O.edge_quality(None, M, N)
    U, V = O.irls_weights(np.zeros((M, N)), dx, dy, wx, wy, 2.0, TAU)
    ok = np.allclose(U[:, :-1], TAU / (1 + TAU)) and np.allclose(V[:-1, :], TAU / (1 + TAU))
    b = O.rhs(U, V, dx, dy)
    res = O.pcg(U, V, b, np.zeros((M, N)), O.Preconditioner("dct", U, V), tol=1e-11, record=True)
    ok &= res.iters == 1 and res.relres < 1e-12
    return bool(ok)


def pin_dct_against_library(O):
    """The orthonormal DCT-II matrix equals scipy's DCT-II (norm='ortho'); the
    eigenvalues of the unit Neumann Laplacian are those of its DCT basis; the DCT
    preconditioner inverts the unit Laplacian on the zero-mean subspace."""
    ok = True
    for n in (1, 2, 7, 64, 384):
        C = O.dct_matrix(n)
        ok &= np.allclose(C, scipy.fft.dct(np.eye(n), type=2, norm="ortho", axis=0), atol=1e-13)
    M, N = 9, 13
    one = np.ones((M, N))
    U = one.copy()
    V = one.copy()
    U[:, -1] = 0
    V[-1, :] = 0
    lam = O.neumann_eigenvalues(M, N)
    CM, CN = O.dct_matrix(M), O.dct_matrix(N)
    for (k, l) in ((0, 0), (1, 0), (0, 5), (4, 7), (8, 12)):
        basis = np.outer(CM[k], CN[l])
        ok &= np.allclose(O.apply_A(U, V, basis), lam[k, l] * basis, atol=1e-12)
    rng = np.random.default_rng(10)
    r = rng.normal(size=(M, N))
    P = O.Preconditioner("dct", U, V)
    s = P.apply(r)
    ok &= np.allclose(O.apply_A(U, V, s), r - r.mean(), atol=1e-12)
    s2 = scipy.fft.idctn(scipy.fft.dctn(r, norm="ortho") * P.inv_lam, norm="ortho")
    ok &= np.allclose(s, s2, atol=1e-12)
    return bool(ok)


def _dense_pattern(M, N):
    D, _ = incidence(M, N)
    return (np.abs(D.T @ D) > 0)


def _dense_ilu0(A, P):
    """KIJ Gaussian elimination with every update outside the pattern P dropped."""
    n = len(A)
    LU = A.copy()
    for k in range(n):
        for i in range(k + 1, n):
            if P[i, k]:
                LU[i, k] /= LU[k, k]
                for j in range(k + 1, n):
                    if P[i, j]:
                        LU[i, j] -= LU[i, k] * LU[k, j]
    L = np.tril(LU, -1) + np.eye(n)
    Uu = np.triu(LU)
    return L, Uu


def _dense_ic0(A, P):
    """Column Cholesky with the factor restricted to the lower pattern P."""
    n = len(A)
    L = np.zeros_like(A)
    for k in range(n):
        L[k, k] = math.sqrt(A[k, k] - np.sum(L[k, :k] ** 2))
        for i in range(k + 1, n):
            if P[i, k]:
                L[i, k] = (A[i, k] - np.sum(L[i, :k] * L[k, :k])) / L[k, k]
    return L


def pin_incomplete_factorizations(O):
    """ILU(0), IC(0) and SSOR against brute-force dense versions on a 5x7 grid with
    random positive weights; the no-fill factors reproduce A on its pattern; and for
    this symmetric five-point matrix ILU(0) and IC(0) give the same preconditioner."""
    rng = np.random.default_rng(11)
    M, N = 5, 7
    U, V = random_weights(M, N, rng)
    rowptr, col, a = O.assemble_csr(U, V)
    A = scipy.sparse.csr_matrix((a, col, rowptr), shape=(M * N, M * N)).toarray()
    P = _dense_pattern(M, N)
    r = rng.normal(size=(M, N))
    ok = True
    L, Uu = _dense_ilu0(A, P)
    ok &= np.allclose((L @ Uu)[P], A[P], atol=1e-13)
    s_ilu = O.Preconditioner("ilu0", U, V).apply(r)
    ok &= np.allclose(s_ilu.ravel(), np.linalg.solve(L @ Uu, r.ravel()), atol=1e-12)
    Lc = _dense_ic0(A, P)
    ok &= np.allclose((Lc @ Lc.T)[P], A[P], atol=1e-13)
    s_ic = O.Preconditioner("ic0", U, V).apply(r)
    ok &= np.allclose(s_ic.ravel(), np.linalg.solve(Lc @ Lc.T, r.ravel()), atol=1e-12)
    ok &= np.allclose(s_ilu, s_ic, atol=1e-12)
    ok &= np.allclose(O.Preconditioner("ilu0", U, V).pivots().ravel(), np.diag(Uu), atol=1e-13)
    Dd = np.diag(np.diag(A))
    Ls = np.tril(A, -1)
    for w in (1.0, 1.4):
        Ms = (Dd / w + Ls) @ np.linalg.inv(Dd / w) @ (Dd / w + Ls.T) / (2.0 - w)
        s = O.Preconditioner("ssor", U, V, omega=w).apply(r)
        ok &= np.allclose(s.ravel(), np.linalg.solve(Ms, r.ravel()), atol=1e-12)
    return bool(ok)


def pin_red_black_factorizations(O):
    """ILU(0), IC(0) and SSOR of the matrix taken in red-black order (i + j even
    first): the ordering puts every even-parity pixel before every odd one and
    keeps row-major order inside each colour; the no-fill factor of P A P^T
    (brute-force dense elimination on the permuted pattern) reproduces P A P^T on
    its pattern and is what the oracle applies; its pivots have the closed form
    of a two-colour ordering (even pixels: the diagonal; odd pixels: the diagonal
    minus the squared couplings to their even neighbours over those neighbours'
    diagonals); IC(0) gives the same preconditioner; SSOR matches its matrix
    formula in the permuted order."""
    rng = np.random.default_rng(19)
    M, N = 5, 7
    U, V = random_weights(M, N, rng)
    rowptr, col, a = O.assemble_csr(U, V)
    A = scipy.sparse.csr_matrix((a, col, rowptr), shape=(M * N, M * N)).toarray()
    P = _dense_pattern(M, N)
    r = rng.normal(size=(M, N))
    perm = np.asarray(O.red_black_order(M, N))
    ii, jj = perm // N, perm % N
    nred = (M * N + 1) // 2
    ok = sorted(perm.tolist()) == list(range(M * N))
    ok &= bool(np.all((ii[:nred] + jj[:nred]) % 2 == 0) and np.all((ii[nred:] + jj[nred:]) % 2 == 1))
    ok &= bool(np.all(np.diff(perm[:nred]) > 0) and np.all(np.diff(perm[nred:]) > 0))
    Ap, Pp = A[np.ix_(perm, perm)], P[np.ix_(perm, perm)]
    L, Uu = _dense_ilu0(Ap, Pp)
    ok &= np.allclose((L @ Uu)[Pp], Ap[Pp], atol=1e-13)
    s_ilu = O.Preconditioner("ilu0_rb", U, V).apply(r)
    want = np.empty(M * N)
    want[perm] = np.linalg.solve(L @ Uu, r.ravel()[perm])
    ok &= np.allclose(s_ilu.ravel(), want, atol=1e-12)
    d = np.diag(A)
    piv = d.copy()
    for q in range(M * N):
        if (q // N + q % N) % 2 == 1:
            nb = [t for t in range(M * N) if t != q and A[q, t] != 0.0]
            piv[q] = d[q] - sum(A[q, t] ** 2 / d[t] for t in nb)
    ok &= np.allclose(O.Preconditioner("ilu0_rb", U, V).pivots().ravel(), piv, atol=1e-13)
    s_ic = O.Preconditioner("ic0_rb", U, V).apply(r)
    ok &= np.allclose(s_ilu, s_ic, atol=1e-12)
    Dd = np.diag(np.diag(Ap))
    Ls = np.tril(Ap, -1)
    for w in (1.0, 1.4):
        Ms = (Dd / w + Ls) @ np.linalg.inv(Dd / w) @ (Dd / w + Ls.T) / (2.0 - w)
        s = O.Preconditioner("ssor_rb", U, V, omega=w).apply(r)
        want[perm] = np.linalg.solve(Ms, r.ravel()[perm])
        ok &= np.allclose(s.ravel(), want, atol=1e-12)
    return bool(ok)


def pin_monotone_descent(O):
    """With exact inner solves the outer loop is majorise-minimise for the
    tau-regularised energy, so the energy never increases (p = 0 and p = 1)."""
    M, N = 32, 32
    psi, _ = noisy_peaks(M, N, 4.0, 0.4, 12)
    dx, dy = O.wrapped_differences(psi)
    wx, wy = O.edge_quality(None, M, N)
    ok = True
    for p in (0.0, 1.0):
        r = O.unwrap(psi, p=p, precond="ilu0", tol=1e-12, k_max=8, outer_tol=0.0, keep_history=True)
        Es = [O.objective(np.zeros((M, N)), dx, dy, wx, wy, p, TAU)]
        Es += [O.objective(f, dx, dy, wx, wy, p, TAU) for f in r.history]
        ok &= all(b <= a * (1 + 1e-12) + 1e-14 for a, b in zip(Es, Es[1:]))
        ok &= Es[-1] < Es[0]
    return bool(ok)


def pin_cg_finite_termination(O):
    """CG on a 3x3 grid (8 nonzero eigenvalues) converges in at most 8 steps."""
    rng = np.random.default_rng(13)
    M, N = 3, 3
    U, V = random_weights(M, N, rng)
    b = rng.normal(size=(M, N))
    b -= b.mean()
    res = O.pcg(U, V, b, np.zeros((M, N)), O.Preconditioner("none", U, V), tol=1e-10)
    return bool(res.iters <= 8 and res.relres < 1e-10)


def pin_normalized_error(O):
    """Eq. (8): Q = 0 for equal signals and 1 for opposite ones."""
    rng = np.random.default_rng(14)
    mu = rng.normal(size=(5, 5))
    return bool(O.normalized_error(mu, mu) == 0.0 and math.isclose(O.normalized_error(mu, -mu), 1.0)
                and math.isclose(O.normalized_error(mu, 0 * mu), 1.0))


def pin_dct_fft_path(O):
    """The O(MN log MN) DCT preconditioner equals the dense one (dct_matrix along
    each axis) on grids of odd, even and unequal sides, and at 512 x 384 it
    inverts the unit-weight Neumann Laplacian on zero-mean vectors."""
    rng = np.random.default_rng(30)
    ok = True
    for M, N in ((7, 5), (24, 40), (64, 48), (130, 96)):
        U = np.ones((M, N))
        V = np.ones((M, N))
        U[:, N - 1] = 0.0
        V[M - 1, :] = 0.0
        r = rng.normal(size=(M, N))
        a = O.Preconditioner("dct", U, V, dct_impl="dense").apply(r)
        b = O.Preconditioner("dct", U, V, dct_impl="fft").apply(r)
        ok &= np.allclose(a, b, rtol=0, atol=1e-12 * np.abs(a).max())
    M, N = 512, 384
    U = np.ones((M, N))
    V = np.ones((M, N))
    U[:, N - 1] = 0.0
    V[M - 1, :] = 0.0
    r = rng.normal(size=(M, N))
    r -= r.mean()
    P = O.Preconditioner("dct", U, V)
    ok &= P.dct_impl == "fft"
    s = P.apply(r)
    ok &= np.allclose(O.apply_A(U, V, s), r, rtol=0, atol=1e-10 * np.abs(r).max())
    ok &= abs(s.mean()) < 1e-12
    return bool(ok)


PINS = [pin_wrap_range_and_ties, pin_wrapped_differences, pin_weights_hand_values,
        pin_normal_equations, pin_gradient_of_energy, pin_laplacian_properties,
        pin_dense_lstsq, pin_scipy_cg, pin_exact_recovery, pin_p2_dct_one_step,
        pin_dct_against_library, pin_incomplete_factorizations, pin_red_black_factorizations,
        pin_monotone_descent,
        pin_cg_finite_termination, pin_normalized_error, pin_dct_fft_path]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_pin(oracle, pin):
    assert pin(oracle)


def test_table1_structure(oracle):
    assert pin_table1_structure(oracle)


def test_paper_parameters_are_the_defaults(oracle):
    """Defaults of the oracle's outer loop are the paper's stopping parameters."""
    import inspect
    vals = {k: float(v) for k, v in read_golden("paper_parameters.txt")}
    sig = inspect.signature(oracle.unwrap).parameters
    assert sig["tau"].default == vals["tau"]
    assert sig["k_max"].default == vals["k_max"]
    assert sig["outer_tol"].default == vals["tol"]
    assert sig["eps_cg"].default == vals["eps"]
    psig = inspect.signature(oracle.pcg).parameters
    assert psig["eps_cg"].default == vals["eps"]


def test_paper_stop_rule_and_caps(oracle):
    """The 'paper' stop rule ends the inner loop at the first iterate with
    delta <= eps^2 delta_0 (delta recomputed here from the iterates); l_max = 1
    caps the inner loop after one step."""
    assert pin_paper_inner_stop(oracle)
    M, N = 16, 16
    psi, _ = noisy_peaks(M, N, 4.0, 0.3, 15)
    r1 = oracle.unwrap(psi, p=0.0, precond="jacobi", l_max=1, k_max=2, outer_tol=0.0)
    assert r1.inner_iters == [1, 1]


# ---------------------------------------------------------------------------
# Algorithm 1's control flow: inner stop test, residual schedule, outer error
# ---------------------------------------------------------------------------
def dense_system(M, N, U, V):
    """A = D^T W D from the incidence matrix, with W the edge weights U (x edges)
    and V (y edges); written independently of the oracle's stencil."""
    D, E = incidence(M, N)
    w = edge_values(E, U, V)
    return D.T @ (w[:, None] * D)


def pin_paper_inner_stop(O):
    """Algorithm 1's inner test: PCG continues while delta > eps^2 delta_0, with
    delta = r^T M^{-1} r.  For Jacobi-PCG on a random weighted grid, delta is
    recomputed from every iterate with a dense A and diag(A): the last iterate
    is the first whose delta is at or below eps^2 delta_0.  A mistake in the
    bound (eps instead of eps^2) stops the loop well before that."""
    ok = True
    for seed, (M, N), eps in ((21, (9, 11), 0.005), (22, (12, 7), 0.05), (23, (10, 10), 0.01)):
        rng = np.random.default_rng(seed)
        U, V = random_weights(M, N, rng, lo=0.02)
        A = dense_system(M, N, U, V)
        b = rng.normal(size=M * N)
        b -= b.mean()
        res = O.pcg(U, V, b.reshape(M, N), np.zeros((M, N)), O.Preconditioner("jacobi", U, V),
                    stop_rule="paper", eps_cg=eps, record_iterates=True)
        dg = np.diag(A)
        deltas = []
        for x in res.iterates:
            r = b - A @ x.ravel()
            deltas.append(float(r @ (r / dg)))
        bound = eps * eps * deltas[0]
        L = res.iters
        ok &= L >= 2 and len(deltas) == L + 1
        ok &= deltas[L] <= bound * (1 + 1e-9)
        ok &= all(d > bound * (1 + 1e-9) for d in deltas[:L])
        # the case is not decided by rounding: both sides of the boundary are clear
        ok &= abs(deltas[L] / bound - 1) > 1e-6 and abs(deltas[L - 1] / bound - 1) > 1e-6
    return bool(ok)


def pin_relres_stop_on_true_residual(O):
    """The relative-residual rule ends at the first iterate whose true residual
    ||b - A x|| (dense A here) is within tol ||b||."""
    ok = True
    for seed, pc in ((24, "none"), (25, "jacobi"), (26, "ilu0")):
        rng = np.random.default_rng(seed)
        M, N = 8, 9
        U, V = random_weights(M, N, rng, lo=0.02)
        A = dense_system(M, N, U, V)
        b = rng.normal(size=M * N)
        b -= b.mean()
        tol = 1e-6
        res = O.pcg(U, V, b.reshape(M, N), np.zeros((M, N)), O.Preconditioner(pc, U, V),
                    tol=tol, record_iterates=True)
        rel = [np.linalg.norm(b - A @ x.ravel()) / np.linalg.norm(b) for x in res.iterates]
        ok &= rel[-1] <= tol * (1 + 1e-6) and all(v > tol for v in rel[:-1])
    return bool(ok)


def _call_trace(O, run):
    """Run ``run(spy_precond)`` with the oracle's stencil product and the
    preconditioner's apply logged: returns the sequence of 'A' / 'M' calls."""
    events = []
    orig = O.apply_A

    def spy_A(U, V, x):
        events.append("A")
        return orig(U, V, x)

    def wrap_precond(P):
        inner = P.apply

        def spy_M(r):
            events.append("M")
            return inner(r)
        P.apply = spy_M
        return P
    O.apply_A = spy_A
    try:
        run(wrap_precond)
    finally:
        O.apply_A = orig
    return events


def pin_residual_replacement_schedule(O):
    """Algorithm 1 recomputes r = b - A x in the iterations l divisible by the
    period (l = 0 included).  Observed from the calls PCG makes: one stencil
    product per iteration (A d), a second one in a replacement iteration, one
    preconditioner apply per iteration."""
    ok = True
    rng = np.random.default_rng(27)
    M, N = 6, 7
    U, V = random_weights(M, N, rng)
    b = rng.normal(size=(M, N))
    b -= b.mean()
    for L, P in ((11, 4), (10, 3), (7, 1), (9, 20)):
        ev = _call_trace(O, lambda w: O.pcg(U, V, b, np.zeros((M, N)), w(O.Preconditioner("jacobi", U, V)),
                                             stop_rule="paper", eps_cg=1e-30, l_max=L, period=P))
        # r0 and s0, then per iteration A [A] M, then the final true residual
        ok &= ev[:2] == ["A", "M"] and ev[-1] == "A"
        body = "".join(ev[2:-1])
        chunks = body.split("M")
        ok &= chunks[-1] == ""
        chunks = chunks[:-1]
        ok &= len(chunks) == L
        replaced = {l for l, c in enumerate(chunks) if c == "AA"}
        ok &= all(c in ("A", "AA") for c in chunks)
        ok &= replaced == {l for l in range(L) if l % P == 0}
    return bool(ok)


def pin_outer_relative_change(O):
    """Algorithm 1's outer error ||phi^{k+1} - phi^k|| / ||phi^k||, recomputed
    from the iterates: every reported value matches, a zero start gives an
    infinite first error, and the loop stops at the first iteration whose error
    is at or below the tolerance."""
    M, N = 14, 12
    psi, _ = noisy_peaks(M, N, 3.0, 0.3, 28)
    phi0 = 0.05 * np.random.default_rng(29).normal(size=(M, N))
    r = O.unwrap(psi, p=0.0, precond="ilu0", tol=1e-12, k_max=4, outer_tol=0.0,
                 phi0=phi0, keep_history=True)
    its = [phi0] + r.history
    want = [np.linalg.norm(b - a) / np.linalg.norm(a) for a, b in zip(its, its[1:])]
    ok = len(r.outer_errs) == 4 and np.allclose(r.outer_errs, want, rtol=1e-12, atol=0)
    ok &= math.isclose(r.outer_err, want[-1], rel_tol=1e-12)
    # from phi0 = 0 the first error is infinite
    r0 = O.unwrap(psi, p=0.0, precond="ilu0", tol=1e-12, k_max=1, outer_tol=0.5)
    ok &= math.isinf(r0.outer_err) and r0.outer_iters == 1 and not r0.converged
    # stop at the first error at or below outer_tol
    e = want
    if e[2] < e[1]:
        tol = math.sqrt(e[1] * e[2])
        first = next(k for k, v in enumerate(e) if v <= tol) + 1
        rs = O.unwrap(psi, p=0.0, precond="ilu0", tol=1e-12, k_max=10, outer_tol=tol, phi0=phi0)
        ok &= rs.converged and rs.outer_iters == first
    else:
        ok = False
    return bool(ok)


def test_algorithm1_control_flow(oracle):
    assert pin_paper_inner_stop(oracle)
    assert pin_relres_stop_on_true_residual(oracle)
    assert pin_residual_replacement_schedule(oracle)
    assert pin_outer_relative_change(oracle)


def test_mutation_paper_bound_eps_not_squared(oracle, monkeypatch):
    """The inner test with eps delta_0 in place of eps^2 delta_0."""
    _mutant(oracle, monkeypatch, "paper_inner_bound", lambda d0, eps: eps * d0)
    assert not pin_paper_inner_stop(oracle)


def test_mutation_outer_error_normalised_by_new_iterate(oracle, monkeypatch):
    """The outer error divided by ||phi^{k+1}|| instead of ||phi^k||."""
    def bad(phi_next, phi):
        n = float(np.linalg.norm(phi_next))
        return float(np.linalg.norm(phi_next - phi)) / n if n > 0 else math.inf
    _mutant(oracle, monkeypatch, "outer_relative_change", bad)
    assert not pin_outer_relative_change(oracle)


def test_mutation_replacement_offset(oracle, monkeypatch):
    """Replacement in the iterations with l mod P == 1 instead of 0."""
    _mutant(oracle, monkeypatch, "replacement_due", lambda l, P: l % P == (1 % P))
    assert not pin_residual_replacement_schedule(oracle)


def test_one_row_map_pivot_floor(oracle):
    """A one-row map is a chain: the no-fill factorization is exact and its last
    pivot vanishes; the pivot floor keeps the preconditioner SPD and PCG converges."""
    rng = np.random.default_rng(16)
    N = 50
    psi = synth.wrap_measurement(np.cumsum(rng.normal(0, 0.5, N))[None, :])
    for pc in ("ilu0", "ic0"):
        r = oracle.unwrap(psi, p=0.0, precond=pc, k_max=3, outer_tol=0.0)
        assert max(r.relres) <= 1e-6


# ---------------------------------------------------------------------------
# mutation checks: plant a plausible mistake in the oracle, a pin must fail
# ---------------------------------------------------------------------------
def _mutant(oracle, monkeypatch, name, fn):
    monkeypatch.setattr(oracle, name, fn)
    return oracle


def test_mutation_wrap_floor_convention(oracle, monkeypatch):
    """W with floor instead of ceil maps +pi to -pi (range [-pi, pi))."""
    orig = oracle.wrap
    _mutant(oracle, monkeypatch, "wrap",
            lambda x: np.asarray(x, float) - 2 * np.pi * np.floor((np.asarray(x, float) + np.pi) / (2 * np.pi)))
    assert not pin_wrap_range_and_ties(oracle)
    monkeypatch.setattr(oracle, "wrap", orig)


def test_mutation_weights_exponent(oracle, monkeypatch):
    """Using |r|^p instead of |r|^(2-p) in Eq. (6)."""
    orig = oracle._abs_pow
    _mutant(oracle, monkeypatch, "_abs_pow", lambda r, p: orig(r, 2.0 - p))
    assert not pin_weights_hand_values(oracle)


def test_mutation_stencil_swapped_weights(oracle, monkeypatch):
    """Eq. (7) with the roles of U and V exchanged (a transposed operand)."""
    orig = oracle.apply_A
    _mutant(oracle, monkeypatch, "apply_A", lambda U, V, x: orig(V, U, x))
    assert not pin_normal_equations(oracle)


def test_mutation_rhs_sign(oracle, monkeypatch):
    """b with the opposite sign."""
    orig = oracle.rhs
    _mutant(oracle, monkeypatch, "rhs", lambda U, V, dx, dy: -orig(U, V, dx, dy))
    assert not pin_gradient_of_energy(oracle)


def test_mutation_dropped_neighbour(oracle, monkeypatch):
    """Eq. (7) missing the north neighbour's off-diagonal term."""
    sh = oracle._shift

    def bad(U, V, x):
        return (oracle.diag_A(U, V) * x
                - (sh(x, 0, 1) * U + sh(x, 1, 0) * V + sh(x, 0, -1) * sh(U, 0, -1)))
    _mutant(oracle, monkeypatch, "apply_A", bad)
    assert not pin_laplacian_properties_matrix_free(oracle)


def pin_laplacian_properties_matrix_free(O):
    rng = np.random.default_rng(17)
    M, N = 5, 6
    U, V = random_weights(M, N, rng)
    n = M * N
    A = np.column_stack([O.apply_A(U, V, np.eye(n)[:, k].reshape(M, N)).ravel() for k in range(n)])
    return bool(np.allclose(A, A.T) and np.allclose(A @ np.ones(n), 0))


def test_matrix_free_properties(oracle):
    assert pin_laplacian_properties_matrix_free(oracle)


def test_mutation_red_black_order(oracle, monkeypatch):
    """A two-colour ordering that keeps the colours interleaved (the natural order)
    is caught."""
    _mutant(oracle, monkeypatch, "red_black_order", lambda M, N: np.arange(M * N))
    assert not pin_red_black_factorizations(oracle)


def test_mutation_dct_unnormalised(oracle, monkeypatch):
    """A DCT matrix missing the orthonormal scale of row 0."""
    orig = oracle.dct_matrix

    def bad(n):
        C = orig(n)
        C[0, :] *= math.sqrt(2.0)
        return C
    _mutant(oracle, monkeypatch, "dct_matrix", bad)
    assert not pin_dct_against_library(oracle)


def test_mutation_pcg_beta(oracle, monkeypatch):
    """PCG with the direction update d = s (beta dropped, steepest descent): the
    finite-termination pin fails."""
    src_pcg = oracle.pcg

    def bad_pcg(U, V, b, x0, M, **kw):
        kw = dict(kw)
        kw["l_max"] = 8
        x = np.array(x0, float)
        r = b - oracle.apply_A(U, V, x)
        for _ in range(8):
            s = M.apply(r)
            q = oracle.apply_A(U, V, s)
            x = x + float(np.sum(r * s)) / float(np.sum(s * q)) * s
            r = b - oracle.apply_A(U, V, x)
        rel = float(np.linalg.norm(r) / np.linalg.norm(b))
        return oracle.PCGResult(x, 8, rel < 1e-10, rel, 0.0, [])
    _mutant(oracle, monkeypatch, "pcg", bad_pcg)
    assert not pin_cg_finite_termination(oracle)
    monkeypatch.setattr(oracle, "pcg", src_pcg)


def test_mutation_dct_fft_inverse_type(oracle, monkeypatch):
    """The FFT path inverting with a DCT-II instead of the DCT-III."""
    _mutant(oracle, monkeypatch, "dct3_ortho", oracle.dct2_ortho)
    assert not pin_dct_fft_path(oracle)
