"""FP64 CPU oracle for L^p-norm phase unwrapping with preconditioned CG.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything under ``oracle/``: only the tests, the smoke check
and the benchmark's CPU-baseline leg use it.  It shares no code with the HIP
path (its only native part, ``sparse_ref.c``, is textbook sparse algebra on
a generic CSR matrix).

Everything follows the paper (Legarda-Saenz, Brito-Loeza, Espinosa-Romero,
"On the performance of preconditioned methods to solve L^p-norm phase
unwrapping", arXiv 2203.13675) in plain, slow, vectorised numpy:

* ``wrap``                -- the wrapping operator W, Eq. (1) range (-pi, pi].
* ``wrapped_differences`` -- Delta^x, Delta^y of Section 2.1.
* ``irls_weights``        -- U, V of Eq. (6) (tau-regularised |r|^(p-2)).
* ``apply_A`` / ``rhs``   -- the two sides of Eq. (7).
* ``Preconditioner``      -- the five M of Section 2.1's list (I, D, ILU(0),
                             IC(0), SOR read as SSOR) plus the DCT Poisson
                             preconditioner (the unweighted Neumann Laplacian),
                             and ILU(0), IC(0) and SSOR of the matrix taken in
                             red-black order (a change of M, not in the paper).
* ``pcg``                 -- the inner loop of Algorithm 1: preconditioned CG
                             with the true residual recomputed on a schedule
                             (``replacement_due``) and the paper's stop test
                             (``paper_inner_bound``).
* ``unwrap``              -- Algorithm 1 (outer fixed-point loop), stopped by
                             ``outer_relative_change``.

Readings where the paper is silent or garbled:

* Grid: M rows (index i) by N columns (index j, contiguous); "x" edges join
  (i,j)-(i,j+1), "y" edges join (i,j)-(i+1,j).  Every in-grid neighbour pair
  is an edge and no edge leaves the grid (this gives Table 1's nonzero count
  5MN - 2(M+N)); the zero-flux boundary condition is U[:, N-1] = 0 and
  V[M-1, :] = 0, so the garbled "backward copy" entries of Delta never enter
  A or b.
* W(x) = x - 2*pi*ceil((x - pi) / (2*pi)), evaluated in FP64.
* U = w_e * tau / (|r|^(2-p) + tau) with p = 0, 1, 2 in closed form (r*r,
  |r|, 1) and pow() otherwise; w_e = min(mask_a, mask_b) is the quality of
  an edge (the mask is an extension: without one, w_e = 1).
* A pixel whose edges all have zero weight is isolated: its row of A is zero,
  every preconditioner returns 0 there and phi keeps its start value.
* SOR is used as SSOR(omega), default omega = 1.
* ILU(0)/IC(0) pivots below ``PIVOT_FLOOR`` times the diagonal are replaced by
  the diagonal (this only happens at the last node of chain-like components,
  e.g. one-row maps, where the no-fill factorization is exact and singular).
* DCT preconditioner: M = L0, the unit-weight Neumann Laplacian on the whole
  grid, applied through orthonormal DCT-II/III with the zero mode dropped.
* Inner stop rules: "paper" (delta_new <= eps^2 delta_0, eps = 0.005) and
  "relres" (||b - A phi|| <= tol ||b||, confirmed on the true residual).
* Residual replacement when l mod P == 0, P = max(1, floor(sqrt(MN))).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * np.pi
PIVOT_FLOOR = 1e-4

PRECONDITIONERS = {"none": 0, "jacobi": 1, "ilu0": 2, "ic0": 3, "ssor": 4, "dct": 5,
                   "ilu0_rb": 6, "ic0_rb": 7, "ssor_rb": 8}

# ---------------------------------------------------------------------------
# native helper (generic CSR ILU(0)/IC(0)/SSOR)
# ---------------------------------------------------------------------------
_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "liblp_oracle_sparse.so")
_lib = None


def build_native(force: bool = False) -> str:
    """Compile sparse_ref.c with gcc into oracle/_build (CPU only)."""
    src = os.path.join(_HERE, "sparse_ref.c")
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _native():
    global _lib
    if _lib is None:
        # LP_ORACLE_SPARSE_SO names another build of sparse_ref.c (the
        # sanitizer test loads an address/undefined-behaviour checked one)
        so = os.environ.get("LP_ORACLE_SPARSE_SO") or _SO
        if so == _SO and not os.path.exists(_SO):
            build_native()
        lib = ctypes.CDLL(so)
        ip = np.ctypeslib.ndpointer(np.int32, flags="C")
        dp = np.ctypeslib.ndpointer(np.float64, flags="C")
        lib.orc_ilu0.argtypes = [ctypes.c_int, ip, ip, dp, ctypes.c_double, dp]
        lib.orc_ilu0.restype = ctypes.c_int
        lib.orc_ic0.argtypes = [ctypes.c_int, ip, ip, dp, ctypes.c_double, dp]
        lib.orc_ic0.restype = ctypes.c_int
        lib.orc_lu_solve.argtypes = [ctypes.c_int, ip, ip, dp, dp, dp]
        lib.orc_llt_solve.argtypes = [ctypes.c_int, ip, ip, dp, dp, dp]
        lib.orc_ssor_solve.argtypes = [ctypes.c_int, ip, ip, dp, ctypes.c_double, dp, dp]
        for f in (lib.orc_lu_solve, lib.orc_llt_solve, lib.orc_ssor_solve):
            f.restype = None
        _lib = lib
    return _lib


# ---------------------------------------------------------------------------
# Eq. (1) and Section 2.1: wrapping and wrapped differences
# ---------------------------------------------------------------------------
def wrap(x):
    """W(x) = x + 2*pi*k with the result in (-pi, pi] (Eq. (1) range)."""
    x = np.asarray(x, dtype=np.float64)
    return x - TWO_PI * np.ceil((x - np.pi) / TWO_PI)


def wrapped_differences(psi: np.ndarray):
    """Delta^x_{i,j} = W(psi_{i,j+1} - psi_{i,j}) (j < N-1) and
    Delta^y_{i,j} = W(psi_{i+1,j} - psi_{i,j}) (i < M-1), Section 2.1.

    The last column of Delta^x and last row of Delta^y are returned as 0: they
    are multiplied by a zero weight under the zero-flux boundary condition."""
    psi = np.asarray(psi, dtype=np.float64)
    M, N = psi.shape
    dx = np.zeros((M, N))
    dy = np.zeros((M, N))
    dx[:, :N - 1] = wrap(psi[:, 1:] - psi[:, :-1])
    dy[:M - 1, :] = wrap(psi[1:, :] - psi[:-1, :])
    return dx, dy


def edge_quality(mask, M: int, N: int):
    """Per-edge quality w_e = min(mask_a, mask_b); edges leaving the grid get 0."""
    wx = np.zeros((M, N))
    wy = np.zeros((M, N))
    if mask is None:
        wx[:, :N - 1] = 1.0
        wy[:M - 1, :] = 1.0
    else:
        m = np.asarray(mask, dtype=np.float64)
        wx[:, :N - 1] = np.minimum(m[:, 1:], m[:, :-1])
        wy[:M - 1, :] = np.minimum(m[1:, :], m[:-1, :])
    return wx, wy


def _abs_pow(r, p):
    a = np.abs(r)
    e = 2.0 - p
    if e == 2.0:
        return r * r
    if e == 1.0:
        return a
    if e == 0.0:
        return np.ones_like(a)
    return np.power(a, e)


def irls_weights(phi, dx, dy, wx, wy, p: float, tau: float):
    """U, V of Eq. (6): tau / (|grad phi - Delta|^(2-p) + tau), times edge quality,
    zero on the last column (U) and last row (V) -- the zero-flux boundary."""
    phi = np.asarray(phi, dtype=np.float64)
    M, N = phi.shape
    U = np.zeros((M, N))
    V = np.zeros((M, N))
    rx = phi[:, 1:] - phi[:, :-1] - dx[:, :N - 1]
    ry = phi[1:, :] - phi[:-1, :] - dy[:M - 1, :]
    U[:, :N - 1] = wx[:, :N - 1] * (tau / (_abs_pow(rx, p) + tau))
    V[:M - 1, :] = wy[:M - 1, :] * (tau / (_abs_pow(ry, p) + tau))
    return U, V


# ---------------------------------------------------------------------------
# Eq. (7): A phi = b
# ---------------------------------------------------------------------------
def _shift(a, di, dj):
    """out[i, j] = a[i + di, j + dj], zero outside the grid."""
    M, N = a.shape
    out = np.zeros_like(a)
    i0, i1 = max(0, -di), min(M, M - di)
    j0, j1 = max(0, -dj), min(N, N - dj)
    out[i0:i1, j0:j1] = a[i0 + di:i1 + di, j0 + dj:j1 + dj]
    return out


def diag_A(U, V):
    """Diagonal of A, Eq. (7): U_{i,j-1} + U_{i,j} + V_{i-1,j} + V_{i,j}."""
    return _shift(U, 0, -1) + U + _shift(V, -1, 0) + V


def apply_A(U, V, x):
    """Left side of Eq. (7) for every pixel."""
    x = np.asarray(x, dtype=np.float64)
    return (diag_A(U, V) * x
            - (_shift(x, 0, 1) * U + _shift(x, 1, 0) * V
               + _shift(x, 0, -1) * _shift(U, 0, -1) + _shift(x, -1, 0) * _shift(V, -1, 0)))


def rhs(U, V, dx, dy):
    """Right side of Eq. (7): Delta^x_{i,j-1}U_{i,j-1} - Delta^x_{i,j}U_{i,j}
    + Delta^y_{i-1,j}V_{i-1,j} - Delta^y_{i,j}V_{i,j}."""
    gx = dx * U
    gy = dy * V
    return _shift(gx, 0, -1) - gx + _shift(gy, -1, 0) - gy


def assemble_csr(U, V):
    """A of Eq. (7) as CSR (row-major pixel numbering p = i*N + j), every row with
    its five-point pattern (in-grid neighbours) and sorted columns.  Explicit zeros
    are kept so the pattern is the structural one of Table 1."""
    M, N = U.shape
    n = M * N
    d = diag_A(U, V).ravel()
    rows, cols, vals = [], [], []
    idx = np.arange(n).reshape(M, N)
    # north (i-1, j): -V_{i-1,j}
    rows.append(idx[1:, :].ravel()); cols.append(idx[:-1, :].ravel()); vals.append(-V[:-1, :].ravel())
    # west (i, j-1): -U_{i,j-1}
    rows.append(idx[:, 1:].ravel()); cols.append(idx[:, :-1].ravel()); vals.append(-U[:, :-1].ravel())
    # centre
    rows.append(idx.ravel()); cols.append(idx.ravel()); vals.append(d)
    # east (i, j+1): -U_{i,j}
    rows.append(idx[:, :-1].ravel()); cols.append(idx[:, 1:].ravel()); vals.append(-U[:, :-1].ravel())
    # south (i+1, j): -V_{i,j}
    rows.append(idx[:-1, :].ravel()); cols.append(idx[1:, :].ravel()); vals.append(-V[:-1, :].ravel())
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    return rowptr, c.astype(np.int32), np.ascontiguousarray(v, dtype=np.float64)


def red_black_order(M: int, N: int) -> np.ndarray:
    """Two-colour ordering of the grid: the pixels with i + j even ("red") first,
    then those with i + j odd ("black"), each colour in row-major order.  Entry k
    is the row-major pixel number i*N + j placed at position k."""
    idx = np.arange(M * N).reshape(M, N)
    red = (np.arange(M)[:, None] + np.arange(N)[None, :]) % 2 == 0
    return np.concatenate([idx[red], idx[~red]]).astype(np.int64)


def permute_csr(rowptr, col, a, perm):
    """P A P^T in CSR with sorted columns, where row k of the result is row perm[k]
    of A (and likewise for columns)."""
    n = len(rowptr) - 1
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    r2, c2 = inv[rows], inv[np.asarray(col, dtype=np.int64)]
    order = np.lexsort((c2, r2))
    r2, c2, v2 = r2[order], c2[order], np.asarray(a)[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, r2 + 1, 1)
    return (np.cumsum(rp).astype(np.int32), c2.astype(np.int32),
            np.ascontiguousarray(v2, dtype=np.float64))


def isolated_pixels(U, V):
    """Pixels whose four edge weights are all zero (a zero row of A)."""
    return diag_A(U, V) == 0.0


# ---------------------------------------------------------------------------
# DCT-II / DCT-III (orthonormal), from the definition
# ---------------------------------------------------------------------------
def dct_matrix(n: int) -> np.ndarray:
    """C[k, j] = s_k cos(pi k (2j+1) / (2n)), s_0 = sqrt(1/n), s_k = sqrt(2/n)."""
    k = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    C = np.cos(np.pi * k * (2 * j + 1) / (2.0 * n))
    C[0, :] *= math.sqrt(1.0 / n)
    C[1:, :] *= math.sqrt(2.0 / n)
    return C


def dct2_ortho(x: np.ndarray) -> np.ndarray:
    """C_M x C_N^T with C = dct_matrix, through scipy's O(MN log MN) DCT-II."""
    import scipy.fft
    return scipy.fft.dctn(x, type=2, norm="ortho")


def dct3_ortho(y: np.ndarray) -> np.ndarray:
    """C_M^T y C_N, the inverse of dct2_ortho (scipy's orthonormal DCT-III)."""
    import scipy.fft
    return scipy.fft.idctn(y, type=2, norm="ortho")


def neumann_eigenvalues(M: int, N: int) -> np.ndarray:
    """Eigenvalues of the unit-weight Neumann 5-point Laplacian in the DCT-II basis."""
    lm = 2.0 - 2.0 * np.cos(np.pi * np.arange(M) / M)
    ln = 2.0 - 2.0 * np.cos(np.pi * np.arange(N) / N)
    return lm[:, None] + ln[None, :]


# ---------------------------------------------------------------------------
# Preconditioners (Section 2.1 list + the DCT Poisson solve)
# ---------------------------------------------------------------------------
@dataclass
class Preconditioner:
    kind: str
    U: np.ndarray
    V: np.ndarray
    omega: float = 1.0
    setup_info: dict = field(default_factory=dict)
    # DCT preconditioner: "dense" multiplies by dct_matrix along each axis,
    # "fft" calls scipy's orthonormal DCT-II / DCT-III (the same transform,
    # O(MN log MN)); "auto" takes "fft" above 256 x 256 pixels
    dct_impl: str = "auto"

    def __post_init__(self):
        if self.kind not in PRECONDITIONERS:
            raise ValueError(self.kind)
        M, N = self.U.shape
        self.shape = (M, N)
        self.iso = isolated_pixels(self.U, self.V)
        self.keep = ~self.iso
        if self.kind == "jacobi":
            d = diag_A(self.U, self.V)
            self.inv_diag = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
        elif self.kind in ("ilu0", "ic0", "ssor", "ilu0_rb", "ic0_rb", "ssor_rb"):
            rowptr, col, a = assemble_csr(self.U, self.V)
            # an isolated pixel's row is replaced by the identity row
            diag_pos = self._diag_positions(rowptr, col)
            a = a.copy()
            a[diag_pos[self.iso.ravel()]] = 1.0
            self.base = self.kind[:-3] if self.kind.endswith("_rb") else self.kind
            # red-black variants: the same factorisation of P A P^T
            self.perm = red_black_order(M, N) if self.kind.endswith("_rb") else None
            if self.perm is not None:
                rowptr, col, a = permute_csr(rowptr, col, a, self.perm)
                diag_pos = self._diag_positions(rowptr, col)
            self.rowptr, self.col, self.a = rowptr, col, a
            self.diag_pos = diag_pos
            if self.base in ("ilu0", "ic0"):
                self._factor()
        elif self.kind == "dct":
            if self.dct_impl == "auto":
                self.dct_impl = "fft" if M * N > 256 * 256 else "dense"
            if self.dct_impl not in ("dense", "fft"):
                raise ValueError(self.dct_impl)
            if self.dct_impl == "dense":
                self.CM = dct_matrix(M)
                self.CN = dct_matrix(N)
            lam = neumann_eigenvalues(M, N)
            lam[0, 0] = 1.0
            self.inv_lam = 1.0 / lam
            self.inv_lam[0, 0] = 0.0

    @staticmethod
    def _diag_positions(rowptr, col):
        n = len(rowptr) - 1
        pos = np.empty(n, dtype=np.int64)
        for_rows = np.repeat(np.arange(n), np.diff(rowptr))
        hit = np.nonzero(col == for_rows)[0]
        pos[for_rows[hit]] = hit
        return pos

    def _factor(self):
        lib = _native()
        n = len(self.rowptr) - 1
        out = np.empty_like(self.a)
        f = lib.orc_ilu0 if self.base == "ilu0" else lib.orc_ic0
        rc = f(n, self.rowptr, self.col, self.a, PIVOT_FLOOR, out)
        if rc < 0:
            raise RuntimeError("row %d has no diagonal entry" % (-rc - 1))
        self.factor = out
        self.setup_info["pivot_floor_hits"] = rc

    def pivots(self):
        """Diagonal of the no-fill factor as a (M, N) array (ILU: U's diagonal,
        IC: squared diagonal of L); both equal the D-ILU pivots for Eq. (7)'s A."""
        p = self.factor[self.diag_pos]
        if self.base == "ic0":
            p = p * p
        if self.perm is not None:
            q = np.empty_like(p)
            q[self.perm] = p
            p = q
        return p.reshape(self.shape)

    def apply(self, r: np.ndarray) -> np.ndarray:
        """s = M^{-1} r (zero on isolated pixels)."""
        r = np.asarray(r, dtype=np.float64)
        k = self.kind
        if k == "none":
            s = r.copy()
        elif k == "jacobi":
            s = r * self.inv_diag
        elif k == "dct" and self.dct_impl == "fft":
            Y = dct2_ortho(r)
            Y *= self.inv_lam
            s = dct3_ortho(Y)
        elif k == "dct":
            Y = self.CM @ r @ self.CN.T
            Y *= self.inv_lam
            s = self.CM.T @ Y @ self.CN
        else:
            lib = _native()
            n = r.size
            rr = r.ravel()
            if self.perm is not None:
                rr = rr[self.perm]
            rr = np.ascontiguousarray(rr)
            s = np.empty(n)
            if self.base == "ilu0":
                lib.orc_lu_solve(n, self.rowptr, self.col, self.factor, rr, s)
            elif self.base == "ic0":
                lib.orc_llt_solve(n, self.rowptr, self.col, self.factor, rr, s)
            else:
                lib.orc_ssor_solve(n, self.rowptr, self.col, self.a, float(self.omega), rr, s)
            if self.perm is not None:
                t = np.empty(n)
                t[self.perm] = s
                s = t
            s = s.reshape(r.shape)
        return np.where(self.keep, s, 0.0)


# ---------------------------------------------------------------------------
# Algorithm 1, inner loop: preconditioned CG
# ---------------------------------------------------------------------------
@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    converged: bool
    relres: float
    delta0: float
    history: list
    deltas: list = field(default_factory=list)    # delta_0, delta_1, ... (record=True)
    iterates: list = field(default_factory=list)  # x_0, x_1, ... (record_iterates=True)


def replacement_due(l: int, period: int) -> bool:
    """Algorithm 1 recomputes the residual from its definition, r = b - A x, in
    the iterations whose counter l is divisible by sqrt(MN) (read as the period
    P = max(1, floor(sqrt(MN))), the first iteration l = 0 included)."""
    return l % period == 0


def paper_inner_bound(delta0: float, eps: float) -> float:
    """Algorithm 1's inner loop continues while delta_new > eps^2 delta_0, where
    delta = r^T M^{-1} r and delta_0 belongs to this solve's first residual."""
    return eps * eps * delta0


def _norm(v) -> float:
    return math.sqrt(float(np.sum(v * v)))


def _step_length(delta: float, d, q, l: int) -> float:
    """alpha = delta / d^T A d (the CG step along d); d^T A d must be positive."""
    curvature = float(np.sum(d * q))
    if not (curvature > 0.0):
        raise FloatingPointError("PCG breakdown: d^T A d <= 0 at l=%d" % l)
    return delta / curvature


def _advance_residual(U, V, b, x, r, alpha, q, l, period, confirm_below):
    """Residual of the new iterate x.  The CG recurrence gives r - alpha A d;
    Algorithm 1 replaces it by the true residual b - A x on its schedule
    (``replacement_due``).  With ``confirm_below`` set (the relative-residual
    stop rule), a recurrence value that meets the bound is replaced by the true
    residual as well, so the stop test is always taken on b - A x."""
    if replacement_due(l, period):
        return b - apply_A(U, V, x)
    r_next = r - alpha * q
    if confirm_below is not None and _norm(r_next) <= confirm_below:
        return b - apply_A(U, V, x)
    return r_next


def pcg(U, V, b, x0, M: Preconditioner, *, stop_rule: str = "relres", tol: float = 1e-6,
        eps_cg: float = 0.005, l_max: int | None = None, period: int | None = None,
        record: bool = False, record_iterates: bool = False) -> PCGResult:
    """Solve A x = b (Eq. (7)) by preconditioned CG from x0, the inner loop of
    Algorithm 1 (warm start from the outer iterate).

    Stop rules: "paper" runs while delta_new > eps_cg^2 delta_0
    (``paper_inner_bound``); "relres" runs while ||r|| > tol ||b||, tested on a
    true residual (``_advance_residual``).  At most l_max iterations (default
    2MN); the residual is recomputed from its definition every ``period``
    iterations (default floor(sqrt(MN))).

    With record=True the result keeps the relative residual after each
    iteration and the sequence delta_0, delta_1, ...; with record_iterates=True
    also every iterate x_0, x_1, ..."""
    n = b.size
    l_max = 2 * n if l_max is None else l_max
    period = max(1, math.isqrt(n)) if period is None else period
    x = np.array(x0, dtype=np.float64, copy=True)
    bnorm = _norm(b)
    r = b - apply_A(U, V, x)
    s = M.apply(r)
    delta = float(np.sum(r * s))
    delta0 = delta
    out = PCGResult(x, 0, True, 0.0, delta0, [])
    if record:
        out.deltas.append(delta)
    if record_iterates:
        out.iterates.append(x.copy())
    if bnorm == 0.0:
        return out
    paper = stop_rule == "paper"
    bound = paper_inner_bound(delta0, eps_cg)
    confirm_below = None if paper else tol * bnorm

    def satisfied(rv, dl):
        return not (dl > bound) if paper else _norm(rv) <= tol * bnorm

    d = s
    l = 0
    while l < l_max and not satisfied(r, delta):
        q = apply_A(U, V, d)
        alpha = _step_length(delta, d, q, l)
        x = x + alpha * d
        r = _advance_residual(U, V, b, x, r, alpha, q, l, period, confirm_below)
        s = M.apply(r)
        # the new direction is M^{-1} r made A-conjugate to the previous one
        delta_prev, delta = delta, float(np.sum(r * s))
        d = s + (delta / delta_prev) * d
        l += 1
        if record:
            out.history.append(_norm(r) / bnorm)
            out.deltas.append(delta)
        if record_iterates:
            out.iterates.append(x.copy())
    out.x, out.iters = x, l
    out.relres = _norm(b - apply_A(U, V, x)) / bnorm
    out.converged = bool(out.relres <= tol) if not paper else bool(not delta > bound)
    return out


# ---------------------------------------------------------------------------
# Algorithm 1, outer loop
# ---------------------------------------------------------------------------
@dataclass
class UnwrapResult:
    phi: np.ndarray
    outer_iters: int
    inner_iters: list
    outer_err: float
    relres: list
    converged: bool
    history: list = field(default_factory=list)
    outer_errs: list = field(default_factory=list)  # the outer error after each iteration


def outer_relative_change(phi_next, phi) -> float:
    """Algorithm 1's outer error ||phi^{k+1} - phi^k||_2 / ||phi^k||_2 (l2 over all
    pixels); +inf when phi^k = 0, so a zero start never stops the loop."""
    nrm = _norm(phi)
    return _norm(phi_next - phi) / nrm if nrm > 0 else math.inf


def unwrap(psi, mask=None, *, p: float = 0.0, tau: float = 0.01, precond: str = "dct",
           tol: float = 1e-6, k_max: int = 500, outer_tol: float = 1e-6, stop_rule: str = "relres",
           eps_cg: float = 0.005, l_max: int | None = None, period: int | None = None,
           omega: float = 1.0, phi0=None, keep_history: bool = False,
           dct_impl: str = "auto") -> UnwrapResult:
    """Algorithm 1: from phi^0, recompute U, V (Eq. (6)), solve Eq. (7) by PCG with
    warm start phi^{k+1} <- phi^k, until k = k_max or the relative change
    ||phi^{k+1} - phi^k|| / ||phi^k|| <= outer_tol (outer_tol <= 0: run k_max)."""
    psi = np.asarray(psi, dtype=np.float64)
    M, N = psi.shape
    dx, dy = wrapped_differences(psi)
    wx, wy = edge_quality(mask, M, N)
    phi = np.zeros((M, N)) if phi0 is None else np.array(phi0, dtype=np.float64, copy=True)
    k = 0
    err = math.inf
    inner, rels, hist, errs = [], [], [], []
    converged = False
    while k < k_max:
        U, V = irls_weights(phi, dx, dy, wx, wy, p, tau)
        b = rhs(U, V, dx, dy)
        P = Preconditioner(precond, U, V, omega=omega, dct_impl=dct_impl)
        res = pcg(U, V, b, phi, P, stop_rule=stop_rule, tol=tol, eps_cg=eps_cg,
                  l_max=l_max, period=period)
        err = outer_relative_change(res.x, phi)
        phi = res.x
        errs.append(err)
        inner.append(res.iters)
        rels.append(res.relres)
        if keep_history:
            hist.append(phi.copy())
        k += 1
        if outer_tol > 0 and err <= outer_tol:
            converged = True
            break
    return UnwrapResult(phi, k, inner, err, rels, converged, hist, errs)


# ---------------------------------------------------------------------------
# Exact inner solves (O-exact) and reporting helpers
# ---------------------------------------------------------------------------
def unwrap_exact(psi, mask=None, *, p=0.0, tau=0.01, outer=10, phi0=None, inner_tol=1e-12,
                 keep_history=False, precond="ic0"):
    """Algorithm 1 with every inner system solved to relres <= inner_tol (IC(0)-PCG by
    default; any preconditioner reaches the same solution): the reference for
    reporting errors of approximate inner solves."""
    return unwrap(psi, mask, p=p, tau=tau, precond=precond, tol=inner_tol, k_max=outer,
                  outer_tol=0.0, phi0=phi0, keep_history=keep_history)


def objective(phi, dx, dy, wx, wy, p: float, tau: float) -> float:
    """E(phi) = sum_e w_e rho(D phi - Delta): the tau-regularised energy whose IRLS
    weights are Eq. (6): rho'(r) = r * tau / (|r|^(2-p) + tau).  p = 0, 1, 2 only."""
    M, N = phi.shape
    rx = (phi[:, 1:] - phi[:, :-1] - dx[:, :N - 1])
    ry = (phi[1:, :] - phi[:-1, :] - dy[:M - 1, :])

    def rho(r):
        a = np.abs(r)
        if p == 0:
            return 0.5 * tau * np.log1p(r * r / tau)
        if p == 1:
            return tau * (a - tau * np.log1p(a / tau))
        if p == 2:
            return 0.5 * tau / (1.0 + tau) * r * r
        raise ValueError("closed-form energy only for p in {0,1,2}")

    return float(np.sum(wx[:, :N - 1] * rho(rx)) + np.sum(wy[:M - 1, :] * rho(ry)))


def normalized_error(mu, nu) -> float:
    """Q(mu, nu) = ||mu - nu||_2 / (||mu||_2 + ||nu||_2), Eq. (8)."""
    mu = np.asarray(mu, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    return float(np.linalg.norm(mu - nu) / (np.linalg.norm(mu) + np.linalg.norm(nu)))


def true_relres(psi, mask, phi_k, phi, *, p=0.0, tau=0.01) -> float:
    """||b - A phi|| / ||b|| for the system Eq. (7) built from the weights at phi_k."""
    psi = np.asarray(psi, dtype=np.float64)
    M, N = psi.shape
    dx, dy = wrapped_differences(psi)
    wx, wy = edge_quality(mask, M, N)
    U, V = irls_weights(phi_k, dx, dy, wx, wy, p, tau)
    b = rhs(U, V, dx, dy)
    r = b - apply_A(U, V, phi)
    return float(np.linalg.norm(r) / np.linalg.norm(b))
