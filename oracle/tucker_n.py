"""FP64 CPU oracle for Tucker decompositions of sparse tensors of any order
N >= 3, for the fourth-order forms of Turney, "Empirical Evaluation of Four
Tensor Decomposition Algorithms" (NRC ERB-1152, 2007).

TEST INFRASTRUCTURE ONLY. Imported by the test-suite and the benchmark, never
by the GPU library, with which it shares no code.

Followed step by step:

* HO-SVD of order N: Section 4.1, Figure 2 (every A(n) from the leading
  eigenvectors of X_(n) X_(n)^T, then the core);
* HOOI of order N: Section 4.2, Figure 4 (A(2..N) from HO-SVD, then per
  iteration A(n) from Z_(n) Z_(n)^T with Z = X projected on every other
  factor, the core, the fit and the Delta_fit rule);
* MP of order four: Section 4.4, Figure 8 (pseudo HO-SVD start of A(2..N)
  from sums of slice products, then per iteration each M_n as the sum, over
  every other mode m, of the products X_s A(m) A(m)^T X_s^T of the
  two-dimensional slices X_s whose free modes are n and m), written here for
  any N (the figure's pattern with N - 1 terms per matrix).

Notation and definitions (n-mode product, matricization with the lower
remaining mode varying fastest, Tucker operator, fit) are those of Section 3.
Readings shared with the third-order oracle: "leading eigenvectors of
M M^T" computed literally for MP, eigenvector signs fixed so that the
largest-magnitude entry of each column is positive, duplicate coordinates
summed, the signed stopping rule with a previous fit of 0.

Parity unpinned: exact factor values on tensors whose leading eigenvalues
are (nearly) tied; only the fit is pinned there.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

__all__ = ["SparseTensorN", "mode_product_dense", "tucker_dense", "lead_eigvecs", "lead_eigvecs_of_MMt",
           "unfolding_gram", "project", "multi_project", "core", "fit_identity", "fit_dense", "mp_gram",
           "mp_init_gram", "hosvd", "hooi", "mp", "Decomposition"]


class SparseTensorN:
    """Sparse I_1 x ... x I_N tensor in coordinate form; duplicates summed."""

    def __init__(self, idx, vals, dims):
        idx = np.asarray(idx, dtype=np.int64)
        vals = np.asarray(vals, dtype=np.float64)
        self.dims = tuple(int(d) for d in dims)
        self.N = len(self.dims)
        if idx.shape != (self.N, vals.size):
            raise ValueError("idx must have shape (N, nnz)")
        lin = np.ravel_multi_index(tuple(idx), self.dims)
        uniq, inv = np.unique(lin, return_inverse=True)
        summed = np.zeros(uniq.size)
        np.add.at(summed, inv, vals)
        self.idx = np.stack(np.unravel_index(uniq, self.dims)).astype(np.int64)
        self.v = summed
        self.nnz = summed.size

    def norm2(self) -> float:
        return math.fsum(float(x) * float(x) for x in self.v)

    def dense(self) -> np.ndarray:
        out = np.zeros(self.dims)
        out[tuple(self.idx)] = self.v
        return out

    def _col(self, modes):
        """Column index of the listed modes, the first listed varying fastest."""
        col = np.zeros(self.nnz, dtype=np.int64)
        stride = 1
        for m in modes:
            col += self.idx[m] * stride
            stride *= self.dims[m]
        return col, stride

    def unfolding(self, n: int):
        """X_(n): I_n x (product of the other sizes), mode-n fibres as columns,
        the lower remaining mode varying fastest (Section 3)."""
        others = [m for m in range(self.N) if m != n]
        col, ncol = self._col(others)
        return sp.csr_matrix((self.v, (self.idx[n], col)), shape=(self.dims[n], ncol))

    def slices(self, n: int, m: int):
        """The two-dimensional slices whose free modes are n (rows) and m
        (columns), one for every combination of the other coordinates, as a
        list of sparse I_n x I_m matrices (empty ones included)."""
        rest = [k for k in range(self.N) if k not in (n, m)]
        key, nkey = self._col(rest)
        rows = key * self.dims[n] + self.idx[n]
        big = sp.csr_matrix((self.v, (rows, self.idx[m])), shape=(nkey * self.dims[n], self.dims[m]))
        In = self.dims[n]
        return [big[s * In:(s + 1) * In] for s in range(nkey)]


# --------------------------------------------------------------------------
# Definitions (Section 3)
# --------------------------------------------------------------------------
def mode_product_dense(X: np.ndarray, A: np.ndarray, n: int) -> np.ndarray:
    """Y = X x_n A: y[..., j, ...] = sum_i x[..., i, ...] a[j, i], written as
    a loop over the output index j."""
    Xn = np.moveaxis(X, n, 0)
    out = np.zeros((A.shape[0],) + Xn.shape[1:])
    for j in range(A.shape[0]):
        out[j] = np.tensordot(A[j], Xn, axes=(0, 0))
    return np.moveaxis(out, 0, n)


def tucker_dense(G: np.ndarray, factors) -> np.ndarray:
    """[[G; A(1), ..., A(N)]] = G x_1 A(1) ... x_N A(N)."""
    out = G
    for n, A in enumerate(factors):
        out = mode_product_dense(out, A, n)
    return out


def project(X: SparseTensorN, A: np.ndarray, m: int) -> np.ndarray:
    """X x_m A^T as a dense tensor (mode m of size A's column count), by the
    matricized form Y_(m) = A^T X_(m), folded back."""
    others = [k for k in range(X.N) if k != m]
    Ym = np.asarray((X.unfolding(m).T @ A).T)           # J x prod(others), first other fastest
    shape = [X.dims[k] for k in reversed(others)]       # C order: last other slowest
    Y = Ym.reshape([A.shape[1]] + shape)                # [J][i_last]...[i_first]
    # axes now: J, others reversed -> put them back in mode order
    perm_src = [m] + list(reversed(others))
    return np.transpose(Y, np.argsort(perm_src))


def multi_project(X: SparseTensorN, factors, skip=None) -> np.ndarray:
    """X x_m A(m)^T over every mode m except `skip` (None: all modes): the
    first product from the sparse tensor, the others dense."""
    modes = [m for m in range(X.N) if m != skip]
    Y = project(X, factors[modes[0]], modes[0])
    for m in modes[1:]:
        Y = mode_product_dense(Y, factors[m].T, m)
    return Y


def core(X: SparseTensorN, factors) -> np.ndarray:
    """G = [[X; A(1)^T, ..., A(N)^T]]."""
    return multi_project(X, factors)


def fit_identity(normX2: float, G) -> float:
    """fit for orthonormal factors and G = [[X; A^T ...]]: ||X - Xhat||^2 =
    ||X||^2 - ||G||^2."""
    g2 = math.fsum(float(x) * float(x) for x in np.ravel(G))
    return 1.0 - math.sqrt(max(0.0, normX2 - g2)) / math.sqrt(normX2)


def fit_dense(Xd: np.ndarray, G, factors) -> float:
    """fit(X, Xhat) = 1 - ||X - Xhat|| / ||X|| with Xhat formed densely."""
    R = Xd - tucker_dense(G, factors)
    return 1.0 - math.sqrt(math.fsum(np.ravel(R * R))) / math.sqrt(math.fsum(np.ravel(Xd * Xd)))


# --------------------------------------------------------------------------
# Leading eigenvectors and Grams
# --------------------------------------------------------------------------
def _canonical(V):
    V = V.copy()
    for c in range(V.shape[1]):
        r = int(np.argmax(np.abs(V[:, c])))
        if V[r, c] < 0:
            V[:, c] = -V[:, c]
    return V


def lead_eigvecs(S: np.ndarray, J: int):
    """J leading eigenvectors of the symmetric S (LAPACK via eigh), columns in
    descending eigenvalue order with canonical signs."""
    S = 0.5 * (S + S.T)
    w, V = np.linalg.eigh(S)
    order = np.argsort(-w, kind="stable")[:J]
    return _canonical(V[:, order]), w[order]


def lead_eigvecs_of_MMt(M: np.ndarray, J: int):
    """"J leading eigenvectors of M M^T" as MP writes it (Figure 8)."""
    return lead_eigvecs(M @ M.T, J)


def unfolding_gram(X: SparseTensorN, n: int) -> np.ndarray:
    """X_(n) X_(n)^T (Figures 2 and 4)."""
    U = X.unfolding(n)
    return (U @ U.T).toarray()


def mp_gram(X: SparseTensorN, n: int, factors) -> np.ndarray:
    """MP's main-loop matrix of mode n (Figure 8): for every other mode m, the
    sum over the slices X_s with free modes (n, m) of X_s A(m) A(m)^T X_s^T."""
    M = np.zeros((X.dims[n], X.dims[n]))
    for m in range(X.N):
        if m == n:
            continue
        for S in X.slices(n, m):
            if S.nnz == 0:
                continue
            P = np.asarray(S @ factors[m])
            M += P @ P.T
    return M


def mp_init_gram(X: SparseTensorN, n: int) -> np.ndarray:
    """MP's pseudo HO-SVD matrix of mode n (Figure 8, before the main loop):
    for every other mode m, the sum over the slices X_s with free modes
    (n, m) of X_s X_s^T."""
    M = np.zeros((X.dims[n], X.dims[n]))
    for m in range(X.N):
        if m == n:
            continue
        for S in X.slices(n, m):
            if S.nnz:
                M += (S @ S.T).toarray()
    return M


# --------------------------------------------------------------------------
# Algorithms
# --------------------------------------------------------------------------
@dataclass
class Decomposition:
    core: np.ndarray
    factors: list
    fits: list = field(default_factory=list)
    iters: int = 0
    extra: dict = field(default_factory=dict)


def _check(X, J):
    if len(J) != X.N or any(int(J[n]) < 1 or int(J[n]) > X.dims[n] for n in range(X.N)):
        raise ValueError("core sizes must satisfy 1 <= J_n <= I_n, one per mode")


def _stop(f, prev, tol):
    return tol > 0 and (f - prev) < tol


def hosvd(X: SparseTensorN, J) -> Decomposition:
    """Figure 2: A(n) <- J_n leading eigenvectors of X_(n) X_(n)^T for every
    n, then G <- [[X; A(1)^T, ..., A(N)^T]] and its fit."""
    _check(X, J)
    facs = [lead_eigvecs(unfolding_gram(X, n), J[n])[0] for n in range(X.N)]
    G = core(X, facs)
    return Decomposition(G, facs, [fit_identity(X.norm2(), G)], 0)


def hooi(X: SparseTensorN, J, max_iters: int = 50, tol: float = 1e-4, init=None) -> Decomposition:
    """Figure 4: A(2..N) from HO-SVD (A(1) needs no start), then per
    iteration, for n = 1..N, Z = X projected on every other factor and A(n)
    <- J_n leading eigenvectors of Z_(n) Z_(n)^T; the core and the fit after
    every iteration, stopping on Delta_fit."""
    _check(X, J)
    facs = [None] * X.N
    for n in range(1, X.N):
        facs[n] = lead_eigvecs(unfolding_gram(X, n), J[n])[0] if init is None else np.array(init[n], dtype=float)
    nx2 = X.norm2()
    fits, prev, t = [], 0.0, 0
    for t in range(1, max_iters + 1):
        for n in range(X.N):
            Z = multi_project(X, facs, skip=n)
            Zn = np.moveaxis(Z, n, 0).reshape(X.dims[n], -1)
            facs[n] = lead_eigvecs(Zn @ Zn.T, J[n])[0]
        G = core(X, facs)
        f = fit_identity(nx2, G)
        fits.append(f)
        if _stop(f, prev, tol):
            break
        prev = f
    if facs[0] is None:
        Z = multi_project(X, facs, skip=0)
        Zn = Z.reshape(X.dims[0], -1)
        facs[0] = lead_eigvecs(Zn @ Zn.T, J[0])[0]
    return Decomposition(core(X, facs), facs, fits, t)


def mp(X: SparseTensorN, J, max_iters: int = 50, tol: float = 1e-4, init=None) -> Decomposition:
    """Figure 8 (for any N): A(2..N) <- leading eigenvectors of M M^T of the
    pseudo HO-SVD matrices, then per iteration A(n) <- leading eigenvectors
    of M_n M_n^T with M_n from the most recent other factors, the core and
    the fit, stopping on Delta_fit."""
    _check(X, J)
    facs = [None] * X.N
    for n in range(1, X.N):
        facs[n] = lead_eigvecs_of_MMt(mp_init_gram(X, n), J[n])[0] if init is None else \
            np.array(init[n], dtype=float)
    nx2 = X.norm2()
    fits, prev, t = [], 0.0, 0
    for t in range(1, max_iters + 1):
        for n in range(X.N):
            facs[n] = lead_eigvecs_of_MMt(mp_gram(X, n, facs), J[n])[0]
        G = core(X, facs)
        f = fit_identity(nx2, G)
        fits.append(f)
        if _stop(f, prev, tol):
            break
        prev = f
    if facs[0] is None:
        facs[0] = lead_eigvecs_of_MMt(mp_gram(X, 0, facs), J[0])[0]
    return Decomposition(core(X, facs), facs, fits, t)
