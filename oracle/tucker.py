"""FP64 CPU oracle for the Tucker decompositions of sparse third-order tensors
evaluated in Turney, "Empirical Evaluation of Four Tensor Decomposition
Algorithms" (NRC ERB-1152, 2007).

TEST INFRASTRUCTURE ONLY. This package is imported by the test-suite, by the
package's ``smoke()`` check and by the benchmark's CPU-baseline leg, nowhere
else. The GPU library shares no code with it.

It is written to be checked by eye against the paper:

* notation, n-mode product, matricization, Tucker operator and the fit
  equation: Section 3 (Notation);
* HO-SVD: Section 4.1, Figure 1 (third order);
* HOOI: Section 4.2, Figure 3 (third order), stopping rule Delta_fit;
* SP: Section 4.3, Figure 5 (third order), stopping rule Delta_G;
* MP: Section 4.4, Figure 7 (third order); per-iteration core and fit as
  the appendix program computes them (one horizontal slice at a time).

All arithmetic is float64. Slices are scipy sparse matrices with the paper's
orientation: the horizontal slice X_{i::} is I2 x I3 (rows j, columns k), the
lateral slice X_{:j:} is I1 x I3 (rows i, columns k) and the frontal slice
X_{::k} is I1 x I2 (rows i, columns j).

Readings taken where the paper leaves a choice (each is listed in the design
notes of the repository):

* "J leading eigenvectors of M M^T" is computed literally for SP and MP (an
  eigendecomposition of the product M M^T); ``lead_eigvecs`` is the shared
  helper. For HO-SVD and HOOI the figures give X_(n) X_(n)^T directly.
* Eigenvector signs are not fixed by the paper; every column is flipped so
  that its entry of largest magnitude is positive.
* Duplicate coordinates are summed (the appendix builds slices with MATLAB's
  ``sparse``, which sums repeated entries).
* The stopping rules compare the signed change with the threshold and start
  from a previous fit of 0 (the appendix program's ``old_fit = 0``); a
  threshold <= 0 means "run exactly max_iters iterations".
* SP's previous core norm before the first iteration is 0.

Parity unpinned: the exact factor values of HOOI, SP and MP on tensors whose
leading eigenvalues are (nearly) tied; only their fit is pinned there.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

__all__ = [
    "SparseTensor3",
    "lead_eigvecs",
    "lead_eigvecs_of_MMt",
    "canonical_signs",
    "mode_product_dense",
    "unfold_dense",
    "tucker_dense",
    "project_dense",
    "project_sparse",
    "core_from_slices",
    "core_entry",
    "fit_slicewise",
    "fit_identity",
    "fit_dense",
    "unfolding_gram",
    "mp_init_grams",
    "mp_gram",
    "sp_gram",
    "hooi_gram",
    "hosvd",
    "hooi",
    "mp",
    "sp_algorithm",
    "Decomposition",
    "subspace_angle",
    "random_start",
]


# --------------------------------------------------------------------------
# Tensor container (Section 3: slices, fibres; appendix: slices of a sparse
# nonzero list)
# --------------------------------------------------------------------------
class SparseTensor3:
    """Sparse I1 x I2 x I3 tensor with its three families of slices.

    Duplicate coordinates are summed. Slices are cut from three CSR matrices
    whose rows enumerate (slice index, slice row).
    """

    def __init__(self, idx, vals, dims):
        idx = np.asarray(idx, dtype=np.int64)
        vals = np.asarray(vals, dtype=np.float64)
        self.dims = tuple(int(d) for d in dims)
        I1, I2, I3 = self.dims
        if idx.shape != (3, vals.size):
            raise ValueError("idx must have shape (3, nnz)")
        lin = (idx[0] * I2 + idx[1]) * I3 + idx[2]
        uniq, inv = np.unique(lin, return_inverse=True)
        summed = np.zeros(uniq.size)
        np.add.at(summed, inv, vals)
        i, j, k = np.unravel_index(uniq, self.dims)
        self.i, self.j, self.k, self.v = i, j, k, summed
        self.nnz = summed.size
        # horizontal slices X_{i::}: rows (i, j), columns k
        self._h = sp.csr_matrix((summed, (i * I2 + j, k)), shape=(I1 * I2, I3))
        # lateral slices X_{:j:}: rows (j, i), columns k
        self._l = sp.csr_matrix((summed, (j * I1 + i, k)), shape=(I2 * I1, I3))
        # frontal slices X_{::k}: rows (k, i), columns j
        self._f = sp.csr_matrix((summed, (k * I1 + i, j)), shape=(I3 * I1, I2))

    def horizontal(self, i):
        """X_{i::}, an I2 x I3 matrix."""
        I2 = self.dims[1]
        return self._h[i * I2:(i + 1) * I2]

    def lateral(self, j):
        """X_{:j:}, an I1 x I3 matrix."""
        I1 = self.dims[0]
        return self._l[j * I1:(j + 1) * I1]

    def frontal(self, k):
        """X_{::k}, an I1 x I2 matrix."""
        I1 = self.dims[0]
        return self._f[k * I1:(k + 1) * I1]

    def norm2(self) -> float:
        """Squared Frobenius norm (Section 3, below the fit equation)."""
        return math.fsum(float(x) * float(x) for x in self.v)

    def dense(self) -> np.ndarray:
        out = np.zeros(self.dims)
        out[self.i, self.j, self.k] = self.v
        return out

    def unfolding(self, n: int):
        """X_(n) as a sparse I_n x (prod of the other sizes) matrix.

        Mode-n fibres become columns (Section 3, matricization); the column
        order follows the paper's examples, with the lower remaining mode
        varying fastest."""
        I1, I2, I3 = self.dims
        if n == 0:
            rows, cols, shape = self.i, self.j + I2 * self.k, (I1, I2 * I3)
        elif n == 1:
            rows, cols, shape = self.j, self.i + I1 * self.k, (I2, I1 * I3)
        else:
            rows, cols, shape = self.k, self.i + I1 * self.j, (I3, I1 * I2)
        return sp.csr_matrix((self.v, (rows, cols)), shape=shape)


# --------------------------------------------------------------------------
# Dense definitions (Section 3)
# --------------------------------------------------------------------------
def mode_product_dense(X: np.ndarray, A: np.ndarray, n: int) -> np.ndarray:
    """Y = X x_n A: y[..., j, ...] = sum_{i_n} x[..., i_n, ...] a[j, i_n]
    (Section 3, n-mode product equation), written as explicit loops over the
    output index j."""
    Xn = np.moveaxis(X, n, 0)
    out = np.zeros((A.shape[0],) + Xn.shape[1:])
    for jj in range(A.shape[0]):
        for ii in range(A.shape[1]):
            out[jj] += A[jj, ii] * Xn[ii]
    return np.moveaxis(out, 0, n)


def unfold_dense(X: np.ndarray, n: int) -> np.ndarray:
    """X_(n): the mode-n fibres of X as columns (Section 3, matricization)."""
    I = X.shape
    cols = []
    others = [m for m in range(3) if m != n]
    a, b = others
    for ib in range(I[b]):
        for ia in range(I[a]):
            sl = [slice(None)] * 3
            sl[a], sl[b] = ia, ib
            cols.append(X[tuple(sl)])
    return np.stack(cols, axis=1)


def tucker_dense(G: np.ndarray, factors) -> np.ndarray:
    """[[G; A1, A2, A3]] = G x_1 A1 x_2 A2 x_3 A3 (Section 3, Tucker operator)."""
    out = G
    for n, A in enumerate(factors):
        out = mode_product_dense(out, A, n)
    return out


def project_dense(X: np.ndarray, A: np.ndarray, m: int) -> np.ndarray:
    """T = X x_m A^T, reordered to [i_a][i_b][r] where a < b are the other
    two modes and r indexes the columns of A."""
    T = mode_product_dense(X, A.T, m)
    return np.moveaxis(T, m, 2)


def project_sparse(X: "SparseTensor3", A: np.ndarray, m: int) -> np.ndarray:
    """T = X x_m A^T for the sparse X, laid out [i_a][i_b][r] as
    ``project_dense`` (a < b the other two modes): by the matricized form of
    the n-mode product (Section 3), T_(m) = A^T X_(m), one sparse product of
    the unfolding, then the columns (i_a fastest) folded back."""
    others = [n for n in range(3) if n != m]
    Ia, Ib = X.dims[others[0]], X.dims[others[1]]
    Tm = np.asarray((X.unfolding(m).T @ A))             # (Ib * Ia) x J, column index ia + Ia * ib
    return Tm.reshape(Ib, Ia, A.shape[1]).transpose(1, 0, 2)


# --------------------------------------------------------------------------
# Leading eigenvectors (every figure: "J leading eigenvectors of ...")
# --------------------------------------------------------------------------
def canonical_signs(V: np.ndarray) -> np.ndarray:
    """Flip each column so that its largest-magnitude entry is positive."""
    V = V.copy()
    for c in range(V.shape[1]):
        r = int(np.argmax(np.abs(V[:, c])))
        if V[r, c] < 0:
            V[:, c] = -V[:, c]
    return V


def lead_eigvecs(S: np.ndarray, J: int):
    """The J eigenvectors of the symmetric matrix S with the largest
    eigenvalues, as columns in descending eigenvalue order (LAPACK syevd via
    numpy.linalg.eigh). Returns (vectors, eigenvalues)."""
    S = 0.5 * (S + S.T)
    w, V = np.linalg.eigh(S)
    order = np.argsort(-w, kind="stable")[:J]
    return canonical_signs(V[:, order]), w[order]


def lead_eigvecs_of_MMt(M: np.ndarray, J: int):
    """"J leading eigenvectors of M M^T" exactly as SP and MP write it
    (Figures 5 and 7). Returns (vectors, eigenvalues of M M^T)."""
    return lead_eigvecs(M @ M.T, J)


# --------------------------------------------------------------------------
# Grams
# --------------------------------------------------------------------------
def unfolding_gram(X: SparseTensor3, n: int) -> np.ndarray:
    """X_(n) X_(n)^T (Figure 1 and the HOOI initialisation of Figure 3)."""
    U = X.unfolding(n)
    return (U @ U.T).toarray()


def mp_init_grams(X: SparseTensor3):
    """Pseudo HO-SVD initialisation of MP (Figure 7, before the main loop):
    M2 = sum_i X_{i::} X_{i::}^T + sum_k X_{::k}^T X_{::k},
    M3 = sum_i X_{i::}^T X_{i::} + sum_j X_{:j:}^T X_{:j:}."""
    I1, I2, I3 = X.dims
    M2 = np.zeros((I2, I2))
    for i in range(I1):
        S = X.horizontal(i)
        M2 += (S @ S.T).toarray()
    for k in range(I3):
        S = X.frontal(k)
        M2 += (S.T @ S).toarray()
    M3 = np.zeros((I3, I3))
    for i in range(I1):
        S = X.horizontal(i)
        M3 += (S.T @ S).toarray()
    for j in range(I2):
        S = X.lateral(j)
        M3 += (S.T @ S).toarray()
    return M2, M3


def _proj_outer(S, F) -> np.ndarray:
    """(S F)(S F)^T for a sparse slice S and a dense factor F."""
    P = np.asarray(S @ F)
    return P @ P.T


def mp_gram(X: SparseTensor3, n: int, A, B, C) -> np.ndarray:
    """The main-loop matrices of MP (Figure 7):
    M1 = sum_k X_{::k} B B^T X_{::k}^T + sum_j X_{:j:} C C^T X_{:j:}^T
    M2 = sum_k X_{::k}^T A A^T X_{::k} + sum_i X_{i::} C C^T X_{i::}^T
    M3 = sum_j X_{:j:}^T A A^T X_{:j:} + sum_i X_{i::}^T B B^T X_{i::}
    (slices on the two modes other than n)."""
    I1, I2, I3 = X.dims
    if n == 0:
        M = np.zeros((I1, I1))
        for k in range(I3):
            M += _proj_outer(X.frontal(k), B)
        for j in range(I2):
            M += _proj_outer(X.lateral(j), C)
    elif n == 1:
        M = np.zeros((I2, I2))
        for k in range(I3):
            M += _proj_outer(X.frontal(k).T, A)
        for i in range(I1):
            M += _proj_outer(X.horizontal(i), C)
    else:
        M = np.zeros((I3, I3))
        for j in range(I2):
            M += _proj_outer(X.lateral(j).T, A)
        for i in range(I1):
            M += _proj_outer(X.horizontal(i).T, B)
    return M


def sp_gram(X: SparseTensor3, n: int, F) -> np.ndarray:
    """The main-loop matrices of SP (Figure 5), each using one other factor:
    M13 = sum_j X_{:j:} C C^T X_{:j:}^T   (n = 0, F = C)
    M21 = sum_k X_{::k}^T A A^T X_{::k}   (n = 1, F = A)
    M32 = sum_i X_{i::}^T B B^T X_{i::}   (n = 2, F = B)."""
    I1, I2, I3 = X.dims
    if n == 0:
        M = np.zeros((I1, I1))
        for j in range(I2):
            M += _proj_outer(X.lateral(j), F)
    elif n == 1:
        M = np.zeros((I2, I2))
        for k in range(I3):
            M += _proj_outer(X.frontal(k).T, F)
    else:
        M = np.zeros((I3, I3))
        for i in range(I1):
            M += _proj_outer(X.horizontal(i).T, F)
    return M


def hooi_gram(X: SparseTensor3, n: int, A, B, C) -> np.ndarray:
    """Z_(n) Z_(n)^T for the HOOI main loop (Figure 3):
    U = [[X; I1, B^T, C^T]]  (n = 0), U[i] = B^T X_{i::} C;
    V = [[X; A^T, I2, C^T]]  (n = 1), V[:, j, :] = A^T X_{:j:} C;
    W = [[X; A^T, B^T, I3]]  (n = 2), W[:, :, k] = A^T X_{::k} B.
    Rows of the unfolding are the vectorised slices of the projected tensor."""
    I1, I2, I3 = X.dims
    if n == 0:
        Z = np.stack([np.ravel(B.T @ np.asarray(X.horizontal(i) @ C)) for i in range(I1)])
    elif n == 1:
        Z = np.stack([np.ravel(A.T @ np.asarray(X.lateral(j) @ C)) for j in range(I2)])
    else:
        Z = np.stack([np.ravel(A.T @ np.asarray(X.frontal(k) @ B)) for k in range(I3)])
    return Z @ Z.T


# --------------------------------------------------------------------------
# Core and fit
# --------------------------------------------------------------------------
def core_from_slices(X: SparseTensor3, A, B, C) -> np.ndarray:
    """G = [[X; A^T, B^T, C^T]] one horizontal slice at a time: row i of the
    J2 J3-wide intermediate is B^T X_{i::} C, then A^T is applied on mode 1
    (the appendix program's core)."""
    I1 = X.dims[0]
    J1, J2, J3 = A.shape[1], B.shape[1], C.shape[1]
    H = np.zeros((I1, J2 * J3))
    for i in range(I1):
        H[i] = np.ravel(B.T @ np.asarray(X.horizontal(i) @ C))
    return (A.T @ H).reshape(J1, J2, J3)


def core_entry(X: SparseTensor3, A, B, C, p: int, q: int, r: int) -> float:
    """One entry of G = X x_1 A^T x_2 B^T x_3 C^T (Section 3, n-mode product)
    by its definition: the sum over the (summed) nonzeros x_ijk of
    x_ijk A[i, p] B[j, q] C[k, r]."""
    return float(np.sum(X.v * A[X.i, p] * B[X.j, q] * C[X.k, r]))


def fit_slicewise(X: SparseTensor3, G, A, B, C) -> float:
    """fit = 1 - ||X - Xhat||_F / ||X||_F (Section 3, fit equation), with
    Xhat = [[G; A, B, C]] reconstructed one horizontal slice at a time:
    Xhat_{i::} = B (sum_p a_ip G_{p::}) C^T (as the appendix program does).
    Valid for any core and factors."""
    I1 = X.dims[0]
    J1 = G.shape[0]
    G1 = G.reshape(J1, -1)
    sq = []
    nx = []
    for i in range(I1):
        S = X.horizontal(i).toarray()
        H = (A[i] @ G1).reshape(G.shape[1], G.shape[2])
        R = S - B @ H @ C.T
        sq.append(float(np.sum(R * R)))
        nx.append(float(np.sum(S * S)))
    return 1.0 - math.sqrt(math.fsum(sq)) / math.sqrt(math.fsum(nx))


def fit_identity(normX2: float, G) -> float:
    """fit for orthonormal factors and the optimal core G = [[X; A^T, ...]]:
    ||X - Xhat||^2 = ||X||^2 - ||G||^2 (Pythagoras for an orthogonal
    projection)."""
    g2 = math.fsum(float(x) * float(x) for x in np.ravel(G))
    return 1.0 - math.sqrt(max(0.0, normX2 - g2)) / math.sqrt(normX2)


def fit_dense(Xd: np.ndarray, G, factors) -> float:
    """fit by brute force on a dense tensor (tiny inputs only)."""
    R = Xd - tucker_dense(G, factors)
    return 1.0 - np.sqrt(np.sum(R * R)) / np.sqrt(np.sum(Xd * Xd))


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


def _check_core(dims, J):
    if len(J) != 3 or any(int(J[n]) < 1 or int(J[n]) > dims[n] for n in range(3)):
        raise ValueError("core sizes must satisfy 1 <= J_n <= I_n")


def _fit(X, G, A, B, C, how: str, normX2: float) -> float:
    if how == "identity":
        return fit_identity(normX2, G)
    return fit_slicewise(X, G, A, B, C)


def _stop(fit_now: float, fit_prev: float, tol: float) -> bool:
    """Delta_fit(t) = fit(t) - fit(t-1) below the threshold (Section 4.2);
    tol <= 0 disables the test."""
    return tol > 0 and (fit_now - fit_prev) < tol


def hosvd(X: SparseTensor3, J, fit: str = "slices") -> Decomposition:
    """HO-SVD, Figure 1: A_n <- J_n leading eigenvectors of X_(n) X_(n)^T,
    then G <- [[X; A^T, B^T, C^T]]."""
    _check_core(X.dims, J)
    facs = [lead_eigvecs(unfolding_gram(X, n), J[n])[0] for n in range(3)]
    G = core_from_slices(X, *facs)
    f = _fit(X, G, *facs, fit, X.norm2())
    return Decomposition(G, facs, [f], 0)


def hooi(X: SparseTensor3, J, max_iters: int = 50, tol: float = 1e-4,
         init=None, fit: str = "slices") -> Decomposition:
    """HOOI, Figure 3. B, C from HO-SVD (A needs no initialisation), then
    Gauss-Seidel updates of A, B, C from U, V, W; the core and the fit are
    formed after every iteration and Delta_fit decides when to stop."""
    _check_core(X.dims, J)
    if init is None:
        B = lead_eigvecs(unfolding_gram(X, 1), J[1])[0]
        C = lead_eigvecs(unfolding_gram(X, 2), J[2])[0]
    else:
        B, C = np.array(init[1], dtype=float), np.array(init[2], dtype=float)
    A = None
    normX2 = X.norm2()
    fits = []
    prev = 0.0
    t = 0
    for t in range(1, max_iters + 1):
        A = lead_eigvecs(hooi_gram(X, 0, None, B, C), J[0])[0]
        B = lead_eigvecs(hooi_gram(X, 1, A, None, C), J[1])[0]
        C = lead_eigvecs(hooi_gram(X, 2, A, B, None), J[2])[0]
        G = core_from_slices(X, A, B, C)
        f = _fit(X, G, A, B, C, fit, normX2)
        fits.append(f)
        if _stop(f, prev, tol):
            break
        prev = f
    if A is None:
        A = lead_eigvecs(hooi_gram(X, 0, None, B, C), J[0])[0]
    G = core_from_slices(X, A, B, C)
    return Decomposition(G, [A, B, C], fits, t)


def mp(X: SparseTensor3, J, max_iters: int = 50, tol: float = 1e-4,
       init=None, fit: str = "slices") -> Decomposition:
    """Multislice Projection, Figure 7. Pseudo HO-SVD initialisation of B and
    C, then per iteration M1 -> A, M2 -> B, M3 -> C (each from the two other,
    most recent factors), the core and the fit (computed slice by slice as in
    the appendix program), and the Delta_fit test."""
    _check_core(X.dims, J)
    if init is None:
        M2, M3 = mp_init_grams(X)
        B = lead_eigvecs_of_MMt(M2, J[1])[0]
        C = lead_eigvecs_of_MMt(M3, J[2])[0]
    else:
        B, C = np.array(init[1], dtype=float), np.array(init[2], dtype=float)
    A = None
    normX2 = X.norm2()
    fits = []
    prev = 0.0
    t = 0
    for t in range(1, max_iters + 1):
        A = lead_eigvecs_of_MMt(mp_gram(X, 0, None, B, C), J[0])[0]
        B = lead_eigvecs_of_MMt(mp_gram(X, 1, A, None, C), J[1])[0]
        C = lead_eigvecs_of_MMt(mp_gram(X, 2, A, B, None), J[2])[0]
        G = core_from_slices(X, A, B, C)
        f = _fit(X, G, A, B, C, fit, normX2)
        fits.append(f)
        if _stop(f, prev, tol):
            break
        prev = f
    if A is None:
        A = lead_eigvecs_of_MMt(mp_gram(X, 0, None, B, C), J[0])[0]
    G = core_from_slices(X, A, B, C)
    return Decomposition(G, [A, B, C], fits, t)


def sp_algorithm(X: SparseTensor3, J, C0, max_iters: int = 50, tol: float = 1e-4,
                 fit: str = "slices") -> Decomposition:
    """Slice Projection, Figure 5. C0 is the random I3 x J3 start (uniform
    on [0,1), drawn by the caller); its columns are normalised here. Per
    iteration M13 -> A, M21 -> B, M32 -> C, then the core; the loop stops when
    the core stops growing, Delta_G(t) = 1 - ||G(t-1)|| / ||G(t)|| below the
    threshold (Section 4.3)."""
    _check_core(X.dims, J)
    C = np.array(C0, dtype=float)
    C = C / np.linalg.norm(C, axis=0, keepdims=True)
    normX2 = X.norm2()
    prev_norm = 0.0
    fits, growth = [], []
    t = 0
    A = B = None
    for t in range(1, max_iters + 1):
        A = lead_eigvecs_of_MMt(sp_gram(X, 0, C), J[0])[0]
        B = lead_eigvecs_of_MMt(sp_gram(X, 1, A), J[1])[0]
        C = lead_eigvecs_of_MMt(sp_gram(X, 2, B), J[2])[0]
        G = core_from_slices(X, A, B, C)
        gn = float(np.sqrt(np.sum(G * G)))
        dG = 1.0 - prev_norm / gn if gn > 0 else 0.0
        growth.append(dG)
        fits.append(_fit(X, G, A, B, C, fit, normX2))
        if tol > 0 and dG < tol:
            break
        prev_norm = gn
    G = core_from_slices(X, A, B, C)
    return Decomposition(G, [A, B, C], fits, t, {"core_growth": growth})


# --------------------------------------------------------------------------
# Comparisons
# --------------------------------------------------------------------------
def subspace_angle(A: np.ndarray, B: np.ndarray) -> float:
    """Largest principal angle between span(A) and span(B) (orthonormal
    columns), as arcsin of the norm of the part of B outside span(A); this
    form stays accurate for small angles."""
    R = B - A @ (A.T @ B)
    s = np.linalg.norm(R, 2)
    return float(np.arcsin(min(1.0, s)))


# --------------------------------------------------------------------------
# Random start (Figure 5: a random matrix with uniform entries on [0, 1],
# columns normalised to unit length)
# --------------------------------------------------------------------------
def random_start(I: int, J: int, n: int, seed: int) -> np.ndarray:
    """The I x J start of mode n drawn from SplitMix64 (Steele, Lea and
    Flood, OOPSLA 2014): entry (i, r) is the top 53 bits of output number
    (n * 2^40 + i * J + r) as a double in [0, 1); then every column is
    divided by its Euclidean norm, as Figure 5 prescribes for C."""
    from .learn import splitmix64_at
    base = n << 40
    U = np.empty((I, J))
    for i in range(I):
        for r in range(J):
            U[i, r] = (splitmix64_at(seed, base + i * J + r) >> 11) * 2.0 ** -53
    return U / np.linalg.norm(U, axis=0, keepdims=True)
