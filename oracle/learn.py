"""FP64 oracle of the learned warm start (test infrastructure only).

The paper starts HOOI from the HO-SVD factors and MP from its pseudo HO-SVD
(Sections 4.2 and 4.4); it has no learned start. This module is the plain
reference for the learned start that the GPU library offers beside them:

1. a Gaussian sketch of every mode-n unfolding, S = X_(n) Omega, whose
   entries come from a counter-based generator of the two other coordinates
   (SplitMix64, Steele, Lea and Flood, OOPSLA 2014, with the Box-Muller
   transform), so that no random matrix is stored;
2. row features: each sketch row divided by its norm rho_i;
3. a two-layer perceptron applied to every row, R_i = rho_i (W2^T relu(W1^T
   s_i + b1) + b2);
4. the start factor: the leading J-dimensional subspace of H_n = X_(n)
   X_(n)^T within the span of the first K = min(128, 2J) network outputs
   (Rayleigh-Ritz on an orthonormal basis Q of span(R[:, :K]));
5. training: a subspace-alignment loss that asks span(R[:, :K]) to contain
   converged factors A*, L = 1 - tr(B^T C^-1 B) / J with C = Rk^T Rk + lam I
   (lam held fixed) and B = Rk^T A*, its gradient, written out by hand, and
   the backward pass of the perceptron.

Every step is written out in FP64 NumPy; the tests pin them against central
finite differences, dense brute force and the generator's published test
vector.
"""
import numpy as np

__all__ = [
    "GAMMA", "splitmix64", "splitmix64_at", "sketch_omega", "sketch_dense_omega", "sketch",
    "row_features", "N_IN", "N_HID", "N_OUT", "param_count", "unpack", "mlp_forward",
    "mlp_backward", "align_loss", "start_factor", "bf16_round", "round_weights", "test_width",
]

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
N_IN, N_HID, N_OUT = 64, 128, 128


def _mix(z: int) -> int:
    """SplitMix64 output function (the variant-13 finaliser of MurmurHash3)."""
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def splitmix64(seed: int, count: int):
    """The first `count` outputs of SplitMix64 seeded with `seed`: the state
    advances by the golden gamma before each output."""
    out, s = [], seed & MASK
    for _ in range(count):
        s = (s + GAMMA) & MASK
        out.append(_mix(s))
    return out


def splitmix64_at(seed: int, k: int) -> int:
    """Output number k (0-based) of SplitMix64 seeded with `seed`."""
    return _mix((seed + (k + 1) * GAMMA) & MASK)


def _unit(x: int) -> float:
    """Top 53 bits as a double in [0, 1)."""
    return (x >> 11) * 2.0 ** -53


def sketch_omega(seed: int, n: int, lin: int) -> np.ndarray:
    """Row `lin` of the mode-n sketch matrix Omega (N_IN Gaussian entries).
    lin = i_a * I_b + i_b is the linear index of the two other coordinates
    (a = n+1, b = n+2 mod 3). Entries 2q, 2q+1 are one Box-Muller pair from
    outputs k = ((n * 2^40 + lin) * 64 + 2q + h), h = 0, 1: u1 = 1 - unit(k0)
    in (0, 1], u2 = unit(k1), r = sqrt(-2 ln u1), angle 2 pi u2."""
    row = np.empty(N_IN)
    base = ((n << 40) + lin) * 64
    for q in range(N_IN // 2):
        u1 = 1.0 - _unit(splitmix64_at(seed, base + 2 * q))
        u2 = _unit(splitmix64_at(seed, base + 2 * q + 1))
        r = np.sqrt(-2.0 * np.log(u1))
        row[2 * q] = r * np.cos(2.0 * np.pi * u2)
        row[2 * q + 1] = r * np.sin(2.0 * np.pi * u2)
    return row


def sketch_dense_omega(seed: int, n: int, dims) -> np.ndarray:
    """The whole Omega for mode n as a dense (I_a * I_b) x N_IN matrix (tiny
    tensors only)."""
    a, b = (n + 1) % 3, (n + 2) % 3
    return np.stack([sketch_omega(seed, n, lin) for lin in range(dims[a] * dims[b])])


def sketch(idx, vals, dims, n: int, seed: int) -> np.ndarray:
    """S = X_(n) Omega, I_n x N_IN: every nonzero adds its value times the
    Omega row of its two other coordinates to row i_n (duplicates add up, as
    in the summed tensor)."""
    a, b = (n + 1) % 3, (n + 2) % 3
    S = np.zeros((dims[n], N_IN))
    lin = idx[a].astype(np.int64) * dims[b] + idx[b].astype(np.int64)
    cache = {}
    for p in range(len(vals)):
        key = int(lin[p])
        if key not in cache:
            cache[key] = sketch_omega(seed, n, key)
        S[int(idx[n][p])] += float(vals[p]) * cache[key]
    return S


def row_features(S: np.ndarray):
    """(S_i / rho_i, rho_i) with rho_i = ||S_i||; zero rows stay zero."""
    rho = np.sqrt((S * S).sum(axis=1))
    F = np.zeros_like(S)
    nz = rho > 0
    F[nz] = S[nz] / rho[nz, None]
    return F, rho


def param_count() -> int:
    return N_IN * N_HID + N_HID + N_HID * N_OUT + N_OUT


def unpack(theta: np.ndarray):
    """Flat parameters -> (W1 [N_IN x N_HID], b1, W2 [N_HID x N_OUT], b2)."""
    o = 0
    W1 = theta[o:o + N_IN * N_HID].reshape(N_IN, N_HID); o += N_IN * N_HID
    b1 = theta[o:o + N_HID]; o += N_HID
    W2 = theta[o:o + N_HID * N_OUT].reshape(N_HID, N_OUT); o += N_HID * N_OUT
    b2 = theta[o:o + N_OUT]
    return W1, b1, W2, b2


def mlp_forward(F: np.ndarray, rho: np.ndarray, theta: np.ndarray):
    """R = diag(rho) (relu(F W1 + b1) W2 + b2); also returns Z1 = F W1 + b1."""
    W1, b1, W2, b2 = unpack(np.asarray(theta, dtype=float))
    Z1 = F @ W1 + b1
    H = np.maximum(Z1, 0.0)
    R = rho[:, None] * (H @ W2 + b2)
    return R, Z1


def mlp_backward(F: np.ndarray, rho: np.ndarray, theta: np.ndarray, Z1: np.ndarray, dR: np.ndarray) -> np.ndarray:
    """Gradient of a scalar with respect to the flat parameters, given its
    gradient dR with respect to R (chain rule through each step of
    mlp_forward, in reverse)."""
    W1, b1, W2, b2 = unpack(np.asarray(theta, dtype=float))
    dZ2 = rho[:, None] * dR              # R = rho * Z2
    H = np.maximum(Z1, 0.0)
    dW2 = H.T @ dZ2                      # Z2 = H W2 + b2
    db2 = dZ2.sum(axis=0)
    dH = dZ2 @ W2.T
    dZ1 = dH * (Z1 > 0)                  # H = relu(Z1)
    dW1 = F.T @ dZ1                      # Z1 = F W1 + b1
    db1 = dZ1.sum(axis=0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2])


def test_width(J: int) -> int:
    """K = min(128, 2J): columns of the network output that span the test
    subspace of a rank-J start."""
    return min(N_OUT, 2 * J)


def align_loss(R: np.ndarray, K: int, A: np.ndarray, lam: float):
    """L = 1 - tr(B^T C^-1 B) / J, C = Rk^T Rk + lam I, B = Rk^T A, Rk the
    first K columns of R and A (n x J) with orthonormal columns: for lam = 0,
    the mean squared sine of the principal angles between span(A) and its
    projection on span(Rk); 0 when span(Rk) contains span(A). Gradient (lam
    held fixed): dL/dRk = -(2/J) (A - Rk C^-1 B) (C^-1 B)^T, zero for the
    other columns. Returns (L, dR)."""
    J = A.shape[1]
    Rk = R[:, :K]
    C = Rk.T @ Rk + lam * np.eye(K)
    B = Rk.T @ A
    CB = np.linalg.solve(C, B)
    L = 1.0 - np.trace(B.T @ CB) / J
    dR = np.zeros_like(R)
    dR[:, :K] = -(2.0 / J) * (A - Rk @ CB) @ CB.T
    return L, dR


def start_factor(R: np.ndarray, H: np.ndarray, J: int):
    """Rayleigh-Ritz of H on span(R[:, :K]), K = test_width(J): Q = an
    orthonormal basis of that span (from the eigenpairs of Rk^T Rk), the J
    leading eigenpairs (theta, V) of Q^T H Q, start = Q V with canonical
    signs. Returns (start, theta, eigenvalues of Rk^T Rk)."""
    K = test_width(J)
    Rk = R[:, :K]
    g, W = np.linalg.eigh(Rk.T @ Rk)
    g, W = g[::-1], W[:, ::-1]
    Q = Rk @ W / np.sqrt(g)
    th, V = np.linalg.eigh(Q.T @ H @ Q)
    th, V = th[::-1][:J], V[:, ::-1][:, :J]
    U = Q @ V
    for c in range(J):
        if U[np.argmax(np.abs(U[:, c])), c] < 0:
            U[:, c] = -U[:, c]
    return U, th, g


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (8-bit significand, ties
    to even) and return them as float64: the upper 16 bits of the float32
    pattern after adding 0x7FFF plus the lowest kept bit (finite inputs)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def round_weights(theta: np.ndarray) -> np.ndarray:
    """The parameters as the network uses them: W1 and W2 rounded to
    bfloat16, the biases kept (FP32 values)."""
    W1, b1, W2, b2 = unpack(np.asarray(theta, dtype=np.float32).astype(np.float64))
    return np.concatenate([bf16_round(W1).ravel(), b1, bf16_round(W2).ravel(), b2])
