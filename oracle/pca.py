"""Algorithm 4 (single-pass PCA) and Algorithm 1 (basic randomised SVD), plain FP64.

Test infrastructure only (see the package docstring).  Notation follows the paper: A is m x n and
row-major, Omega is n x l with l = t*b, G = A Omega (m x l), H = A^T G (n x l), Q (m x l) and
B (l x n) are built one column block of width b at a time.
"""
from dataclasses import dataclass, field
import numpy as np
from scipy.linalg import solve_triangular


@dataclass
class PCAResult:
    S: np.ndarray                 # k singular values, descending, zero-padded past the rank
    V: np.ndarray                 # n x k right singular vectors (principal components)
    U: np.ndarray                 # m x k left singular vectors (None when not requested)
    rank: int                     # number of basis vectors kept (l unless the guard stopped early)
    G: np.ndarray = None
    H: np.ndarray = None
    Q: np.ndarray = None
    B: np.ndarray = None
    R: list = field(default_factory=list)


def _qr_nonneg(X):
    """Economy QR without pivoting (the paper's qr(X,0), Sec. 2.2), normalised so diag(R) >= 0."""
    Q, R = np.linalg.qr(X, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d, R * d[:, None]


def sketch_pass(blocks, Omega):
    """The single pass of Algorithm 4 (steps 3-8) and Eq. (10).

    For each block a of consecutive rows: g = a Omega is appended to G, and H accumulates a^T g,
    so that H = sum over rows of a_r^T g_r = A^T G.  Each block is converted to FP64 on arrival,
    as the paper does with its single-precision files (Sec. 4.2).
    """
    Omega = np.asarray(Omega, dtype=np.float64)
    n, l = Omega.shape
    H = np.zeros((n, l))
    G_parts = []
    for a in blocks:
        a = np.asarray(a, dtype=np.float64)
        if a.ndim != 2 or a.shape[1] != n:
            raise ValueError("every row block must have n columns")
        g = a @ Omega
        G_parts.append(g)
        H += a.T @ g
    G = np.vstack(G_parts) if G_parts else np.zeros((0, l))
    return G, H


def qb_from_sketch(G, H, Omega, b, tau=1e-10):
    """The column-block loop of Algorithm 4 (steps 9-15) with the re-orthogonalisation of Sec. 3.2.

    For i = 1..t, on columns c = (i-1)b+1 : ib:
      Y_i = G(:,c) - Q (B Omega_i)                        (first iteration: Q, B empty, term dropped)
      [Q_i, R_i] = qr(Y_i)
      [Q_i, R~_i] = qr(Q_i - Q (Q^T Q_i))                 (Eq. 7)
      R_i = R~_i R_i
      B_i = R_i^{-T} (H(:,c)^T - Y_i^T Q B - Omega_i^T B^T B)   (Eq. 9)
      Q = [Q, Q_i];  B = [B; B_i]
    Rank guard (a reading; the paper assumes full-rank sketches, Sec. 3.1 proof): with r0 the first
    diagonal entry of the first combined R, keep only the leading columns of a block whose combined
    R diagonal exceeds tau*r0, and stop the loop at the first block that loses a column.
    Returns (Q, B, rank, R_list).
    """
    G = np.asarray(G, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    Omega = np.asarray(Omega, dtype=np.float64)
    m, l = G.shape
    n = H.shape[0]
    if l % b != 0:
        raise ValueError("l must be a multiple of b")
    t = l // b
    Q = np.zeros((m, 0))
    B = np.zeros((0, n))
    R_list = []
    r0 = None
    for i in range(t):
        c = np.arange(i * b, (i + 1) * b)
        Omega_i = Omega[:, c]
        Y = G[:, c] - Q @ (B @ Omega_i)
        Qi, Ri = _qr_nonneg(Y)
        Qi, Rt = _qr_nonneg(Qi - Q @ (Q.T @ Qi))
        Ri = Rt @ Ri
        if r0 is None:
            r0 = Ri[0, 0]
        d = np.abs(np.diag(Ri))
        keep = 0
        while keep < len(c) and d[keep] > tau * r0:
            keep += 1
        if keep < len(c):
            c, Qi, Ri, Y = c[:keep], Qi[:, :keep], Ri[:keep, :keep], Y[:, :keep]
        if keep > 0:
            numer = H[:, c].T - (Y.T @ Q) @ B - (B @ Omega[:, c]).T @ B
            Bi = solve_triangular(Ri.T, numer, lower=True)
            Q = np.hstack([Q, Qi])
            B = np.vstack([B, Bi])
            R_list.append(Ri)
        if keep < b:
            break
    return Q, B, Q.shape[1], R_list


def apply_sign_convention(U, V):
    """Flip each (u_j, v_j) pair so the largest-magnitude entry of v_j is positive.

    The paper leaves singular-vector signs open; this reading breaks ties by the lowest index.
    """
    V = V.copy()
    U = None if U is None else U.copy()
    for j in range(V.shape[1]):
        col = V[:, j]
        if not np.any(col):
            continue
        p = int(np.argmax(np.abs(col)))
        if col[p] < 0:
            V[:, j] = -col
            if U is not None:
                U[:, j] = -U[:, j]
    return U, V


def svd_from_qb(Q, B, k, want_u=True):
    """Steps 16-19 of Algorithm 4: [U~, S, V] = svd(B), U = Q U~, keep the first k.

    Columns past the computed rank are returned as zeros.
    """
    m, r = Q.shape
    n = B.shape[1]
    S = np.zeros(k)
    V = np.zeros((n, k))
    U = np.zeros((m, k)) if want_u else None
    if r > 0:
        Ut, s, Vt = np.linalg.svd(B, full_matrices=False)
        kk = min(k, len(s))
        S[:kk] = s[:kk]
        V[:, :kk] = Vt[:kk].T
        if want_u:
            U[:, :kk] = Q @ Ut[:, :kk]
    U, V = apply_sign_convention(U, V)
    return S, U, V


def single_pass_pca(blocks, Omega, k, b, tau=1e-10, want_u=True, keep_state=False):
    """Algorithm 4 end to end on an iterable of row blocks (the rows of A in order)."""
    Omega = np.asarray(Omega, dtype=np.float64)
    l = Omega.shape[1]
    if not (1 <= k <= l):
        raise ValueError("need 1 <= k <= l")
    G, H = sketch_pass(blocks, Omega)
    Q, B, rank, Rs = qb_from_sketch(G, H, Omega, b, tau)
    S, U, V = svd_from_qb(Q, B, k, want_u)
    res = PCAResult(S=S, V=V, U=U, rank=rank)
    if keep_state:
        res.G, res.H, res.Q, res.B, res.R = G, H, Q, B, Rs
    return res


def basic_randqb_svd(A, Omega, k, want_u=True):
    """Algorithm 1 (two passes over A): Q = orth(A Omega), B = Q^T A, svd(B), U = Q U~."""
    A = np.asarray(A, dtype=np.float64)
    Q, _ = _qr_nonneg(A @ Omega)
    B = Q.T @ A
    S, U, V = svd_from_qb(Q, B, k, want_u)
    return PCAResult(S=S, V=V, U=U, rank=Q.shape[1], Q=Q, B=B)


def power_omega(H):
    """The power scheme with P = 1 for Algorithm 4 (Sec. 2.2, last paragraph of Sec. 3.3, and the
    P = 1 runs after Table 1 in Sec. 4.2): the second pass uses Omega replaced by orth(H).

    orth(H) is the Q factor of an economy QR of H (Sec. 2.2, diag R >= 0).  Reading: it is scaled
    by sqrt(n), so its entries keep the unit variance of the Gaussian Omega; Algorithm 4 depends on
    Omega only through its column span, so the scale changes no result in exact arithmetic.
    """
    H = np.asarray(H, dtype=np.float64)
    Q, _ = _qr_nonneg(H)
    return np.sqrt(H.shape[0]) * Q


def single_pass_pca_power(blocks, Omega, k, b, tau=1e-10, want_u=True, keep_state=False,
                          centred=False):
    """Algorithm 4 with one power iteration (P = 1): a first pass gives H = A^T A Omega, then the
    pass and the column-block loop run again with Omega_2 = power_omega(H) (two passes over A in
    all).  `blocks` is a list of row blocks (it is read twice).  The result carries Omega_2.
    With centred=True both passes act on the column-centred matrix (centred implicitly, as in
    single_pass_pca_centred), so Omega_2 = power_omega(A_c^T A_c Omega)."""
    blocks = list(blocks)
    if centred:
        G1, H1, s_A, s_G, m = sketch_pass_centred(blocks, Omega)
        _, H1, _ = centre_sketch(G1, H1, Omega, s_A, s_G, m)
        Om2 = power_omega(H1)
        res = single_pass_pca_centred(blocks, Om2, k, b, tau, want_u, keep_state)
    else:
        _, H1 = sketch_pass(blocks, Omega)
        Om2 = power_omega(H1)
        res = single_pass_pca(blocks, Om2, k, b, tau, want_u, keep_state)
    res.Omega = Om2
    return res


def sketch_pass_centred(blocks, Omega):
    """The single pass with the column sums needed for implicit centring (PCA of a centred A,
    Sec. 2.1, where the data is assumed centred).  Besides G and H (Eq. 10) it returns
    s_A = A^T 1 (n) and s_G = G^T 1 (l), both sums over all rows, and the row count m."""
    blocks = [np.asarray(a, dtype=np.float64) for a in blocks]
    G, H = sketch_pass(blocks, Omega)
    n = np.asarray(Omega).shape[0]
    s_A = np.zeros(n)
    for a in blocks:
        s_A += a.sum(axis=0)
    s_G = G.sum(axis=0)
    return G, H, s_A, s_G, G.shape[0]


def centre_sketch(G, H, Omega, s_A, s_G, m):
    """The sketch of the column-centred matrix A_c = A - 1 mu^T, mu = s_A / m, from the sketch of A:

      G_c = A_c Omega   = G - 1 (Omega^T mu)^T
      H_c = A_c^T G_c   = H - s_A w^T - mu s_G^T + m mu w^T = H - mu s_G^T   (w = Omega^T mu,
                                                                             s_A = m mu)
    so the centred PCA stays single-pass."""
    Omega = np.asarray(Omega, dtype=np.float64)
    mu = np.asarray(s_A, dtype=np.float64) / m
    w = Omega.T @ mu
    Gc = np.asarray(G, dtype=np.float64) - w[None, :]
    Hc = np.asarray(H, dtype=np.float64) - np.outer(mu, np.asarray(s_G, dtype=np.float64))
    return Gc, Hc, mu


def single_pass_pca_centred(blocks, Omega, k, b, tau=1e-10, want_u=True, keep_state=False):
    """Algorithm 4 on the column-centred matrix, centred implicitly: one pass with column sums,
    the sketch corrected by centre_sketch, then the column-block loop and SVD as usual.  U holds
    the left singular vectors of A_c.  The result carries mu."""
    G, H, s_A, s_G, m = sketch_pass_centred(blocks, Omega)
    if m == 0:
        return single_pass_pca([], Omega, k, b, tau, want_u, keep_state)
    Gc, Hc, mu = centre_sketch(G, H, Omega, s_A, s_G, m)
    Q, B, rank, Rs = qb_from_sketch(Gc, Hc, Omega, b, tau)
    S, U, V = svd_from_qb(Q, B, k, want_u)
    res = PCAResult(S=S, V=V, U=U, rank=rank)
    res.mu = mu
    if keep_state:
        res.G, res.H, res.Q, res.B, res.R = Gc, Hc, Q, B, Rs
    return res
