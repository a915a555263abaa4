"""Dense test matrices with an exactly known SVD, plus Gaussian test matrices.

* ``small_matrix``: A = U diag(sigma) V^T with U, V the sign-fixed Q factors of seeded Gaussian
  matrices (the paper builds its 3000x3000 accuracy matrices from randomly drawn orthogonal factors,
  Sec. 4.1).
* ``KronMatrix``: U = U1 (x) U2 and V = V1 (x) V2, so a row of A costs two small products and the
  spectrum is exactly the multiset of the assigned values; used for the large workloads.
* ``StackedPool``: A = [A0; A0; ...; A0] (c copies) with A0 scaled by 1/sqrt(c); the singular values
  of A are exactly the target ones and every row block is a contiguous slice of a small pool.
"""
import math
import numpy as np


def orthonormal_factor(rows: int, cols: int, rng: np.random.Generator) -> np.ndarray:
    """rows x cols matrix with orthonormal columns: Q of a Gaussian matrix, signs fixed by diag(R)."""
    if cols > rows:
        raise ValueError("orthonormal_factor needs rows >= cols")
    q, r = np.linalg.qr(rng.standard_normal((rows, cols)))
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def small_matrix(m: int, n: int, sigma: np.ndarray, seed: int):
    """A = U diag(sigma) V^T; returns (A, U, sigma, V) with U m x p, V n x p, p = min(m, n)."""
    p = min(m, n)
    sigma = np.asarray(sigma, dtype=np.float64)
    if len(sigma) != p:
        raise ValueError("sigma must have min(m, n) entries")
    rng = np.random.default_rng(seed)
    U = orthonormal_factor(m, p, rng)
    V = orthonormal_factor(n, p, rng)
    A = (U * sigma) @ V.T
    return A, U, sigma, V


def low_rank_matrix(m: int, n: int, sigma: np.ndarray, seed: int):
    """A of exact rank len(sigma): U diag(sigma) V^T with orthonormal U (m x r), V (n x r)."""
    r = len(sigma)
    rng = np.random.default_rng(seed)
    U = orthonormal_factor(m, r, rng)
    V = orthonormal_factor(n, r, rng)
    return (U * np.asarray(sigma, dtype=np.float64)) @ V.T, U, np.asarray(sigma, np.float64), V


def gaussian_omega(n: int, l: int, seed: int) -> np.ndarray:
    """n x l matrix of independent standard normal draws (a caller-supplied test matrix)."""
    return np.random.default_rng(seed).standard_normal((n, l))


class KronMatrix:
    """A = (U1 (x) U2) diag(vec S) (V1 (x) V2)^T, generated row block by row block.

    m = m1*m2, n = n1*n2, U1: m1 x n1, U2: m2 x n2 (orthonormal columns), V1: n1 x n1,
    V2: n2 x n2 (orthogonal).  The n target singular values are assigned to the (a, b) index pairs
    by a seeded permutation, so sigma(A) is exactly that multiset.  Row r = r1*m2 + r2 of A,
    reshaped to n1 x n2, equals V1 @ (U1[r1,:]^T U2[r2,:] * S) @ V2^T.
    """

    def __init__(self, m1: int, m2: int, n1: int, n2: int, sigma: np.ndarray, seed: int):
        if m1 < n1 or m2 < n2:
            raise ValueError("KronMatrix needs m1 >= n1 and m2 >= n2")
        sigma = np.asarray(sigma, dtype=np.float64)
        if len(sigma) != n1 * n2:
            raise ValueError("sigma must have n1*n2 entries")
        rng = np.random.default_rng(seed)
        self.m1, self.m2, self.n1, self.n2 = m1, m2, n1, n2
        self.m, self.n = m1 * m2, n1 * n2
        self.U1 = orthonormal_factor(m1, n1, rng)
        self.U2 = orthonormal_factor(m2, n2, rng)
        self.V1 = orthonormal_factor(n1, n1, rng)
        self.V2 = orthonormal_factor(n2, n2, rng)
        perm = rng.permutation(n1 * n2)
        S = np.empty(n1 * n2)
        S[perm] = sigma
        self.S = S.reshape(n1, n2)
        self.sigma = np.sort(sigma)[::-1].copy()

    def right_vectors(self, count: int) -> np.ndarray:
        """The right singular vectors of the ``count`` largest values, n x count."""
        flat = self.S.reshape(-1)
        order = np.argsort(-flat, kind="stable")[:count]
        a, b = order // self.n2, order % self.n2
        V = np.einsum("ck,dk->cdk", self.V1[:, a], self.V2[:, b]).reshape(self.n, count)
        return V

    def _check_rows(self, r0: int, count: int):
        if r0 < 0 or count < 0 or r0 + count > self.m:
            raise ValueError(f"rows {r0} .. {r0 + count - 1} outside the matrix's {self.m} rows")

    def rows(self, r0: int, count: int) -> np.ndarray:
        """Rows r0 .. r0+count-1 in float64 (NumPy)."""
        self._check_rows(r0, count)
        r = np.arange(r0, r0 + count)
        r1, r2 = r // self.m2, r % self.m2
        M = self.U1[r1][:, :, None] * self.U2[r2][:, None, :] * self.S[None]
        out = np.einsum("ca,rab,db->rcd", self.V1, M, self.V2, optimize=True)
        return out.reshape(count, self.n)

    def rows_torch(self, r0: int, count: int, device, out=None):
        """Rows r0 .. r0+count-1 computed in float64 with torch on ``device``.

        Returns a float64 tensor, or writes float32 rows into ``out`` (count x n) when given.
        """
        import torch
        self._check_rows(r0, count)      # an index past m would be read out of bounds on the device
        cache = getattr(self, "_tcache", None)
        if cache is None or cache[0] != str(device):
            t = lambda x: torch.as_tensor(x, dtype=torch.float64, device=device)
            cache = (str(device), t(self.U1), t(self.U2), t(self.V1), t(self.V2), t(self.S))
            self._tcache = cache
        _, U1, U2, V1, V2, S = cache
        r = torch.arange(r0, r0 + count, device=device)
        r1, r2 = r // self.m2, r % self.m2
        M = U1[r1][:, :, None] * U2[r2][:, None, :] * S[None]
        X = torch.matmul(V1.unsqueeze(0), M)              # count x n1 x n2
        X = torch.matmul(X, V2.t().contiguous().unsqueeze(0))
        X = X.reshape(count, self.n)
        if out is not None:
            out.copy_(X)
            return out
        return X


class StackedPool:
    """A = [A0; ...; A0] (c copies) with A0 = KronMatrix(sigma / sqrt(c)); sigma(A) = sigma exactly.

    ``pool`` holds A0 plus its first ``ext`` rows appended again, so any block of at most ``ext``
    rows starting at any row of A is the contiguous slice pool[r0 % m0 : r0 % m0 + count].
    """

    def __init__(self, m1, m2, n1, n2, copies: int, sigma: np.ndarray, seed: int, ext: int):
        self.copies = copies
        self.base = KronMatrix(m1, m2, n1, n2, np.asarray(sigma) / math.sqrt(copies), seed)
        self.m0, self.n = self.base.m, self.base.n
        self.m = self.m0 * copies
        self.ext = ext
        self.sigma = np.sort(np.asarray(sigma, np.float64))[::-1].copy()

    def slice_bounds(self, r0: int, count: int):
        if count > self.ext:
            raise ValueError("block larger than the pool extension")
        s = r0 % self.m0
        return s, s + count

    def fill_pool(self, pool, chunk: int = 2048, device=None):
        """Write the (m0 + ext) x n pool into ``pool`` (a NumPy array or a torch tensor)."""
        total = self.m0 + self.ext
        for r0 in range(0, total, chunk):
            cnt = min(chunk, total - r0)
            src0 = r0 % self.m0
            # rows may wrap at m0; generate in at most two pieces
            first = min(cnt, self.m0 - src0)
            pieces = [(r0, src0, first)]
            if first < cnt:
                pieces.append((r0 + first, 0, cnt - first))
            for dst, src, c in pieces:
                if device is None:
                    pool[dst:dst + c] = self.base.rows(src, c)
                else:
                    pool[dst:dst + c].copy_(self.base.rows_torch(src, c, device).to(pool.dtype))
        return pool
