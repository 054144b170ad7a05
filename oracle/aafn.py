"""Dense FP64 oracle of the additive AFN preconditioner (AAFN, Sec. 2.3).

TEST INFRASTRUCTURE ONLY (see the package header): only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
use it.

Sec. 2.3 describes the preconditioner in words: landmark points chosen by
farthest point sampling (FPS) in every feature window and merged into the
(1,1) block of a 2 x 2 block partition of the regularised kernel matrix;
M is built from the Cholesky factorisation of that block and an approximate
inverse of the Schur complement.  Readings taken where the paper is silent
(each also listed in the design notes):

* FPS in window s works on the window's features in caller units.  Its first
  point is the one farthest from the window centre c0_s (the box-scaling
  centre); every further point maximises the distance to the points already
  chosen.  Ties go to the smallest index; squared distances are sums over
  the window's features in order.
* Merging: the windows' FPS lists are interleaved by rank (rank 0 of every
  window, then rank 1, ...), duplicates skipped, until max_rank points are
  taken; the landmark block holds them in ascending index order.  The rank is
  fixed by the caller (the adaptive rank estimate of the cited AFN paper is
  not described).
* The approximate inverse of the Schur complement S = K22 - K21 K11^-1 K12
  is block diagonal: the other points, ordered by the grid cell of window 0
  (tiles, then cells inside a tile; ties by index), are cut into consecutive
  blocks of at most `block` points (the fill level), and S is replaced by its
  diagonal blocks S_BB.  This is a factorised sparse approximate inverse with
  the pattern "lower triangle of the block": its factor is L_B^-1 with
  S_BB = L_B L_B^T.
* The kernel entries are those of the exact kernel (not of its trigonometric
  interpolant): M approximates Khat = sigma_f^2 sum_s K_s + sigma_eps^2 I.

With the landmarks first (order perm = [landmarks, others]):

    M = [[K11, K12], [K21, K21 K11^-1 K12 + blockdiag(S_BB)]] = F F^T,
    F = [[L11, 0], [K21 L11^-T, blockdiag(L_B)]].
"""
from __future__ import annotations

import numpy as np

# tile edge of the cell order by window dimension (64 cells in 1-D, 16 x 16
# in 2-D, 8 x 8 x 8 in 3-D)
_TILE = {1: 64, 2: 16, 3: 8}


def fps(x: np.ndarray, centre: np.ndarray, k: int) -> np.ndarray:
    """Farthest point sampling of k rows of x (n x d): the first row is the one
    farthest from `centre`, every next one maximises the distance to those
    already taken (ties: smallest index).  Stops early when every remaining
    point coincides with a chosen one."""
    n, d = x.shape
    k = min(k, n)
    if k <= 0:
        return np.zeros(0, dtype=np.int64)
    dist = np.zeros(n)
    for q in range(d):
        dist = dist + (x[:, q] - centre[q]) * (x[:, q] - centre[q])
    chosen = [int(np.argmax(dist))]
    mind = np.full(n, np.inf)
    while len(chosen) < k:
        last = x[chosen[-1]]
        dl = np.zeros(n)
        for q in range(d):
            dl = dl + (x[:, q] - last[q]) * (x[:, q] - last[q])
        mind = np.minimum(mind, dl)
        j = int(np.argmax(mind))
        if mind[j] <= 0.0:
            break
        chosen.append(j)
    return np.array(chosen, dtype=np.int64)


def landmarks(pb, per_window: int, max_rank: int) -> np.ndarray:
    """Merged landmark indices (ascending)."""
    lists = [fps(pb.X[:, w], pb.scale[s][0], per_window) for s, w in enumerate(pb.windows)]
    taken, seen = [], set()
    for r in range(max((len(v) for v in lists), default=0)):
        for v in lists:
            if r < len(v) and len(taken) < max_rank and int(v[r]) not in seen:
                seen.add(int(v[r]))
                taken.append(int(v[r]))
    return np.array(sorted(taken), dtype=np.int64)


def cell_order(pb, idx: np.ndarray) -> np.ndarray:
    """The points idx ordered by their grid cell of window 0 at bandwidth
    N_0: tile, then cell inside the tile, row-major; ties by index.  Cells
    come from t = 2N c (x - c0) + N in FP64, evaluated in that order."""
    w = pb.windows[0]
    d = len(w)
    N = pb.N[0]
    ng = 2 * N
    tb = min(_TILE[d], ng)
    nb = ng // tb
    c0, c = pb.scale[0]
    tile = np.zeros(len(idx), dtype=np.int64)
    loc = np.zeros(len(idx), dtype=np.int64)
    for q in range(d):
        t = (c * (pb.X[idx, w[q]] - c0[q])) * ng + N
        cell = np.clip(np.floor(t).astype(np.int64), 0, ng - 1)
        tile = tile * nb + cell // tb
        loc = loc * tb + cell % tb
    key = tile * tb ** d + loc
    return idx[np.argsort(key, kind="stable")]


class AAFN:
    """Dense AAFN preconditioner of the problem pb (its theta) for given
    landmark count per window, rank cap and block size."""

    def __init__(self, pb, per_window: int, max_rank: int, block: int):
        from . import dense_matrix
        n = pb.n
        self.pb = pb
        self.lm = landmarks(pb, per_window, max_rank)
        k = len(self.lm)
        rest = np.setdiff1d(np.arange(n), self.lm)
        self.ord = cell_order(pb, rest)
        self.perm = np.concatenate([self.lm, self.ord])
        self.k = k
        self.blocks = [(k + b, k + min(b + block, n - k)) for b in range(0, n - k, block)]
        Ks = [dense_matrix(pb, s) for s in range(pb.P)]
        Kd = [dense_matrix(pb, s, deriv=True) for s in range(pb.P)]
        sf, se = pb.sigma_f, pb.sigma_eps
        Kh = sf ** 2 * sum(Ks) + se ** 2 * np.eye(n)
        # derivative matrices in the order (sigma_f, ell_1..ell_P, sigma_eps)
        dK = [2 * sf * sum(Ks)] + [sf ** 2 * D for D in Kd] + [2 * se * np.eye(n)]
        p = self.perm
        self.Kh = Kh
        self.dK = dK
        Kp = Kh[np.ix_(p, p)]
        self.Mp, self.Fp = self._build(Kp)
        self.dMp = [self._dbuild(Kp, D[np.ix_(p, p)]) for D in dK]
        M = np.empty_like(self.Mp)
        M[np.ix_(p, p)] = self.Mp
        self.M = M

    def _build(self, Kp):
        k = self.k
        K11, C2 = Kp[:k, :k], Kp[k:, :k]
        L11 = np.linalg.cholesky(K11)
        V = np.linalg.solve(L11, C2.T).T                  # C2 L11^-T
        nys = V @ V.T                                     # C2 K11^-1 C2^T
        n = Kp.shape[0]
        Mp = np.zeros_like(Kp)
        Fp = np.zeros_like(Kp)
        Mp[:k, :k] = K11
        Mp[k:, :k] = C2
        Mp[:k, k:] = C2.T
        Mp[k:, k:] = nys
        Fp[:k, :k] = L11
        Fp[k:, :k] = V
        for b0, b1 in self.blocks:
            S = Kp[b0:b1, b0:b1] - nys[b0 - k:b1 - k, b0 - k:b1 - k]
            Mp[b0:b1, b0:b1] += S
            Fp[b0:b1, b0:b1] = np.linalg.cholesky(S)
        assert Mp.shape == (n, n)
        return Mp, Fp

    def _dbuild(self, Kp, Dp):
        """dM in the landmark-first order for the derivative matrix Dp of Khat."""
        k = self.k
        K11, C2 = Kp[:k, :k], Kp[k:, :k]
        D11, D2 = Dp[:k, :k], Dp[k:, :k]
        A = np.linalg.solve(K11, C2.T)                    # K11^-1 C2^T
        dnys = D2 @ A + A.T @ D2.T - A.T @ D11 @ A
        dM = np.zeros_like(Kp)
        dM[:k, :k] = D11
        dM[k:, :k] = D2
        dM[:k, k:] = D2.T
        dM[k:, k:] = dnys
        for b0, b1 in self.blocks:
            dM[b0:b1, b0:b1] += Dp[b0:b1, b0:b1] - dnys[b0 - k:b1 - k, b0 - k:b1 - k]
        return dM

    # ---- quantities in the original point order
    def logdet(self) -> float:
        return 2.0 * float(np.sum(np.log(np.diag(self.Fp))))

    def solve(self, V):
        """M^-1 V."""
        return np.linalg.solve(self.M, V)

    def factor(self, xi):
        """F xi (a sample with covariance M when xi has identity covariance)."""
        out = np.empty_like(xi)
        out[self.perm] = self.Fp @ xi[self.perm]
        return out

    def factor_invt(self, xi):
        """F^-T xi (= M^-1 F xi)."""
        out = np.empty_like(xi)
        out[self.perm] = np.linalg.solve(self.Fp.T, xi[self.perm])
        return out

    def dlogdet(self) -> np.ndarray:
        """tr(M^-1 dM/dtheta_j) for theta = (sigma_f, ell_1..ell_P, sigma_eps)."""
        Mi = np.linalg.inv(self.Mp)
        return np.array([float(np.sum(Mi * D)) for D in self.dMp])

    def dquad(self, W) -> np.ndarray:
        """w_c^T (dM/dtheta_j) w_c, shape (P + 2, columns)."""
        W = np.asarray(W, dtype=np.float64).reshape(self.pb.n, -1)
        Wp = W[self.perm]
        return np.array([np.sum(Wp * (D @ Wp), axis=0) for D in self.dMp])


def pcg(matvec, psolve, B, tol, maxit):
    """Preconditioned CG per column from a zero start (stop: ||r|| <= tol ||b||).
    Returns X, iteration counts and per column the (alpha, beta) list."""
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    n, kc = B.shape
    X = np.zeros_like(B)
    its = np.zeros(kc, dtype=np.int64)
    hist = [[] for _ in range(kc)]
    for c in range(kc):
        b = B[:, c]
        x = np.zeros(n)
        r = b.copy()
        z = psolve(r)
        p = z.copy()
        rz = r @ z
        nb = np.sqrt(b @ b)
        it = 0
        while it < maxit and np.sqrt(r @ r) > tol * nb:
            Ap = matvec(p)
            a = rz / (p @ Ap)
            x += a * p
            r -= a * Ap
            z = psolve(r)
            rz_new = r @ z
            beta = rz_new / rz
            hist[c].append((a, beta))
            p = z + beta * p
            rz = rz_new
            it += 1
        X[:, c] = x
        its[c] = it
    return X, its, hist
