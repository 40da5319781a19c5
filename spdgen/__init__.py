"""Seeded synthetic inputs for the SPD solve A X = B (Eq. (1)-(2) of the paper).

This module only *builds inputs*: it holds none of the solver's arithmetic
(no factorisation, no substitution, no refinement).  Both the CPU oracle and
the GPU library are fed from here, so that they provably see identical bytes.

Recipes
-------
* ``logspaced(n, cond, seed)``: A = Q diag(lambda) Q^T with Q from the QR of a
  seeded N(0,1) n x n matrix (column signs fixed so diag(R) > 0) and lambda
  log-spaced from 1 to ``cond``; then A <- (A + A^T)/2 so A is exactly
  symmetric.  cond_2(A) = ``cond`` up to rounding.
* ``rhs(n, m, seed)``: X_true ~ N(0,1), column-major n x m.
* ``accurate_product(A, X)``: B = A X computed in double-double (error-free
  products by Veltkamp/Dekker splitting, pairwise TwoSum reduction), so the
  rounding of B does not pollute a forward-error check against X_true.
* Closed-form matrices used as pins: the [-1, 2, -1] tridiagonal, min(i, j),
  Hilbert, and the paper's model covariance matrix (Section 4:
  a_ij = 1/|i-j|^d off the diagonal, 1 + sqrt(i) on it, 1-based i).
* ``indefinite(n, j0, seed)``: an exactly symmetric matrix whose Cholesky
  factorisation breaks down at column j0 (1-based) with a clearly negative
  radicand.

Seeds follow ``seed_G = 2**20 * config + 2 * system`` and ``seed_X = seed_G + 1``.
Small n use numpy's PCG64 on the CPU; ``backend="torch"`` builds the same
recipe with torch on a device (Philox), used for n >= 16384 where a CPU QR
would take minutes.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "seeds", "logspaced", "logspaced_kron", "rhs", "accurate_product", "system",
    "tridiag", "minij", "hilbert", "covariance", "indefinite",
    "batch_shapes", "sha256", "SPDSystem",
]


def seeds(config: int, system: int = 0) -> tuple[int, int]:
    g = (1 << 20) * config + 2 * system
    return g, g + 1


def _eigs(n: int, cond: float, xp, **kw):
    if n == 1:
        return xp.ones(1, **kw)
    i = xp.arange(n, **kw)
    return float(cond) ** (i / (n - 1))


def logspaced(n: int, cond: float, seed: int, backend: str = "numpy", device=None):
    """A = Q diag(lambda) Q^T, lambda_i = cond^((i-1)/(n-1)); exactly symmetric."""
    if backend == "numpy":
        rng = np.random.Generator(np.random.PCG64(seed))
        G = rng.standard_normal((n, n))
        Q, R = np.linalg.qr(G)
        Q = Q * np.sign(np.diag(R))[None, :]
        lam = _eigs(n, cond, np, dtype=np.float64)
        A = (Q * lam[None, :]) @ Q.T
        A = 0.5 * (A + A.T)
        return np.asfortranarray(A)
    if backend == "torch":
        import torch
        if n * n >= 2 ** 31:
            return logspaced_kron(n, cond, seed, device=device)
        gen = torch.Generator(device=device)
        gen.manual_seed(seed)
        G = torch.randn(n, n, dtype=torch.float64, device=device, generator=gen)
        Q, R = torch.linalg.qr(G)
        del G
        Q = Q * torch.sign(torch.diagonal(R))[None, :]
        del R
        lam = _eigs(n, cond, torch, dtype=torch.float64, device=device)
        A = (Q * lam[None, :]) @ Q.T
        del Q
        A = 0.5 * (A + A.T)
        # column-major view: A is symmetric, so A.T (contiguous as A^T) has the
        # same values; callers read it with lda = n.
        return A.contiguous()
    raise ValueError(f"unknown backend {backend!r}")


def _haar(k: int, gen, device):
    """Orthogonal k x k from the QR of a seeded N(0,1) matrix, diag(R) > 0."""
    import torch
    G = torch.randn(k, k, dtype=torch.float64, device=device, generator=gen)
    Q, R = torch.linalg.qr(G)
    return Q * torch.sign(torch.diagonal(R))[None, :]


def _kron_apply(Q1, Q2, M):
    """(Q1 kron Q2) M for M of shape (a b, c): row i = i1 b + i2."""
    a, b, c = Q1.shape[0], Q2.shape[0], M.shape[1]
    T = (Q1 @ M.reshape(a, b * c)).reshape(a, b, c).transpose(0, 1).reshape(b, a * c)
    return (Q2 @ T).reshape(b, a, c).transpose(0, 1).reshape(a * b, c)


def _kron_split(n: int) -> tuple[int, int]:
    a = int(math.isqrt(n))
    while a > 1 and n % a:
        a -= 1
    if a < 2:
        raise ValueError(f"n = {n} is prime: no factorisation a b with 2 <= a <= b")
    return a, n // a


def logspaced_kron(n: int, cond: float, seed: int, device=None, chunk: int = 2048):
    """A = Q diag(lambda) Q^T with lambda log-spaced from 1 to ``cond`` as in
    ``logspaced``, for orders whose n x n arrays exceed 2^31 elements (torch's
    dense QR returned a rank-deficient Q beyond that on ROCm, so no order-n
    QR is taken).  Q = (Q1 kron Q2) P (Q3 kron Q4): Q1, Q3 of order a and Q2,
    Q4 of order b (n = a b, a the largest divisor <= sqrt(n)) from seeded
    Gaussian QRs, P a seeded permutation -- dense and orthogonal up to
    rounding, with the same eigenvalues.  A is built a block of ``chunk``
    columns at a time (A E_J = Q Lambda Q^T E_J), every intermediate below 2^31
    elements, then symmetrised exactly."""
    import torch
    a, b = _kron_split(n)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    Q1, Q2, Q3, Q4 = _haar(a, gen, device), _haar(b, gen, device), _haar(a, gen, device), _haar(b, gen, device)
    perm = torch.randperm(n, generator=gen, device=device)
    lam = _eigs(n, cond, torch, dtype=torch.float64, device=device)
    A = torch.empty(n, n, dtype=torch.float64, device=device)
    for j0 in range(0, n, chunk):
        c = min(chunk, n - j0)
        M = torch.zeros(n, c, dtype=torch.float64, device=device)
        M[torch.arange(j0, j0 + c, device=device), torch.arange(c, device=device)] = 1.0
        M = _kron_apply(Q1.T, Q2.T, M)          # K1^T E_J
        Mp = torch.empty_like(M)
        Mp[perm] = M                            # P^T
        M = _kron_apply(Q3.T, Q4.T, Mp) * lam[:, None]
        M = _kron_apply(Q3, Q4, M)[perm]        # K2, then P
        A[:, j0:j0 + c] = _kron_apply(Q1, Q2, M)
        del M, Mp
    A = 0.5 * (A + A.T)
    return A.contiguous()


def rhs(n: int, m: int, seed: int, backend: str = "numpy", device=None):
    """X_true ~ N(0,1), column-major: returned as an (m, n) row-major array whose
    row c is column c of X (so the memory layout is column-major n x m)."""
    if backend == "numpy":
        rng = np.random.Generator(np.random.PCG64(seed))
        return rng.standard_normal((m, n))
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    return torch.randn(m, n, dtype=torch.float64, device=device, generator=gen)


# --- error-free transformations for an accurate right-hand side --------------
_SPLIT = 134217729.0  # 2**27 + 1 (Veltkamp splitting constant for binary64)


def _split(a):
    c = a * _SPLIT
    hi = c - (c - a)
    return hi, a - hi


def _two_prod(a, b):
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    e = al * bl - (((p - ah * bh) - al * bh) - ah * bl)
    return p, e


def _two_sum(a, b):
    s = a + b
    bb = s - a
    e = (a - (s - bb)) + (b - bb)
    return s, e


def _dd_rowsum(hi, lo, xp):
    """Pairwise double-double reduction of hi+lo along axis 1."""
    while hi.shape[1] > 1:
        if hi.shape[1] % 2:
            z = xp.zeros_like(hi[:, :1])
            hi = xp.concatenate([hi, z], axis=1) if xp is np else xp.cat([hi, z], dim=1)
            lo = xp.concatenate([lo, z], axis=1) if xp is np else xp.cat([lo, z], dim=1)
        s, e = _two_sum(hi[:, 0::2], hi[:, 1::2])
        lo = lo[:, 0::2] + lo[:, 1::2] + e
        hi = s
    return hi[:, 0] + lo[:, 0]


def accurate_product(A, Xt, row_chunk: int | None = None):
    """B = A X in double-double, rounded once to binary64.

    ``A`` is symmetric n x n; ``Xt`` holds X column-major as (m, n).  Returns Bt
    with the same (m, n) layout.  Works on numpy arrays or torch tensors.
    """
    is_np = isinstance(A, np.ndarray)
    if is_np:
        xp = np
        out = np.empty_like(Xt)
    else:
        import torch as xp  # noqa: N813
        out = xp.empty_like(Xt)
    n = A.shape[0]
    if row_chunk is None:
        row_chunk = n if n <= 4096 else 2048
    for c in range(Xt.shape[0]):
        x = Xt[c]
        for r0 in range(0, n, row_chunk):
            blk = A[r0:r0 + row_chunk, :]
            p, e = _two_prod(blk, x[None, :])
            out[c, r0:r0 + row_chunk] = _dd_rowsum(p, e, xp)
    return out


@dataclass
class SPDSystem:
    A: np.ndarray          # n x n symmetric (column-major == row-major)
    Xt: np.ndarray         # (m, n): column c of X_true
    Bt: np.ndarray         # (m, n): column c of B = A X_true (double-double)
    cond: float
    seed_G: int
    seed_X: int

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def m(self) -> int:
        return self.Xt.shape[0]


def system(n: int, cond: float, m: int, config: int = 0, index: int = 0,
           backend: str = "numpy", device=None) -> SPDSystem:
    sg, sx = seeds(config, index)
    A = logspaced(n, cond, sg, backend=backend, device=device)
    Xt = rhs(n, m, sx, backend=backend, device=device)
    Bt = accurate_product(A, Xt)
    return SPDSystem(A, Xt, Bt, cond, sg, sx)


# --- closed-form matrices (pins) --------------------------------------------
def tridiag(n: int) -> np.ndarray:
    """The [-1, 2, -1] second-difference matrix."""
    A = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    return np.asfortranarray(A)


def minij(n: int) -> np.ndarray:
    """a_ij = min(i, j) (1-based); its Cholesky factor is the all-ones lower triangle."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.asfortranarray(np.minimum.outer(i, i))


def hilbert(n: int) -> np.ndarray:
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.asfortranarray(1.0 / (i[:, None] + i[None, :] - 1.0))


def covariance(n: int, d: float, backend: str = "numpy", device=None, chunk: int = 2048):
    """Model covariance matrix of Section 4: 1/|i-j|^d off the diagonal, 1+sqrt(i) on it (1-based i).

    The torch backend builds it on the device a block of columns at a time
    (n = 70000 in binary64 is 39 GB; the temporaries stay at n x chunk)."""
    if backend == "numpy":
        i = np.arange(1, n + 1, dtype=np.float64)
        dist = np.abs(i[:, None] - i[None, :])
        with np.errstate(divide="ignore"):
            A = 1.0 / dist ** d
        A[np.arange(n), np.arange(n)] = 1.0 + np.sqrt(i)
        return np.asfortranarray(A)
    if backend == "torch":
        import torch
        A = torch.empty(n, n, dtype=torch.float64, device=device)
        i = torch.arange(1, n + 1, dtype=torch.float64, device=device)
        # the diagonal from numpy, so that both backends give the same bits
        diag = torch.from_numpy(1.0 + np.sqrt(np.arange(1, n + 1, dtype=np.float64))).to(device)
        for c0 in range(0, n, chunk):
            c1 = min(n, c0 + chunk)
            j = i[c0:c1]
            blk = (i[:, None] - j[None, :]).abs_().pow_(d).reciprocal_()
            k = torch.arange(c0, c1, device=device)
            blk[k, k - c0] = diag[c0:c1]
            A[:, c0:c1] = blk  # symmetric: row-major storage is the column-major matrix
            del blk
        return A
    raise ValueError(f"unknown backend {backend!r}")


def covariance_cond_bound(n: int, d: int) -> float:
    """Closed-form bound on cond(covariance(n, d)) for d in {1, 2, 4}.

    The off-diagonal part is the symmetric Toeplitz matrix with symbol
    f_d(t) = 2 sum_k cos(k t) / k^d; the eigenvalues of its finite sections lie
    in [min f_d, max f_d], min f_d = f_d(pi) = -2 eta(d) (the alternating zeta:
    ln 2, pi^2/12, 7 pi^4/720) and max f_d <= 2 sum_{k<n} k^-d.  With the
    diagonal in [2, 1 + sqrt(n)]: lambda_min >= 2 - 2 eta(d) and
    lambda_max <= 1 + sqrt(n) + 2 sum_{k<n} k^-d."""
    import math
    eta = {1: math.log(2.0), 2: math.pi ** 2 / 12.0, 4: 7.0 * math.pi ** 4 / 720.0}[int(d)]
    zeta_n = sum(k ** -float(d) for k in range(1, n))
    return (1.0 + math.sqrt(n) + 2.0 * zeta_n) / (2.0 - 2.0 * eta)


def indefinite(n: int, j0: int, seed: int = 7) -> np.ndarray:
    """Symmetric A = M S M^T with M = I + N, N strictly lower triangular with
    N(0, 1/(4n)) entries (so ||N|| is about 1/2 and M is well conditioned),
    and S = diag(1,..,1,-1,1,..) with the -1 at 1-based position j0.  In exact
    arithmetic the Cholesky pivots (Schur complements) are exactly the entries
    of S: the leading j0-1 succeed with pivot 1 and column j0 has radicand -1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    M = np.eye(n) + np.tril(rng.standard_normal((n, n)) * (0.5 / np.sqrt(n)), -1)
    s = np.ones(n)
    s[j0 - 1] = -1.0
    A = (M * s[None, :]) @ M.T
    A = 0.5 * (A + A.T)
    return np.asfortranarray(A)


def batch_shapes(batch: int, config: int = 3, nmin: int = 32, nmax: int = 512,
                 logc: tuple[float, float] = (1.0, 6.0), mmax: int = 8):
    """Per-system (n, cond, m) for a batch: n ~ U{nmin..nmax}, cond = 10^U(logc), m ~ U{1..mmax}."""
    rng = np.random.Generator(np.random.PCG64((1 << 20) * config + (1 << 19)))
    ns = rng.integers(nmin, nmax + 1, size=batch)
    conds = 10.0 ** rng.uniform(logc[0], logc[1], size=batch)
    ms = rng.integers(1, mmax + 1, size=batch)
    return [(int(a), float(b), int(c)) for a, b, c in zip(ns, conds, ms)]


@dataclass
class PackedBatch:
    """A batch of systems packed for the batched entry point: A_s column-major
    n_s x n_s at a_off[s], B_s / Xt_s column-major n_s x m_s at b_off[s]."""
    n: np.ndarray
    m: np.ndarray
    cond: np.ndarray
    a_off: np.ndarray
    b_off: np.ndarray
    A: object
    B: object
    Xt: object


def packed_batch(shapes, config: int = 3, first_index: int = 0, backend: str = "numpy", device=None) -> PackedBatch:
    """Generate every system of `shapes` ((n, cond, m) per system, e.g. from
    batch_shapes) with the single-system recipe and pack them."""
    ns = np.array([s[0] for s in shapes], dtype=np.int32)
    ms = np.array([s[2] for s in shapes], dtype=np.int32)
    conds = np.array([s[1] for s in shapes], dtype=np.float64)
    a_off = np.zeros(len(shapes), dtype=np.int64)
    b_off = np.zeros(len(shapes), dtype=np.int64)
    if len(shapes):
        a_off[1:] = np.cumsum(ns.astype(np.int64) ** 2)[:-1]
        b_off[1:] = np.cumsum(ns.astype(np.int64) * ms)[:-1]
    na = int((ns.astype(np.int64) ** 2).sum())
    nbx = int((ns.astype(np.int64) * ms).sum())
    if backend == "torch":
        import torch
        A = torch.empty(na, dtype=torch.float64, device=device)
        B = torch.empty(nbx, dtype=torch.float64, device=device)
        Xt = torch.empty(nbx, dtype=torch.float64, device=device)
    else:
        A, B, Xt = np.empty(na), np.empty(nbx), np.empty(nbx)
    for s, (n, cond, m) in enumerate(shapes):
        sy = system(n, cond, m, config=config, index=first_index + s, backend=backend, device=device)
        # row-major (m, n) right-hand sides are column-major n x m already;
        # A is symmetric, so its row-major bytes are its column-major bytes
        A[a_off[s]:a_off[s] + n * n] = sy.A.reshape(-1)
        B[b_off[s]:b_off[s] + n * m] = sy.Bt.reshape(-1)
        Xt[b_off[s]:b_off[s] + n * m] = sy.Xt.reshape(-1)
    return PackedBatch(ns, ms, conds, a_off, b_off, A, B, Xt)


def packed_batch_grouped(shapes, seed: int, device="cuda") -> PackedBatch:
    """A faster generator of the same distribution for large training sets.
    Systems are reordered by n and those of equal n are drawn together: one
    seeded N(0,1) tensor per n, Q = G R^{-1} with R = chol(G^T G) (the Q of
    G's QR with positive diag(R), by batched level-3 operations),
    A = Q diag(lambda) Q^T with each system's own log-spaced spectrum,
    X_true ~ N(0,1), B = A X_true in plain binary64.  Not the per-system
    recipe of `system` (different random streams and order)."""
    import torch
    shapes = sorted(shapes, key=lambda s: s[0])
    ns = np.array([s[0] for s in shapes], dtype=np.int32)
    ms = np.array([s[2] for s in shapes], dtype=np.int32)
    conds = np.array([s[1] for s in shapes], dtype=np.float64)
    a_off = np.zeros(len(shapes), dtype=np.int64)
    b_off = np.zeros(len(shapes), dtype=np.int64)
    if len(shapes):
        a_off[1:] = np.cumsum(ns.astype(np.int64) ** 2)[:-1]
        b_off[1:] = np.cumsum(ns.astype(np.int64) * ms)[:-1]
    A = torch.empty(int((ns.astype(np.int64) ** 2).sum()), dtype=torch.float64, device=device)
    B = torch.empty(int((ns.astype(np.int64) * ms).sum()), dtype=torch.float64, device=device)
    Xt = torch.empty_like(B)
    for n in np.unique(ns):
        idx = np.nonzero(ns == n)[0]
        n = int(n)
        k = len(idx)
        gen = torch.Generator(device=device)
        gen.manual_seed((int(seed) << 12) + n)
        G = torch.randn(k, n, n, dtype=torch.float64, device=device, generator=gen)
        R = torch.linalg.cholesky(G.transpose(1, 2).contiguous() @ G, upper=True)
        Q = torch.linalg.solve_triangular(R, G, upper=True, left=False)
        i = torch.arange(n, dtype=torch.float64, device=device)
        expo = i / (n - 1) if n > 1 else torch.zeros(1, dtype=torch.float64, device=device)
        lam = torch.tensor(conds[idx], dtype=torch.float64, device=device)[:, None] ** expo[None, :]
        As = (Q * lam[:, None, :]) @ Q.transpose(1, 2).contiguous()
        As = 0.5 * (As + As.transpose(1, 2))
        A[a_off[idx[0]]:a_off[idx[-1]] + n * n] = As.reshape(-1)
        for s in idx:  # right-hand sides: per system (m varies)
            m = int(ms[s])
            X = torch.randn(m, n, dtype=torch.float64, device=device, generator=gen)
            Xt[b_off[s]:b_off[s] + n * m] = X.reshape(-1)
            B[b_off[s]:b_off[s] + n * m] = (X @ As[s - idx[0]]).reshape(-1)
    return PackedBatch(ns, ms, conds, a_off, b_off, A, B, Xt)


def sha256(arr) -> str:
    if not isinstance(arr, np.ndarray):
        arr = arr.detach().cpu().numpy()
    return hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()


def rnd_unif_rhs(n: int, m: int, seed: int) -> np.ndarray:
    """Right-hand sides with entries uniform in [0, 1], as in Section 4 of the paper; (m, n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 1.0, (m, n))


def log_uniform(lo: float, hi: float, size: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return 10.0 ** rng.uniform(math.log10(lo), math.log10(hi), size=size)
