"""Oracle of the learned precision picker -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; it shares no code with the GPU library.

The paper has no picker: this is the project's own addition around
Algorithm 1 (which precision to run it in, with plain binary64 Cholesky as
the fallback).  Everything here is written from its definition in binary64
NumPy, with no blocking or reordering:

* ``features(A, m)``: the 16 per-system features (below);
* ``mlp_forward`` / ``mlp_loss_grad``: a 16 -> 64 -> 64 -> 4 perceptron with
  ReLU hidden layers and softmax cross-entropy (mean over the samples);
* ``adam_step``: one step of Adam (Kingma and Ba, 2015, Algorithm 1 of that
  paper), bias-corrected moments;
* ``label``: the cheapest precision whose run converged (ties within 2 %
  go to the higher precision).

Features of an n x n SPD matrix A (lower triangle read) and m right-hand
sides.  d_i = a_ii^{-1/2} (1 where a_ii <= 0), H = D A D,
r_i = sum_{j != i} |h_ij| (Gershgorin radius).  Lanczos: K = 4 steps on H
from v_1 = (1, ..., 1)/sqrt(n) without reorthogonalisation, stopping early if
some beta_k <= 1e-12 * alpha-scale; theta = eigenvalues of the resulting
tridiagonal T (ascending).
   f0  log2(n) / 9                  f8  clip(1 - max r_i, -10, 1) / 10
   f1  m / 8                        f9  log10(theta_max) / 3
   f2  log10(max a_ii/min a_ii) / 6 f10 log10(max(theta_min, 1e-16)) / 6
   f3  mean(log10 a_ii) / 6         f11 log10(theta_max / max(theta_min, 1e-16)) / 6
   f4  std(log10 a_ii) / 3          f12 max_{i != j} |h_ij|
   f5  log10(1 + max r_i) / 3       f13 log10(||H||_F / sqrt(n)) / 3
   f6  log10(1 + mean r_i) / 3      f14 beta_last / theta_max (0 after an early stop)
   f7  fraction of rows, r_i < 1    f15 (theta_2 - theta_1) / (theta_max - theta_1) (0 if K < 3)
(log10 a_ii uses |a_ii| floored at 1e-300.)
"""
from __future__ import annotations

import numpy as np

NFEAT, NH, NCLS = 16, 64, 4
NPARAM = NH * NFEAT + NH + NH * NH + NH + NCLS * NH + NCLS  # 5508
LANCZOS_K = 4
PREC_CLASSES = ("bf16", "fp16", "fp32", "fp64")


def _sym(A):
    """The symmetric matrix whose lower triangle is that of A."""
    L = np.tril(A)
    return L + np.tril(A, -1).T


def lanczos(H, v1, k):
    """Plain Lanczos (no reorthogonalisation): (alpha, beta) of T_k."""
    alpha, beta = [], []
    v_prev = np.zeros_like(v1)
    v = v1.copy()
    b_prev = 0.0
    for j in range(k):
        w = H @ v
        a = float(w @ v)
        alpha.append(a)
        w = w - a * v - b_prev * v_prev
        b = float(np.sqrt(w @ w))
        if j == k - 1:
            beta.append(b)
            break
        if b <= 1e-12 * max(abs(a), 1.0):
            beta.append(0.0)
            break
        beta.append(b)
        v_prev, v = v, w / b
        b_prev = b
    return np.array(alpha), np.array(beta)


def ritz_values(alpha, beta):
    """Eigenvalues (ascending) of the tridiagonal with diagonal alpha and
    off-diagonal beta[:-1]."""
    k = len(alpha)
    T = np.diag(alpha)
    for i in range(k - 1):
        T[i, i + 1] = T[i + 1, i] = beta[i]
    return np.linalg.eigvalsh(T)


def features(A, m):
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    S = _sym(A)
    a = np.diag(S).copy()
    d = np.where(a > 0, 1.0 / np.sqrt(np.where(a > 0, a, 1.0)), 1.0)
    H = (d[:, None] * S) * d[None, :]
    off = H - np.diag(np.diag(H))
    r = np.abs(off).sum(axis=1)
    la = np.log10(np.maximum(np.abs(a), 1e-300))
    alpha, beta = lanczos(H, np.ones(n) / np.sqrt(n), LANCZOS_K)
    th = ritz_values(alpha, beta)
    tmin, tmax = th[0], th[-1]
    f = np.zeros(NFEAT)
    f[0] = np.log2(n) / 9
    f[1] = m / 8
    f[2] = (la.max() - la.min()) / 6
    f[3] = la.mean() / 6
    f[4] = la.std() / 3
    f[5] = np.log10(1 + r.max()) / 3
    f[6] = np.log10(1 + r.mean()) / 3
    f[7] = np.mean(r < 1)
    f[8] = np.clip(1 - r.max(), -10, 1) / 10
    f[9] = np.log10(tmax) / 3
    f[10] = np.log10(max(tmin, 1e-16)) / 6
    f[11] = np.log10(tmax / max(tmin, 1e-16)) / 6
    f[12] = np.abs(off).max() if n > 1 else 0.0
    f[13] = np.log10(np.sqrt((H * H).sum()) / np.sqrt(n)) / 3
    early = len(alpha) < LANCZOS_K
    f[14] = 0.0 if early else beta[-1] / tmax
    f[15] = (th[1] - th[0]) / (tmax - th[0]) if len(th) >= 3 and tmax > th[0] else 0.0
    return f


# ---- the perceptron ---------------------------------------------------------
def unpack(p):
    """Parameter vector -> (W1 (64x16), b1, W2 (64x64), b2, W3 (4x64), b3), row-major [out][in]."""
    p = np.asarray(p, dtype=np.float64)
    o = 0
    out = []
    for shape in ((NH, NFEAT), (NH,), (NH, NH), (NH,), (NCLS, NH), (NCLS,)):
        k = int(np.prod(shape))
        out.append(p[o:o + k].reshape(shape))
        o += k
    assert o == NPARAM
    return out


def mlp_forward(p, X):
    """Logits (N x 4) for features X (N x 16)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    h1 = np.maximum(X @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ W3.T + b3


def mlp_loss_grad(p, X, y):
    """Mean softmax cross-entropy over the samples and its gradient (flat, like p)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[0]
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ W3.T + b3
    zmax = z3.max(axis=1, keepdims=True)
    e = np.exp(z3 - zmax)
    P = e / e.sum(axis=1, keepdims=True)
    loss = float(np.mean(-np.log(P[np.arange(N), y])))
    g3 = P.copy()
    g3[np.arange(N), y] -= 1.0
    g3 /= N
    gW3 = g3.T @ h2
    gb3 = g3.sum(axis=0)
    g2 = (g3 @ W3) * (z2 > 0)
    gW2 = g2.T @ h1
    gb2 = g2.sum(axis=0)
    g1 = (g2 @ W2) * (z1 > 0)
    gW1 = g1.T @ X
    gb1 = g1.sum(axis=0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, grad


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t >= 1); returns new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def label(converged, cost):
    """Index of the cheapest converged precision (classes ordered BF16, FP16,
    FP32, FP64); among precisions within 2 % of the cheapest, the highest."""
    cand = [k for k in range(NCLS) if converged[k]]
    if not cand:
        return NCLS - 1
    best = min(cost[k] for k in cand)
    return max(k for k in cand if cost[k] <= 1.02 * best)
