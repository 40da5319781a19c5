"""Pins of the picker oracle (CPU): features against closed forms, the
perceptron's gradient against central differences and a hand-expanded
two-layer case, Adam against its closed form, the label rule."""
import math

import numpy as np
import pytest

import spdgen
from oracle import picker as pk


def test_parameter_count():
    assert pk.NPARAM == 5508


def test_features_identity_and_diagonal():
    n = 40
    f = pk.features(np.eye(n), 3)
    assert f[0] == pytest.approx(math.log2(n) / 9)
    assert f[1] == pytest.approx(3 / 8)
    # H = I: no spread, no off-diagonal, Lanczos stops after one step at theta = 1
    assert np.allclose(f[2:7], 0) and f[7] == 1 and f[8] == pytest.approx(0.1)
    assert np.allclose(f[9:], 0)
    # a diagonal matrix equilibrates to I; only the diagonal statistics move
    lam = np.logspace(0, 4, n)
    g = pk.features(np.diag(lam), 1)
    assert g[2] == pytest.approx(4 / 6)
    assert g[3] == pytest.approx(np.mean(np.log10(lam)) / 6)
    assert g[4] == pytest.approx(np.std(np.log10(lam)) / 3)
    assert np.allclose(g[5:7], 0) and np.allclose(g[9:], 0)


def test_features_tridiagonal_closed_form():
    # 2 [-1, 2, -1] (diagonal 4, so d = 1/2 and H = I - (1/2) offdiag exactly):
    # r_i = 1 inside, 1/2 at the ends;
    # ones/sqrt(n) is reversal-symmetric, so Lanczos only sees the symmetric
    # eigenvectors: for n = 6 and K >= 3 the Ritz values are exactly
    # 1 - cos(k pi / 7), k = 1, 3, 5 (K = 4 stops early at the third step)
    n = 6
    A = 2.0 * spdgen.tridiag(n)
    f = pk.features(A, 1)
    assert f[7] == pytest.approx(2 / n)
    assert f[12] == pytest.approx(0.5)
    assert f[13] == pytest.approx(math.log10(math.sqrt(n + 2 * (n - 1) / 4) / math.sqrt(n)) / 3)
    th = sorted(1 - math.cos(k * math.pi / 7) for k in (1, 3, 5))
    assert f[9] == pytest.approx(math.log10(th[-1]) / 3, abs=1e-12)
    assert f[10] == pytest.approx(math.log10(th[0]) / 6, abs=1e-12)
    assert f[15] == pytest.approx((th[1] - th[0]) / (th[2] - th[0]), abs=1e-12)
    assert f[14] == 0.0  # early stop


def test_lanczos_ritz_values_bracket_spectrum():
    A = spdgen.logspaced(120, 1e4, 3)
    d = 1 / np.sqrt(np.diag(A))
    H = (d[:, None] * A) * d[None, :]
    lam = np.linalg.eigvalsh(H)
    al, be = pk.lanczos(H, np.ones(120) / np.sqrt(120), 4)
    th = pk.ritz_values(al, be)
    assert lam[0] - 1e-12 <= th[0] and th[-1] <= lam[-1] + 1e-12  # Cauchy interlacing


def _rand_params(seed, scale=0.3):
    return np.random.Generator(np.random.PCG64(seed)).normal(0, scale, pk.NPARAM)


def test_mlp_gradient_central_differences():
    rng = np.random.Generator(np.random.PCG64(1))
    X = rng.normal(0, 1, (7, 16))
    y = rng.integers(0, 4, 7)
    p = _rand_params(2)
    loss, g = pk.mlp_loss_grad(p, X, y)
    h = 1e-6
    idx = rng.choice(pk.NPARAM, 60, replace=False)
    for k in idx:
        e = np.zeros(pk.NPARAM)
        e[k] = h
        fd = (pk.mlp_loss_grad(p + e, X, y)[0] - pk.mlp_loss_grad(p - e, X, y)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(fd)), (k, fd, g[k])
    # the logits' gradient rows sum to zero, so the last bias gradient does
    assert abs(g[-4:].sum()) < 1e-14


def test_mlp_forward_hand_expanded():
    # only a path through hidden unit 0 of each layer is non-zero
    p = np.zeros(pk.NPARAM)
    W1, b1, W2, b2, W3, b3 = pk.unpack(p)  # views into p
    W1[0, 3] = 2.0
    b1[0] = -1.0
    W2[0, 0] = 0.5
    W3[2, 0] = 3.0
    b3[:] = [0.1, 0.2, 0.3, 0.4]
    X = np.array([[0] * 3 + [2.0] + [0] * 12, [0] * 3 + [0.25] + [0] * 12])
    z = pk.mlp_forward(p, X)
    # x3 = 2: h1 = relu(4 - 1) = 3, h2 = 1.5, logit2 = 4.5 + 0.3; x3 = 0.25: h1 = 0
    assert np.allclose(z[0], [0.1, 0.2, 4.8, 0.4])
    assert np.allclose(z[1], [0.1, 0.2, 0.3, 0.4])


def test_softmax_loss_uniform_logits():
    p = np.zeros(pk.NPARAM)
    X = np.ones((5, 16))
    loss, g = pk.mlp_loss_grad(p, X, np.array([0, 1, 2, 3, 0]))
    assert loss == pytest.approx(math.log(4))


def test_adam_closed_form_first_step():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.1, 0.0])
    p1, m1, v1 = pk.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # first step: mhat = g, vhat = g^2, so the move is lr * sign(g) (g != 0)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_label_rule():
    assert pk.label([True, True, True, True], [1.0, 2.0, 3.0, 4.0]) == 0
    assert pk.label([False, True, True, True], [9.0, 2.0, 2.03, 4.0]) == 2  # tie within 2 % -> higher
    assert pk.label([False, False, False, True], [0, 0, 0, 7.0]) == 3
    assert pk.label([False, False, False, False], [0, 0, 0, 0]) == 3


def test_features_arrow_matrix_max_and_mean_radius():
    # arrow matrix with unit diagonal: h_1j = h_j1 = c (j > 1), zero elsewhere;
    # SPD for c sqrt(n - 1) < 1.  Radii: r_1 = (n - 1) c, r_j = c, so the
    # largest radius (f5) and the mean radius (f6) differ in closed form
    n, c = 5, 0.25
    A = np.eye(n)
    A[0, 1:] = A[1:, 0] = c
    f = pk.features(A, 1)
    rmax, rmean = (n - 1) * c, 2 * (n - 1) * c / n
    assert f[5] == pytest.approx(math.log10(1 + rmax) / 3, abs=1e-15)
    assert f[6] == pytest.approx(math.log10(1 + rmean) / 3, abs=1e-15)
    assert f[7] == pytest.approx((n - 1) / n)          # r_1 = 1 is not < 1
    assert f[8] == pytest.approx(np.clip(1 - rmax, -10, 1) / 10)
    assert f[12] == pytest.approx(c)


def test_feature_f14_full_lanczos_against_krylov_basis():
    # K = 4 steps with no early stop: 2 [-1, 2, -1] of order 10 has five
    # eigenvectors that are symmetric under reversal, so ones/sqrt(n) spans
    # a Krylov space of dimension 5 > 4.  Independently of the three-term
    # recurrence, T_4 = Q^T H Q with Q an orthonormal basis of
    # span{v, Hv, H^2 v, H^3 v} (numpy QR), and beta_4 = ||(I - Q Q^T) H q_4||.
    n = 10
    A = 2.0 * spdgen.tridiag(n)
    f = pk.features(A, 1)
    d = 1 / np.sqrt(np.diag(A))
    H = (d[:, None] * A) * d[None, :]
    v = np.ones(n) / np.sqrt(n)
    K = np.stack([np.linalg.matrix_power(H, j) @ v for j in range(4)], axis=1)
    Q, R = np.linalg.qr(K)
    Q = Q * np.sign(np.diag(R))[None, :]
    T = Q.T @ H @ Q
    th = np.linalg.eigvalsh(T)
    w = H @ Q[:, 3]
    beta4 = np.linalg.norm(w - Q @ (Q.T @ w))
    assert beta4 > 1e-3  # no early stop
    assert f[14] == pytest.approx(beta4 / th[-1], rel=1e-9)
    assert f[9] == pytest.approx(math.log10(th[-1]) / 3, rel=1e-9)
    assert f[15] == pytest.approx((th[1] - th[0]) / (th[-1] - th[0]), rel=1e-9)
