"""Literal numpy float64 transcription of the paper's tensor formulas -- TEST INFRASTRUCTURE.

For tiny inputs only: it materialises the D x n x n association and conflict
tensors exactly as the paper writes them (Section 3, steps 1-4), with library
matrix products as its only building blocks.  It is used to pin the C oracle,
which computes the same quantities by one-hot gathers.
"""
from __future__ import annotations

import numpy as np


def one_hot_argmax(W: np.ndarray) -> np.ndarray:
    """Step 1: S = one_hot(argmax(W)) along the colour axis (numpy argmax: first maximum)."""
    D, n, k = W.shape
    S = np.zeros((D, n, k))
    idx = np.argmax(W, axis=2)
    for d in range(D):
        S[d, np.arange(n), idx[d]] = 1.0
    return S


def association(S: np.ndarray) -> np.ndarray:
    """M = S . S' (product over the colour axis), [D, n, n]."""
    return S @ np.transpose(S, (0, 2, 1))


def fitness_color(A: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Eq. (individual fitness): f_color(S_d) = 1/2 sum(C_d), C = A o M."""
    C = A[None, :, :] * association(S)
    return 0.5 * C.sum(axis=(1, 2))


def equity_fitness(S: np.ndarray) -> np.ndarray:
    """Eq. (equity fitness): sum_l min(|#V_dl - c1|, |#V_dl - c2|), c1 = floor(n/k), c2 = c1 + 1
    (c2 = c1 when k divides n)."""
    D, n, k = S.shape
    c1 = n // k
    c2 = c1 if n % k == 0 else c1 + 1
    V = S.sum(axis=1)
    return np.minimum(np.abs(V - c1), np.abs(V - c2)).sum(axis=1)


def group_concentration(S: np.ndarray) -> np.ndarray:
    """Eq. (tilde M): sum of the association tensor along the population axis."""
    return association(S).sum(axis=0)


def _pow(x: np.ndarray, p: float) -> np.ndarray:
    # |x|^p, equal to x^p on the non-negative integers and 0 at 0 for p > 0
    return np.abs(x) ** p


def kappa(A: np.ndarray, S: np.ndarray, alpha: float) -> float:
    """Eq. (penalisation): sum_ij a_ij mt_ij^alpha."""
    return float((A * _pow(group_concentration(S), alpha)).sum())


def varpi(A: np.ndarray, S: np.ndarray, beta: float, bonus_diag: int = 1) -> float:
    """Eq. (bonus): sum_ij (1 - a_ij) mt_ij^beta with J - A (diagonal dropped if bonus_diag = 0)."""
    n = A.shape[0]
    Abar = np.ones((n, n)) - A
    if not bonus_diag:
        np.fill_diagonal(Abar, 0.0)
    return float((Abar * _pow(group_concentration(S), beta)).sum())


def global_loss(A, S, t, alpha, lam, beta, mu, nu, problem, bonus_diag=1) -> float:
    """Eq. (global loss): f_color + nu t f_eq + lambda t kappa - mu t varpi."""
    L = fitness_color(A, S).sum()
    if problem == 1:
        L += nu * t * equity_fitness(S).sum()
    L += lam * t * kappa(A, S, alpha)
    L -= mu * t * varpi(A, S, beta, bonus_diag)
    return float(L)


def grad_equity(S: np.ndarray) -> np.ndarray:
    """Eq. (gradient of the equity fitness) broadcast over the vertices."""
    D, n, k = S.shape
    c1 = n // k
    c2 = c1 if n % k == 0 else c1 + 1
    V = S.sum(axis=1)
    g = np.where(V > c2, 1.0, np.where(V < c1, -1.0, 0.0))
    return np.broadcast_to(g[:, None, :], (D, n, k)).copy()


def grad_s(A, S, t, alpha, lam, beta, mu, nu, problem, bonus_diag=1) -> np.ndarray:
    """Eq. (global loss gradient):
    A.S + nu t grad f_eq + 2 alpha lambda t (A o Mt^(alpha-1)).S - 2 beta mu t (Abar o Mt^(beta-1)).S
    """
    n = A.shape[0]
    Mt = group_concentration(S)
    Abar = np.ones((n, n)) - A
    if not bonus_diag:
        np.fill_diagonal(Abar, 0.0)
    g = A[None] @ S
    if problem == 1:
        g = g + nu * t * grad_equity(S)
    g = g + 2 * alpha * lam * t * ((A * _pow(Mt, alpha - 1))[None] @ S)
    g = g - 2 * beta * mu * t * ((Abar * _pow(Mt, beta - 1))[None] @ S)
    return g


def softmax(W: np.ndarray) -> np.ndarray:
    """Eq. (softmax) along the colour axis."""
    e = np.exp(W - W.max(axis=2, keepdims=True))
    return e / e.sum(axis=2, keepdims=True)


def grad_w(W: np.ndarray, gS: np.ndarray) -> np.ndarray:
    """Eq. (tensor gradient): S_hat o (gS - (S_hat o gS) . J), J the k x k matrix of ones."""
    k = W.shape[2]
    Sh = softmax(W)
    J = np.ones((k, k))
    return Sh * (gS - (Sh * gS) @ J)
