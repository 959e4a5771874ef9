"""Literal numpy float64 transcription of the paper's tensor formulas -- TEST INFRASTRUCTURE.

For tiny inputs only: it materialises the D x n x n association and conflict
tensors exactly as the paper writes them (Section 3, steps 1-4), with library
matrix products as its only building blocks.  It is used to pin the C oracle,
which computes the same quantities by one-hot gathers.

Problems: 0 k-colouring, 1 equitable colouring, 2 k-partitioning and 3 balanced
k-partitioning (Section 6: M replaced by J - M, so the group concentration
becomes D J - Mt), 4 minimum sum colouring (Section 6: the equity fitness
replaced by sum_il s_il z_l, z_l = l + 1).
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


def top_c(W: np.ndarray, demand: np.ndarray) -> np.ndarray:
    """Section 6, multicolouring: S marks the demand[i] largest weights of each row (a stable
    sort of the negated weights, so equal weights go to the lower colour first)."""
    D, n, k = W.shape
    S = np.zeros((D, n, k))
    order = np.argsort(-W, axis=2, kind="stable")
    for d in range(D):
        for i in range(n):
            S[d, i, order[d, i, :demand[i]]] = 1.0
    return S


def association(S: np.ndarray) -> np.ndarray:
    """M = S . S' (product over the colour axis), [D, n, n]."""
    return S @ np.transpose(S, (0, 2, 1))


def fitness_color(A: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Eq. (individual fitness): f_color(S_d) = 1/2 sum(C_d), C = A o M."""
    C = A[None, :, :] * association(S)
    return 0.5 * C.sum(axis=(1, 2))


def fitness_cut(A: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Section 6, k-partitioning: 1/2 sum(A o (J - M_d)), the cut edges of each member."""
    n = A.shape[0]
    J = np.ones((n, n))
    return 0.5 * (A[None, :, :] * (J[None] - association(S))).sum(axis=(1, 2))


def colour_costs(k: int) -> np.ndarray:
    """z_l = l + 1: colour l (counted from 0) costs l + 1."""
    return np.arange(1, k + 1, dtype=float)


def fitness_mscp(S: np.ndarray) -> np.ndarray:
    """Section 6, minimum sum colouring: sum_i sum_l s_il z_l."""
    return (S * colour_costs(S.shape[2])[None, None, :]).sum(axis=(1, 2))


def _is_partition(problem: int) -> bool:
    return problem in (2, 3)


def _concentration(S: np.ndarray, problem: int) -> np.ndarray:
    """Mt (colouring) or D J - Mt = sum_d (J - M_d) (partitioning)."""
    Mt = group_concentration(S)
    return S.shape[0] - Mt if _is_partition(problem) else Mt


def equity_fitness(S: np.ndarray) -> np.ndarray:
    """Eq. (equity fitness): sum_l min(|#V_dl - c1|, |#V_dl - c2|), c1 = floor(n/k), c2 = c1 + 1
    (c2 = c1 when k divides n)."""
    D, n, k = S.shape
    c1 = n // k
    c2 = c1 if n % k == 0 else c1 + 1
    V = S.sum(axis=1)
    return np.minimum(np.abs(V - c1), np.abs(V - c2)).sum(axis=1)


def class_conflicts(A: np.ndarray, S: np.ndarray) -> np.ndarray:
    """S_d' A S_d for each member (k x k), by matrix products."""
    return np.transpose(S, (0, 2, 1)) @ (A[None] @ S)


def group_concentration(S: np.ndarray) -> np.ndarray:
    """Eq. (tilde M): sum of the association tensor along the population axis."""
    return association(S).sum(axis=0)


def _pow(x: np.ndarray, p: float) -> np.ndarray:
    # |x|^p, equal to x^p on the non-negative integers and 0 at 0 for p > 0
    return np.abs(x) ** p


def kappa(A: np.ndarray, S: np.ndarray, alpha: float, problem: int = 0) -> float:
    """Eq. (penalisation): sum_ij a_ij mt_ij^alpha (D - mt_ij for partitioning)."""
    return float((A * _pow(_concentration(S, problem), alpha)).sum())


def varpi(A: np.ndarray, S: np.ndarray, beta: float, bonus_diag: int = 1, problem: int = 0) -> float:
    """Eq. (bonus): sum_ij (1 - a_ij) mt_ij^beta with J - A (diagonal dropped if bonus_diag = 0)."""
    n = A.shape[0]
    Abar = np.ones((n, n)) - A
    if not bonus_diag:
        np.fill_diagonal(Abar, 0.0)
    return float((Abar * _pow(_concentration(S, problem), beta)).sum())


def global_loss(A, S, t, alpha, lam, beta, mu, nu, problem, bonus_diag=1) -> float:
    """Eq. (global loss): f + nu t f_sec + lambda t kappa - mu t varpi, with f = f_color or the
    cut, f_sec = f_eq (problems 1, 3), f_mscp (problem 4) or absent."""
    L = fitness_cut(A, S).sum() if _is_partition(problem) else fitness_color(A, S).sum()
    if problem in (1, 3):
        L += nu * t * equity_fitness(S).sum()
    elif problem == 4:
        L += nu * t * fitness_mscp(S).sum()
    L += lam * t * kappa(A, S, alpha, problem)
    L -= mu * t * varpi(A, S, beta, bonus_diag, problem)
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
    """Eq. (global loss gradient), colouring:
    A.S + nu t (grad f_eq or z) + 2 alpha lambda t (A o Mt^(alpha-1)).S - 2 beta mu t (Abar o Mt^(beta-1)).S
    and partitioning (X = D J - Mt, whose derivative in S is minus that of Mt):
    -A.S + nu t grad f_eq - 2 alpha lambda t (A o X^(alpha-1)).S + 2 beta mu t (Abar o X^(beta-1)).S
    """
    n = A.shape[0]
    X = _concentration(S, problem)
    sgn = -1.0 if _is_partition(problem) else 1.0
    Abar = np.ones((n, n)) - A
    if not bonus_diag:
        np.fill_diagonal(Abar, 0.0)
    g = sgn * (A[None] @ S)
    if problem in (1, 3):
        g = g + nu * t * grad_equity(S)
    elif problem == 4:
        g = g + nu * t * np.broadcast_to(colour_costs(S.shape[2])[None, None, :], S.shape)
    g = g + sgn * 2 * alpha * lam * t * ((A * _pow(X, alpha - 1))[None] @ S)
    g = g - sgn * 2 * beta * mu * t * ((Abar * _pow(X, beta - 1))[None] @ S)
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
