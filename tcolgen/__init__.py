"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no arithmetic of the colouring method itself: it only draws
random numbers and builds graphs and initial weight tensors.  Both the GPU
library and the CPU oracle receive what it produces as plain arrays.

Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), implemented here from
its published definition.  A draw is addressed by (key = seed, counter =
(index_lo, index_hi, stream, 0)); each counter gives four 32-bit words.

Streams:
  0  edges of G(n, p) and of the planted graph
  1  initial weights W0
  2  finite-difference entry selection (tests)
  3  planted-partition vertex relabelling
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

STREAM_EDGES = 0
STREAM_W0 = 1
STREAM_FD = 2
STREAM_PERM = 3

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint32(0x9E3779B9)
_W1 = np.uint32(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32 with 10 rounds.

    ctr: uint32 array of shape (..., 4); key: two uint32 words.
    Returns uint32 array of shape (..., 4).
    """
    ctr = np.asarray(ctr, dtype=np.uint32)
    x0 = ctr[..., 0].astype(np.uint64)
    x1 = ctr[..., 1].astype(np.uint32)
    x2 = ctr[..., 2].astype(np.uint64)
    x3 = ctr[..., 3].astype(np.uint32)
    k0 = np.uint32(key[0])
    k1 = np.uint32(key[1])
    for r in range(10):
        if r:
            k0 = np.uint32((int(k0) + int(_W0)) & 0xFFFFFFFF)
            k1 = np.uint32((int(k1) + int(_W1)) & 0xFFFFFFFF)
        p0 = x0 * _M0
        p1 = x2 * _M1
        hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
        lo0 = (p0 & _MASK32).astype(np.uint32)
        hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
        lo1 = (p1 & _MASK32).astype(np.uint32)
        n0 = hi1 ^ x1 ^ k0
        n2 = hi0 ^ x3 ^ k1
        x0 = n0.astype(np.uint64)
        x1 = lo1
        x2 = n2.astype(np.uint64)
        x3 = lo0
    return np.stack([x0.astype(np.uint32), x1, x2.astype(np.uint32), x3], axis=-1)


def _key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)


def random_words(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    """`count` consecutive 32-bit words of one stream, starting at word `offset`.

    Word w lives in counter block w // 4, lane w % 4.
    """
    if count <= 0:
        return np.zeros(0, dtype=np.uint32)
    first = offset // 4
    last = (offset + count - 1) // 4
    blocks = np.arange(first, last + 1, dtype=np.uint64)
    ctr = np.zeros((blocks.size, 4), dtype=np.uint32)
    ctr[:, 0] = (blocks & _MASK32).astype(np.uint32)
    ctr[:, 1] = (blocks >> np.uint64(32)).astype(np.uint32)
    ctr[:, 2] = np.uint32(stream)
    out = philox4x32_10(ctr, _key(seed)).reshape(-1)
    start = offset - first * 4
    return out[start:start + count]


def uniform24(words: np.ndarray) -> np.ndarray:
    """Map 32-bit words to uniforms in [0, 1) with 24 bits: (w >> 8) * 2^-24."""
    return (words >> np.uint32(8)).astype(np.float64) * (1.0 / 16777216.0)


def uniform53(w_hi: np.ndarray, w_lo: np.ndarray) -> np.ndarray:
    """Two words to a uniform in (0, 1] with 53 bits (never 0, so log() is safe)."""
    a = (w_hi >> np.uint32(5)).astype(np.float64)   # 27 bits
    b = (w_lo >> np.uint32(6)).astype(np.float64)   # 26 bits
    return (a * 67108864.0 + b + 1.0) * (1.0 / 9007199254740992.0)


# ----------------------------------------------------------------------------
# graphs: symmetric 0/1 adjacency, zero diagonal, uint8 [n, n]
# ----------------------------------------------------------------------------

def _upper_pairs(n: int):
    iu, ju = np.triu_indices(n, k=1)
    return iu, ju


def gnp(n: int, p: float, seed: int) -> np.ndarray:
    """Erdos-Renyi G(n, p): edge {i<j} iff u24(word i*n+j of stream 0) < p."""
    A = np.zeros((n, n), dtype=np.uint8)
    if n < 2:
        return A
    iu, ju = _upper_pairs(n)
    idx = iu.astype(np.int64) * n + ju
    words = random_words(seed, STREAM_EDGES, n * n)
    u = uniform24(words[idx])
    e = u < p
    A[iu[e], ju[e]] = 1
    A[ju[e], iu[e]] = 1
    return A


def equitable_sizes(n: int, k: int) -> np.ndarray:
    """Class sizes of an equitable partition: the first n mod k classes get one more."""
    base, extra = divmod(n, k)
    return np.array([base + 1 if l < extra else base for l in range(k)], dtype=np.int64)


@dataclass
class Planted:
    A: np.ndarray
    classes: np.ndarray   # int16 [n], hidden class of each vertex
    p_cross: float


def planted(n: int, k: int, seed: int, density: float = 0.5,
            p_cross: Optional[float] = None) -> Planted:
    """Flat k-partite graph with a hidden equitable k-colouring.

    Vertices are split into k equitable classes, then relabelled by a seeded
    random permutation (stream 3).  Pairs in different classes are joined with
    probability p_cross; pairs in the same class never are, so the hidden
    classes are a legal k-colouring.  By default p_cross is chosen so the
    expected global density is `density`.
    """
    sizes = equitable_sizes(n, k)
    if p_cross is None:
        total = n * (n - 1) / 2.0
        same = float(np.sum(sizes * (sizes - 1) / 2.0))
        p_cross = density * total / (total - same) if total > same else 0.0
    cls_sorted = np.repeat(np.arange(k, dtype=np.int64), sizes)
    # random permutation by sorting 53-bit keys (stream 3)
    w = random_words(seed, STREAM_PERM, 2 * n)
    keys = uniform53(w[0::2], w[1::2])
    perm = np.argsort(keys, kind="stable")
    classes = np.empty(n, dtype=np.int64)
    classes[perm] = cls_sorted
    A = np.zeros((n, n), dtype=np.uint8)
    if n >= 2:
        iu, ju = _upper_pairs(n)
        idx = iu.astype(np.int64) * n + ju
        u = uniform24(random_words(seed, STREAM_EDGES, n * n)[idx])
        e = (u < p_cross) & (classes[iu] != classes[ju])
        A[iu[e], ju[e]] = 1
        A[ju[e], iu[e]] = 1
    return Planted(A=A, classes=classes.astype(np.int16), p_cross=float(p_cross))


def mycielski(m: int) -> np.ndarray:
    """Mycielski graph M_m (M_2 = K_2, M_3 = C_5, M_4 = Groetzsch, ...); chromatic number m.

    Textbook construction: from G on vertices v_1..v_N add u_1..u_N and w,
    join u_i to every neighbour of v_i, and join w to every u_i.
    """
    if m < 2:
        raise ValueError("m >= 2")
    A = np.array([[0, 1], [1, 0]], dtype=np.uint8)
    for _ in range(m - 2):
        N = A.shape[0]
        B = np.zeros((2 * N + 1, 2 * N + 1), dtype=np.uint8)
        B[:N, :N] = A
        B[N:2 * N, :N] = A
        B[:N, N:2 * N] = A
        B[N:2 * N, 2 * N] = 1
        B[2 * N, N:2 * N] = 1
        A = B
    return A


def greedy_colour_count(A: np.ndarray) -> int:
    """Colours used by first-fit greedy colouring in index order (a legal colouring exists with this many)."""
    n = A.shape[0]
    col = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        used = set(col[np.nonzero(A[i, :i])[0]].tolist())
        c = 0
        while c in used:
            c += 1
        col[i] = c
    return int(col.max()) + 1 if n else 0


def weights0(D: int, n: int, k: int, seed: int, sigma0: float = 0.01) -> np.ndarray:
    """Initial weights W0 ~ N(0, sigma0^2), fp32 [D, n, k] (stream 1).

    Box-Muller in FP64: counter block b gives two 53-bit uniforms (u1, u2) and
    the two normals r*cos(2 pi u2), r*sin(2 pi u2) with r = sqrt(-2 ln u1),
    for flat entries 2b and 2b+1; scaled by sigma0 and rounded to fp32.
    """
    cnt = D * n * k
    nb = (cnt + 1) // 2
    w = random_words(seed, STREAM_W0, 4 * nb)
    u1 = uniform53(w[0::4], w[1::4])
    u2 = uniform53(w[2::4], w[3::4])
    r = np.sqrt(-2.0 * np.log(u1))
    th = 2.0 * math.pi * u2
    z = np.empty(2 * nb, dtype=np.float64)
    z[0::2] = r * np.cos(th)
    z[1::2] = r * np.sin(th)
    return (z[:cnt] * sigma0).astype(np.float32).reshape(D, n, k)


def fd_entries(count: int, D: int, n: int, k: int, seed: int) -> np.ndarray:
    """`count` (d, i, j) index triples for finite-difference checks (stream 2)."""
    w = random_words(seed, STREAM_FD, 3 * count)
    d = (w[0::3] % np.uint32(D)).astype(np.int64)
    i = (w[1::3] % np.uint32(n)).astype(np.int64)
    j = (w[2::3] % np.uint32(k)).astype(np.int64)
    return np.stack([d, i, j], axis=1)


# ----------------------------------------------------------------------------
# workloads: shapes and parameters of the benchmark graphs the paper measures
# on, as synthetic stand-ins (DIMACS-like G(n, p), flat planted graphs)
# ----------------------------------------------------------------------------

KCOL, ECP, KPART, BKPART, MSCP = 0, 1, 2, 3, 4
FP32, BF16, FP8, FP4 = 0, 1, 2, 3


@dataclass
class GraphCase:
    name: str
    problem: int
    n: int
    k: int
    D: int
    precision: int
    graph: str             # "gnp" | "planted" | "mycielski"
    p: float = 0.5
    graph_seed: int = 1
    w_seed: int = 0
    eta: float = 1e-3
    rho: float = 100.0
    nb_iter: int = 5
    alpha: float = 2.5
    lam: float = 1e-5
    beta: float = 1.2
    mu: float = 1e-6
    nu: float = 0.0
    bonus_diag: int = 1
    stop_on_legal: int = 1
    momentum: float = 0.0

    def adjacency(self) -> np.ndarray:
        if self.graph == "gnp":
            return gnp(self.n, self.p, self.graph_seed)
        if self.graph == "planted":
            return planted(self.n, self.k, self.graph_seed, density=self.p).A
        if self.graph == "mycielski":
            A = mycielski(self.p_int())
            assert A.shape[0] == self.n
            return A
        raise ValueError(self.graph)

    def p_int(self) -> int:
        return int(round(self.p))

    def weights(self) -> np.ndarray:
        return weights0(self.D, self.n, self.k, self.w_seed)

    def params(self) -> dict:
        return dict(problem=self.problem, precision=self.precision, n=self.n, k=self.k, D=self.D,
                    eta=self.eta, rho=self.rho, nb_iter=self.nb_iter, alpha=self.alpha,
                    lam=self.lam, beta=self.beta, mu=self.mu, nu=self.nu,
                    bonus_diag=self.bonus_diag, stop_on_legal=self.stop_on_legal, momentum=self.momentum)


def paper_gcp(**kw) -> dict:
    """Parameter table of the paper for the GCP (k-COL)."""
    d = dict(problem=KCOL, eta=1e-3, nb_iter=5, alpha=2.5, lam=1e-5, beta=1.2, mu=1e-6, nu=0.0)
    d.update(kw)
    return d


def paper_ecp(**kw) -> dict:
    """Parameter table of the paper for the ECP."""
    d = dict(problem=ECP, eta=1e-3, nb_iter=5, alpha=2.5, lam=1e-5, beta=1.2, mu=0.0, nu=1e-5)
    d.update(kw)
    return d


def case_c1() -> GraphCase:
    return GraphCase("kcol_gnp125_k18_D8", KCOL, 125, 18, 8, FP32, "gnp", 0.5, graph_seed=1)


def case_c2(precision: int = FP32) -> GraphCase:
    return GraphCase("kcol_gnp500_k50_D64", KCOL, 500, 50, 64, precision, "gnp", 0.5, graph_seed=2)


def case_c3(precision: int = FP8) -> GraphCase:
    return GraphCase("kcol_planted1000_k28_D128", KCOL, 1000, 28, 128, precision, "planted", 0.5,
                     graph_seed=3)


def case_c4(precision: int = BF16) -> GraphCase:
    return GraphCase("ecp_gnp1000_k90_D256", ECP, 1000, 90, 256, precision, "gnp", 0.5, graph_seed=4,
                     mu=0.0, nu=1e-5)


def case_c5(precision: int = FP8) -> GraphCase:
    return GraphCase("kcol_gnp4000_k280_D32", KCOL, 4000, 280, 32, precision, "gnp", 0.5, graph_seed=5)


def cases_c5b(precision: int = BF16, count: int = 16) -> List[GraphCase]:
    """Batch of graphs with uneven sizes: n ~ U{250..2000}, p cycles .1/.5/.9, D = 16,
    k = first-fit greedy colour count (a legal k-colouring exists), density-specific
    alpha/mu deviations of the paper (alpha 1.5 at p=.9, mu 1e-7 at p=.1)."""
    out = []
    w = random_words(100, STREAM_EDGES, count, offset=0)
    for g in range(count):
        n = 250 + int(w[g] % np.uint32(1751))
        p = (0.1, 0.5, 0.9)[g % 3]
        seed = 100 + g
        A = gnp(n, p, seed)
        k = greedy_colour_count(A)
        c = GraphCase(f"batch{g}_gnp{n}_p{p}_k{k}", KCOL, n, k, 16, precision, "gnp", p,
                      graph_seed=seed)
        if p == 0.9:
            c.alpha = 1.5
        if p == 0.1:
            c.mu = 1e-7
        out.append(c)
    return out
