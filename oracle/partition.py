"""Oracle of the atom decomposition of Sec. 3.1 (test infrastructure only).

Plain numpy, FP64, written from the paper's description: the modified
recursive bisection (Sec. 3.1.2) whose every split projects the atoms on the
principal axis of their inertia tensor (Sec. 3.1.3, Eq. (11)-(18)), with the
per-atom weights of Eq. (19) (Sec. 3.1.4), in the order of Sec. 3.1.5:

    leaf if one process or no atoms; else
    centre (Eq. (12)) -> inertia tensor (Eq. (17), (18)) -> diagonalise ->
    choose the eigenvector that maximises F (Eq. (14)) -> project (Eq. (13))
    -> sort -> split where the two weight sums match the process split.

Readings (where the paper leaves a choice open):
  * Eq. (12) divides the weighted sum by the atom count; the centre used here
    divides by the total weight, which is the same for unit weights and keeps
    the split independent of where the origin is for any weights.
  * A node of n processes gives ceil(n/2) of them to the child holding the
    lower projections and the rest to the other child.
  * The split index makes the lower child's weight nearest to its share
    W * ceil(n/2) / n of the node's weight W; on a tie the lower child takes
    one more atom (the paper's 13 atoms on 2 processes become 7 and 6).
  * Sorting is ascending in t with ties by atom index, and the eigenvector's
    sign makes its largest-magnitude component positive (first on a tie), so
    that the order is defined.  Inside a leaf the atoms keep the order of the
    last sort.
  * When two eigenvectors give the same F (a degenerate tensor) any of them is
    a valid axis; this code takes the first that numpy returns, so such inputs
    only admit property checks.

Only tests/, the smoke check and the CPU baseline may import this module; the
library never does.  Pins: tests/test_partition.py (the paper's 26-atom
example, closed forms of the inertia tensor, brute-force maximality of F,
translation/rotation/weight-scale invariances, balance bounds).
"""
from __future__ import annotations

import numpy as np


def centre(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Weighted centre of the atoms (Eq. (12), normalised by the total weight)."""
    return (w[:, None] * x).sum(axis=0) / w.sum()


def inertia_tensor(x: np.ndarray, w: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Inertia tensor about c, element by element as in Eq. (17) with the
    relative coordinates of Eq. (18)."""
    X = x[:, 0] - c[0]
    Y = x[:, 1] - c[1]
    Z = x[:, 2] - c[2]
    T = np.empty((3, 3))
    T[0, 0] = np.sum(w * (Y * Y + Z * Z))
    T[1, 1] = np.sum(w * (X * X + Z * Z))
    T[2, 2] = np.sum(w * (X * X + Y * Y))
    T[0, 1] = T[1, 0] = -np.sum(w * X * Y)
    T[0, 2] = T[2, 0] = -np.sum(w * X * Z)
    T[1, 2] = T[2, 1] = -np.sum(w * Y * Z)
    return T


def projection(x: np.ndarray, c: np.ndarray, a: np.ndarray) -> np.ndarray:
    """t_i of Eq. (13)."""
    return a[0] * (x[:, 0] - c[0]) + a[1] * (x[:, 1] - c[1]) + a[2] * (x[:, 2] - c[2])


def objective(x: np.ndarray, w: np.ndarray, c: np.ndarray, a: np.ndarray) -> float:
    """F of Eq. (14) on the unit sphere (the multiplier term vanishes there)."""
    t = projection(x, c, a)
    return float(np.sum(w * t * t))


def principal_axis(x: np.ndarray, w: np.ndarray):
    """Centre and principal axis of a set of atoms (Sec. 3.1.3): the
    eigenvectors of the inertia tensor are the stationary points of F on
    |a| = 1 (Eq. (15), (16)); the one with the largest F is taken."""
    c = centre(x, w)
    T = inertia_tensor(x, w, c)
    _, vecs = np.linalg.eigh(T)
    F = [objective(x, w, c, vecs[:, k]) for k in range(3)]
    a = vecs[:, int(np.argmax(F))].copy()
    a /= np.linalg.norm(a)
    big = int(np.argmax(np.abs(a)))
    if a[big] < 0:
        a = -a
    return c, a


def split_index(w_sorted: np.ndarray, n_lower: int, n: int) -> int:
    """Number of atoms (taken in projection order) for the child with n_lower
    of the node's n processes: the prefix whose weight is nearest to that
    child's share of the total, the longer prefix on a tie."""
    cum = np.concatenate([[0.0], np.cumsum(w_sorted)])
    target = cum[-1] * n_lower / n
    d = np.abs(cum - target)
    return int(np.flatnonzero(d == d.min()).max())


def decompose(pos, nparts: int, weights=None):
    """Atom decomposition (Sec. 3.1.5).  Returns (order, part, part_start):
    atom indices grouped by part in the tree's leaf order, the part of each
    atom, and the nparts + 1 offsets of the parts in `order`."""
    x = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    natoms = x.shape[0]
    w = np.ones(natoms) if weights is None else np.asarray(weights, dtype=np.float64).reshape(-1)
    if nparts < 1:
        raise ValueError("nparts must be >= 1")
    if w.shape[0] != natoms or np.any(~(w > 0)) or not np.all(np.isfinite(w)):
        raise ValueError("weights must be finite and > 0, one per atom")
    if not np.all(np.isfinite(x)):
        raise ValueError("positions must be finite")

    leaves = []  # (first part, number of parts, atom indices in order)

    def node(idx: np.ndarray, n: int, p0: int):
        if n == 1 or idx.size == 0:
            leaves.append((p0, n, idx))
            return
        c, a = principal_axis(x[idx], w[idx])
        t = projection(x[idx], c, a)
        srt = idx[np.lexsort((idx, t))]
        n_lower = (n + 1) // 2
        k = split_index(w[srt], n_lower, n)
        node(srt[:k], n_lower, p0)
        node(srt[k:], n - n_lower, p0 + n_lower)

    node(np.arange(natoms), nparts, 0)
    leaves.sort(key=lambda e: e[0])
    order = np.concatenate([e[2] for e in leaves]).astype(np.int64) if natoms else np.zeros(0, np.int64)
    part = np.empty(natoms, dtype=np.int64)
    start = np.zeros(nparts + 1, dtype=np.int64)
    for p0, n, idx in leaves:
        part[idx] = p0
        start[p0 + 1] = idx.size  # parts p0+1 .. p0+n-1 of an empty or one-part leaf hold nothing
    start = np.cumsum(start)
    return order, part, start
