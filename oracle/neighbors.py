"""Neighbour pairs of the SPH discretisation (oracle, FP64).

Pair predicate (the paper leaves it implicit; reading recorded with the
design notes): particles i != j are neighbours when

    r_ij^2 < (kappa * max(h_i, h_j))^2,

with r_ij^2 accumulated in axis order, ((dx*dx + dy*dy) + dz*dz), every
operation rounded separately (numpy never contracts to FMA), and kappa the
kernel support in units of h.  Taking the larger smoothing length keeps every
pair for which either term of the symmetrised kernel (Sec. 2.3) is non-zero,
and makes the relation symmetric.

Results are CSR in user (input) order with ascending neighbour index per row:
``ptr`` (int64, n+1) and ``idx`` (int32).
"""
from __future__ import annotations

import itertools

import numpy as np


def disp(pos: np.ndarray, ax: int, i, j, period=None):
    """x_i - x_j along axis ax; on a periodic axis of length L (period[ax] > 0)
    the nearest image: one period is subtracted above L/2 and added below
    -L/2 (positions lie in [0, L), so one correction suffices)."""
    d = pos[ax][i] - pos[ax][j]
    if period is not None and period[ax] > 0.0:
        L = float(period[ax])
        half = 0.5 * L
        d = np.where(d > half, d - L, np.where(d < -half, d + L, d))
    return d


def pair_r2(pos: np.ndarray, i, j, period=None):
    """Squared distance accumulated in axis order, no fused operations."""
    d2 = np.zeros(np.broadcast(np.asarray(i), np.asarray(j)).shape)
    for ax in range(pos.shape[0]):
        d = disp(pos, ax, i, j, period)
        d2 = d2 + d * d
    return d2


def pair_mask(pos, h, i, j, kappa: float, period=None):
    t = kappa * np.maximum(h[i], h[j])
    return (np.asarray(i) != np.asarray(j)) & (pair_r2(pos, i, j, period) < t * t)


def _to_csr(n: int, pi: np.ndarray, pj: np.ndarray):
    order = np.lexsort((pj, pi))
    pi = pi[order]
    pj = pj[order]
    counts = np.bincount(pi, minlength=n)
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    return ptr, pj.astype(np.int32)


def brute_force(pos: np.ndarray, h: np.ndarray, kappa: float, chunk: int = 512, period=None):
    """All pairs by testing every (i, j): O(N^2), for small inputs (nearest
    images on the periodic axes of ``period``)."""
    n = h.shape[0]
    PI, PJ = [], []
    allj = np.arange(n)
    for i0 in range(0, n, chunk):
        ii = np.arange(i0, min(n, i0 + chunk))
        I, J = np.meshgrid(ii, allj, indexing="ij")
        I = I.reshape(-1)
        J = J.reshape(-1)
        m = pair_mask(pos, h, I, J, kappa, period)
        PI.append(I[m])
        PJ.append(J[m])
    return _to_csr(n, np.concatenate(PI), np.concatenate(PJ))


def neighbors_of(pos: np.ndarray, h: np.ndarray, i: int, kappa: float,
                 period=None) -> np.ndarray:
    """Ascending neighbour list of one particle by testing it against all others."""
    n = h.shape[0]
    J = np.arange(n)
    return J[pair_mask(pos, h, np.full(n, i), J, kappa, period)].astype(np.int32)


def cell_list(pos: np.ndarray, h: np.ndarray, kappa: float, chunk: int = 1 << 18):
    """The same pairs found through a uniform grid of cells no smaller than
    the largest support kappa*max(h): only particles in the same or adjacent
    cells are tested with the predicate."""
    dim, n = pos.shape
    size = kappa * float(h.max()) * (1.0 + 1e-9)
    lo = pos.min(axis=1)
    ncell = np.floor((pos.max(axis=1) - lo) / size).astype(np.int64) + 1
    cc = np.floor((pos - lo[:, None]) / size).astype(np.int64)
    cc = np.minimum(np.maximum(cc, 0), ncell[:, None] - 1)
    strides = np.ones(dim, dtype=np.int64)
    for ax in range(1, dim):
        strides[ax] = strides[ax - 1] * ncell[ax - 1]
    cid = (cc * strides[:, None]).sum(axis=0)
    order = np.argsort(cid, kind="stable")
    sorted_cid = cid[order]
    PI, PJ = [], []
    for off in itertools.product((-1, 0, 1), repeat=dim):
        off = np.array(off, dtype=np.int64)
        for i0 in range(0, n, chunk):
            ii = np.arange(i0, min(n, i0 + chunk))
            nc = cc[:, ii] + off[:, None]
            ok = np.all((nc >= 0) & (nc < ncell[:, None]), axis=0)
            ii = ii[ok]
            ncid = (nc[:, ok] * strides[:, None]).sum(axis=0)
            start = np.searchsorted(sorted_cid, ncid, side="left")
            stop = np.searchsorted(sorted_cid, ncid, side="right")
            cnt = stop - start
            I = np.repeat(ii, cnt)
            base = np.repeat(start - np.concatenate([[0], np.cumsum(cnt)[:-1]]), cnt)
            J = order[base + np.arange(cnt.sum())]
            m = pair_mask(pos, h, I, J, kappa)
            PI.append(I[m])
            PJ.append(J[m])
    return _to_csr(n, np.concatenate(PI), np.concatenate(PJ))


def build(pos: np.ndarray, h: np.ndarray, kappa: float, period=None):
    """Neighbour CSR: brute force for small inputs, cell list otherwise;
    periodic inputs (test-sized) always by brute force."""
    if h.shape[0] <= 6000 or (period is not None and np.any(np.asarray(period) > 0.0)):
        return brute_force(pos, h, kappa, period=period)
    return cell_list(pos, h, kappa)


def pairs(ptr: np.ndarray, idx: np.ndarray):
    """Expand CSR to (i, j) arrays."""
    n = ptr.shape[0] - 1
    return np.repeat(np.arange(n), np.diff(ptr)), idx.astype(np.int64)


class Sampled:
    """Ascending neighbour lists of chosen particles in a large set, without
    building every pair: candidates within kappa * max(h) (slightly enlarged)
    come from a k-d tree range query (a library primitive), and each candidate
    is then decided by the pair predicate above."""

    def __init__(self, pos: np.ndarray, h: np.ndarray, kappa: float):
        from scipy.spatial import cKDTree
        self.pos, self.h, self.kappa = pos, h, kappa
        self.tree = cKDTree(np.ascontiguousarray(pos.T))
        self.radius = kappa * float(np.max(h)) * (1.0 + 1e-9)
        self.cache = {}

    def of(self, i: int) -> np.ndarray:
        i = int(i)
        if i not in self.cache:
            cand = np.asarray(self.tree.query_ball_point(self.pos[:, i], self.radius),
                              dtype=np.int64)
            m = pair_mask(self.pos, self.h, np.full(cand.shape, i), cand, self.kappa)
            self.cache[i] = np.sort(cand[m]).astype(np.int32)
        return self.cache[i]
