"""The paper's dense array formulation, used as an independent O(n^2) check of
the oracle on tiny inputs.

Sec. V (Neighborhoods): per axis, the distance matrix is the row-repeated
value array minus its transpose (Eq. 3), thresholded at |D| <= r (Eq. 4); the
adjacency A is the Hadamard product over X, Y and ToF (Eq. 5).  Pixels of
different laser shots never share a neighbourhood (each shot is its own slice
along the batching axis, Sec. VI), so A is also multiplied by the shot-equality
matrix.  A hit here is a connected component, i.e. the transitive closure A*
of A, found by repeated boolean squaring of (I or A).  Centroids are Eq. (9)
evaluated on the rows of A*:  X_i = sum_j X_j A*_ij ToT_j / sum_j ToT_j A*_ij.
The local-maximum step (Eqs. 6-7) is provided for the worked example.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def distance_matrix(v):
    """Eq. (3): repeated row matrix minus its transpose, D_ij = v_j - v_i."""
    v = np.asarray(v, dtype=np.int64)
    rep = np.tile(v, (v.size, 1))
    return rep - rep.T


def threshold(D, r):
    """Eq. (4): A_ij = 1 where |D_ij| <= r."""
    return (np.abs(D) <= r).astype(np.int64)


def adjacency(x, y, t, shot, r_xy, r_t):
    """Eq. (5) plus the per-shot batching axis."""
    A = threshold(distance_matrix(x), r_xy) * threshold(distance_matrix(y), r_xy) \
        * threshold(distance_matrix(t), r_t)
    same_shot = (distance_matrix(shot) == 0).astype(np.int64)
    return A * same_shot


def closure(A):
    """Reachability: (I or A) squared until it stops changing."""
    n = A.shape[0]
    R = ((A + np.eye(n, dtype=np.int64)) > 0).astype(np.int64)
    while True:
        R2 = ((R @ R) > 0).astype(np.int64)
        if np.array_equal(R2, R):
            return R
        R = R2


def labels(x, y, toa, shot, r_xy=1, r_t=128):
    """label_i = the first column set in row i of A* (smallest reachable index)."""
    n = len(x)
    if n == 0:
        return np.zeros(0, np.int64)
    t = np.asarray(toa, dtype=np.int64) - int(np.min(toa))
    R = closure(adjacency(x, y, t, shot, r_xy, r_t))
    return np.argmax(R > 0, axis=1).astype(np.int64)


def centroid_rows(x, y, tof, tot, R):
    """Eq. (9) on every row of a 0/1 neighbourhood matrix, as exact fractions.
    Rows with zero total ToT fall back to the plain mean over the row."""
    x = np.asarray(x, np.int64)
    y = np.asarray(y, np.int64)
    tof = np.asarray(tof, np.int64)
    tot = np.asarray(tot, np.int64)
    out = []
    for i in range(R.shape[0]):
        row = R[i].astype(np.int64)
        w = int(row @ tot)
        if w > 0:
            out.append((Fraction(int(row @ (tot * x)), w), Fraction(int(row @ (tot * y)), w),
                        Fraction(int(row @ (tot * tof)), w), False))
        else:
            c = int(row.sum())
            out.append((Fraction(int(row @ x), c), Fraction(int(row @ y), c),
                        Fraction(int(row @ tof), c), True))
    return out


def hits(x, y, tot, shot, toa, trig, r_xy=1, r_t=128):
    """One hit per component, sorted by (shot, label), with exact centroids.
    ToF is in ticks relative to the shot's trigger."""
    n = len(x)
    if n == 0:
        return []
    t = np.asarray(toa, dtype=np.int64) - int(np.min(toa))
    R = closure(adjacency(x, y, t, shot, r_xy, r_t))
    lab = np.argmax(R > 0, axis=1)
    tof = np.asarray(toa, np.int64) - np.asarray(trig, np.int64)[np.asarray(shot, np.int64)]
    cents = centroid_rows(x, y, tof, tot, R)
    out = []
    for i in range(n):
        if lab[i] == i:
            members = np.nonzero(R[i])[0]
            cx, cy, ct, flagged = cents[i]
            out.append(dict(shot=int(shot[i]), label=i, npix=int(members.size),
                            tot_sum=int(np.sum(np.asarray(tot, np.int64)[members])),
                            toa_first=int(np.min(np.asarray(toa, np.int64)[members])),
                            x=cx, y=cy, tof_ticks=ct, flagged=flagged))
    out.sort(key=lambda h: (h["shot"], h["label"]))
    return out


def local_maxima(tot, A):
    """Eqs. (6)-(7): M = ToT (row-repeated) Hadamard A; a row of M - M^T whose
    maximum is 0 marks a local maximum."""
    tot = np.asarray(tot, dtype=np.int64)
    M = np.tile(tot, (tot.size, 1)) * A
    Dm = M - M.T
    return M, Dm, np.nonzero(Dm.max(axis=1) == 0)[0]
