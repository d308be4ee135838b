"""The paper's five-pixel worked example (Sec. V, Eqs. 2-4, 6-7, 9) pins both
the dense brute-force checker and the oracle."""
import json
import os
from fractions import Fraction

import numpy as np

import bruteforce as bf

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_example.json")))


def test_bruteforce_reproduces_printed_matrices():
    X = np.array(GOLD["X"])
    D = bf.distance_matrix(X)
    assert D.tolist() == GOLD["D_X"]                      # Eq. (3)
    A = bf.threshold(D, GOLD["radius"])
    assert A.tolist() == GOLD["A_X"]                      # Eq. (4)
    M, Dm, maxima = bf.local_maxima(GOLD["ToT"], A)
    assert M.tolist() == GOLD["ToT_odot_A"]               # Eq. (6)
    assert Dm.tolist() == GOLD["difference"]              # Eq. (7)
    assert (maxima + 1).tolist() == GOLD["local_maxima_1based"]


def test_bruteforce_centroids_at_local_maxima():
    X = np.array(GOLD["X"])
    A = bf.threshold(bf.distance_matrix(X), GOLD["radius"])
    zeros = np.zeros_like(X)
    cents = bf.centroid_rows(X, zeros, zeros, GOLD["ToT"], A)
    for row, num, den in zip(GOLD["centroid_rows_0based"], GOLD["centroid_num"],
                             GOLD["centroid_den"]):
        assert cents[row][0] == Fraction(num, den)       # Eq. (9)


def test_oracle_on_worked_example(orc):
    """One axis only: y and ToA constant, radius 5 in x.  The neighbourhoods
    of the example are already cliques, so closure changes nothing and the two
    hits are exactly the paper's two local-maximum rows."""
    X = np.array(GOLD["X"], np.uint16)
    n = X.size
    y = np.zeros(n, np.uint16)
    shot = np.zeros(n, np.uint32)
    toa = np.full(n, 1000, np.uint64)
    lab, nc = orc.cluster(X, y, shot, toa, dxy=GOLD["radius"], dt_ticks=0)
    assert lab.tolist() == [0, 0, 2, 2, 0]
    assert nc == 2
    hits = orc.centroid(X, y, np.array(GOLD["ToT"], np.uint16), shot, toa, lab,
                        np.array([1000], np.uint64))
    assert hits.size == 2
    for h, num, den in zip(hits, GOLD["centroid_num"], GOLD["centroid_den"]):
        assert h["x"] == num / den
        assert h["y"] == 0.0 and h["tof_ns"] == 0.0
    assert hits["x"][0] == 20.0
    assert abs(hits["x"][1] - 90.15384615384616) < 1e-12
    assert hits["npix"].tolist() == [3, 2]
    assert hits["tot_sum"].tolist() == [350, 325]
    assert hits["label"].tolist() == [0, 2]
