"""Pins of the oracle's other metrics (inner product, angular).

The paper states its method for Euclidean distance and leaves inner
product and angular distance open (Section 7).  The index reduces both to
squared Euclidean distance over transformed vectors (unit rows; the
one-coordinate transform of Bachrach et al., RecSys 2014).  These tests pin
``oracle.exact_metric`` and ``oracle.metric_store64`` to facts that do not
come from the oracle itself:
  * a hand-worked example whose three orders all differ;
  * the transform's identities: every transformed row has norm M, and the
    Euclidean order over transformed rows is the inner-product order;
  * special cases: on unit rows, all three metrics give the same order;
    angular order does not change when rows are rescaled by positive factors.
"""
from __future__ import annotations

import numpy as np

import oracle

L2, ANG, IP = oracle.METRIC_L2, oracle.METRIC_ANGULAR, oracle.METRIC_IP


def test_hand_example():
    # X = (1,0) (0,2) (3,3) (-1,0) (2,1), q = (3,1)
    # squared distances 5, 10, 4, 17, 1      -> 4, 2, 0, 1, 3
    # inner products    3, 2, 12, -3, 7      -> 2, 4, 0, 1, 3
    # cosines 3/sqrt10 = .949, 2/(2 sqrt10) = .316, 12/sqrt180 = .894,
    #         -.949, 7/sqrt50 = .990          -> 4, 0, 2, 1, 3
    X = np.array([[1, 0], [0, 2], [3, 3], [-1, 0], [2, 1]], np.float64)
    q = np.array([3, 1], np.float64)
    want = {L2: ([4, 2, 0, 1, 3], [1, 4, 5, 10, 17]),
            IP: ([2, 4, 0, 1, 3], [12, 7, 3, 2, -3]),
            ANG: ([4, 0, 2, 1, 3], [7 / np.sqrt(50), 3 / np.sqrt(10), 12 / np.sqrt(180),
                                    2 / np.sqrt(40), -3 / np.sqrt(10)])}
    for m, (order, score) in want.items():
        pos, s = oracle.exact_metric(X, q, 0, 4, 5, m)
        assert pos[0].tolist() == order, m
        assert np.allclose(s[0], score, rtol=1e-12), m
    # a subrange [1, 3] and k above its width: -1 / nan padding
    pos, s = oracle.exact_metric(X, q, 1, 3, 4, IP)
    assert pos[0].tolist() == [2, 1, 3, -1] and np.isnan(s[0, 3])
    pos, _ = oracle.exact_metric(X, q, 0, 2, 3, ANG)
    assert pos[0].tolist() == [0, 2, 1]


def test_inner_product_transform_identities():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((400, 12)) * np.exp(0.6 * rng.standard_normal(400))[:, None]
    Q = rng.standard_normal((30, 12))
    S, m2 = oracle.metric_store64(X, IP)
    assert S.shape == (400, 13)
    n2 = np.sum(X * X, axis=1)
    assert m2 == n2.max()
    assert np.allclose(np.sum(S * S, axis=1), m2, rtol=1e-12)       # every row at norm M
    assert S[np.argmax(n2), 12] == 0.0 and np.all(S[:, 12] >= 0)
    assert np.array_equal(S[:, :12], X)
    Qa = np.hstack([Q, np.zeros((30, 1))])
    d2 = np.sum((S[None] - Qa[:, None]) ** 2, axis=2)
    closed = m2 + np.sum(Q * Q, axis=1)[:, None] - 2 * Q @ X.T
    assert np.allclose(d2, closed, rtol=1e-9, atol=1e-9)
    # Euclidean order over the stored rows = inner-product order over the originals
    l = rng.integers(0, 200, 30)
    r = l + rng.integers(0, 200, 30)
    pe, _ = oracle.exact_metric(S, Qa, l, r, 10, L2)
    pi, si = oracle.exact_metric(X, Q, l, r, 10, IP)
    assert np.array_equal(pe, pi)
    dif = np.diff(si, axis=1)
    assert np.all(dif[~np.isnan(dif)] <= 0)


def test_angular_transform_and_invariance():
    rng = np.random.default_rng(8)
    X = rng.standard_normal((300, 9))
    Q = rng.standard_normal((20, 9)) * 3.0
    S, m2 = oracle.metric_store64(X, ANG)
    assert m2 == 0.0 and np.allclose(np.linalg.norm(S, axis=1), 1.0, rtol=1e-14)
    l = np.zeros(20, np.int64)
    r = np.full(20, 299, np.int64)
    pa, sa = oracle.exact_metric(X, Q, l, r, 15, ANG)
    # Euclidean order over unit rows is cosine order, for any query norm
    pe, _ = oracle.exact_metric(S, Q, l, r, 15, L2)
    assert np.array_equal(pa, pe)
    # rescaling rows by positive factors keeps the cosine order
    ps, _ = oracle.exact_metric(X * rng.uniform(0.1, 10, (300, 1)), Q, l, r, 15, ANG)
    assert np.array_equal(pa, ps)
    assert np.all(np.abs(sa) <= 1 + 1e-12)


def test_unit_rows_all_metrics_agree():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((250, 6))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    Q = rng.standard_normal((25, 6))
    l = rng.integers(0, 100, 25)
    r = l + 100
    p2, _ = oracle.exact_metric(X, Q, l, r, 12, L2)
    pa, _ = oracle.exact_metric(X, Q, l, r, 12, ANG)
    pi, _ = oracle.exact_metric(X, Q, l, r, 12, IP)
    assert np.array_equal(p2, pa) and np.array_equal(p2, pi)
    # and agree with the Euclidean brute force of the filtered k-NN definition
    pb, _ = oracle.bruteforce(X.astype(np.float32), Q.astype(np.float32), l, r, 12)
    assert np.mean(pb == p2) > 0.99
