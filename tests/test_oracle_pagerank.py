"""Pins for the oracle's PageRank (power iteration, Page et al. 1998): closed
forms on a cycle, an edgeless graph and a star; the fixed point of small
random graphs against a dense linear solve; the L1 contraction by the
damping factor; ranks summing to one."""
import numpy as np
import pytest

from paper_2103_10116_amd import inputs as I


def _google_fixed_point(G, alpha):
    """x = alpha (P^T x + (dangling . x)/n 1) + (1 - alpha)/n 1 with sum x = 1,
    solved densely: (I - alpha (P^T + 1 dang^T / n)) x = (1 - alpha)/n 1."""
    n = G.n
    outdeg = np.bincount(G.col, minlength=n)
    M = np.zeros((n, n))
    for j in range(n):
        for i in G.col[G.rowptr[j]:G.rowptr[j + 1]]:
            M[j, i] += 1.0 / outdeg[i]
    dang = (outdeg == 0).astype(float)
    A = np.eye(n) - alpha * (M + np.outer(np.ones(n), dang) / n)
    return np.linalg.solve(A, np.full(n, (1 - alpha) / n))


def test_cycle_and_edgeless_are_uniform(orc):
    for G in (I.cycle_graph(50), I.inlinks(40, [], [])):
        st, x, it, d = orc.pagerank(G, 0.85, 1e-14)
        assert st == orc.OK
        assert np.abs(x - 1.0 / G.n).max() <= 4e-16 * 1.0 / G.n * G.n


@pytest.mark.parametrize("m,alpha", [(5, 0.85), (40, 0.5)])
def test_star_closed_form(orc, m, alpha):
    # by symmetry x_hub = h, x_leaf = a with h = alpha m a + c and
    # a = alpha h / m + c, c = (1 - alpha)/(m + 1)
    c = (1 - alpha) / (m + 1)
    h = c * (1 + alpha * m) / (1 - alpha ** 2)
    a = alpha * h / m + c
    st, x, it, d = orc.pagerank(I.star_graph(m), alpha, 1e-15, 5000)
    assert st == orc.OK
    assert abs(x[0] - h) <= 1e-13 and np.abs(x[1:] - a).max() <= 1e-13
    assert abs(h + m * a - 1.0) <= 1e-14


@pytest.mark.parametrize("n,p,seed", [(30, 0.1, 1), (60, 0.03, 2), (45, 0.2, 3)])
def test_random_graph_fixed_point(orc, n, p, seed):
    G = I.random_graph(n, p, seed)
    assert (np.bincount(G.col, minlength=n) == 0).any() or p > 0.1  # dangling nodes occur
    for alpha in (0.5, 0.85):
        xs = _google_fixed_point(G, alpha)
        st, x, it, d = orc.pagerank(G, alpha, 1e-14, 10000)
        assert st == orc.OK and d <= 1e-14
        assert np.abs(x - xs).sum() <= 1e-12
        assert abs(x.sum() - 1.0) <= 1e-13


def test_l1_contraction(orc):
    # the Google matrix is a contraction by alpha in the L1 norm (on vectors
    # summing to one): ||x_k - x*||_1 <= alpha^k ||x_0 - x*||_1
    G = I.random_graph(80, 0.05, 4)
    alpha = 0.85
    xs = _google_fixed_point(G, alpha)
    e0 = np.abs(1.0 / G.n - xs).sum()
    for k in (1, 2, 5, 10, 20):
        st, x, it, d = orc.pagerank(G, alpha, 0.0, k)
        assert st == orc.NOT_CONVERGED and it == k
        assert np.abs(x - xs).sum() <= alpha ** k * e0 * (1 + 1e-9) + 1e-15


def test_powerlaw_graph_sums_to_one(orc):
    G = I.powerlaw_graph(20000, seed=5)
    st, x, it, d = orc.pagerank(G, 0.85, 1e-10)
    assert st == orc.OK and d <= 1e-10
    assert abs(x.sum() - 1.0) <= 1e-12 and (x > 0).all()
