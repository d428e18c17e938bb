"""Input generators (CPU): the per-edge weight settings are symmetric, in
range and have the requested moments; they carry none of the method."""

import numpy as np

from workloads import chung_lu, normal_p, rmat, uniform_p


def _symmetric(g, ps):
    rows = np.repeat(np.arange(g.n), g.degrees())
    d = {(int(r), int(c)): x for r, c, x in zip(rows, g.col, ps)}
    return all(d[(c, r)] == x for (r, c), x in d.items())


def test_uniform_weights():
    g = chung_lu(3000, 20000, 2.3, 4)
    ps = uniform_p(g, 4)
    assert ps.shape == (g.nnz,) and _symmetric(g, ps)
    assert ps.min() >= 0.0 and ps.max() < 0.1
    und = ps[::2]  # about one value per undirected edge
    se = 0.1 / np.sqrt(12 * und.size)
    assert abs(und.mean() - 0.05) < 5 * se
    assert not np.array_equal(ps, uniform_p(g, 5))  # the seed matters


def test_normal_weights():
    g = rmat(14, 8, 0.57, 0.19, 0.19, 6)
    ps = normal_p(g, 6)
    assert _symmetric(g, ps) if g.nnz < 300000 else True
    assert ps.min() >= 0.0 and ps.max() <= 1.0
    # clipping at 0 (2.3% of the mass lies below it): E[max(X, 0)] =
    # mu * Phi(2) + sd * phi(2) = 0.05021, and the spread shrinks a little
    assert abs(ps.mean() - 0.05021) < 0.001
    assert 0.022 < ps.std() < 0.0255
    assert 0.015 < (ps == 0.0).mean() < 0.032


def test_rmat_directed_is_a_simple_digraph():
    from workloads import rmat_directed

    g = rmat_directed(10, 6, 0.57, 0.19, 0.19, 5)
    assert g.directed and g.m == g.nnz
    rp = g.row_ptr.astype(np.int64)
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(rows != g.col)  # no self-loops
    for u in range(g.n):
        row = g.col[rp[u]:rp[u + 1]]
        assert np.all(np.diff(row.astype(np.int64)) > 0)  # sorted, no duplicate arcs
    # not symmetrised: some arc has no reverse
    fwd = set(zip(rows.tolist(), g.col.tolist()))
    assert any((v, u) not in fwd for (u, v) in fwd)
    assert g.nnz <= 6 * g.n


def test_wc_weights_sum_to_one_into_each_vertex():
    from workloads import random_small_digraph, wc_p

    g = random_small_digraph(50, 300, 2)
    p = wc_p(g)
    into = np.zeros(g.n)
    np.add.at(into, g.col.astype(np.int64), p)
    indeg = np.bincount(g.col.astype(np.int64), minlength=g.n)
    assert np.allclose(into[indeg > 0], 1.0) and np.all(into[indeg == 0] == 0)
    assert np.all((p > 0) & (p <= 1))
