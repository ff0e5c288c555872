"""The nested-dissection ordering of the sparse solve (host part of
rbf_solve_plan, run through rbf_solve_order_host on the CPU): the order is
a permutation, the tree is one tree in postorder, and no edge of calH's
graph joins two nodes of which neither is an ancestor of the other (the
property that makes the factor's fill stay inside the fronts). Patterns:
the Gram pattern of the 40k-center map (pairs within 2 cutoff sigma_t, by
a k-d tree), a disconnected pattern, and small degenerate graphs."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.spatial import cKDTree

from paper_2509_26222_amd import api, synth


def csr_from_pairs(n, pairs, diag=True):
    i, j = (pairs[:, 0], pairs[:, 1]) if len(pairs) else (np.zeros(0, int), np.zeros(0, int))
    rows = np.concatenate([i, j] + ([np.arange(n)] if diag else []))
    cols = np.concatenate([j, i] + ([np.arange(n)] if diag else []))
    A = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(n, n))
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32)


def gram_csr(centers, r):
    pairs = cKDTree(centers).query_pairs(r, output_type="ndarray")
    return csr_from_pairs(centers.shape[0], pairs)


def check_order(rp, ci, leaf=0):
    N = rp.shape[0] - 1
    new2old, node_of, parent = api.solve_order_host(rp, ci, leaf)
    assert np.array_equal(np.sort(new2old), np.arange(N))
    nn = parent.shape[0]
    assert (parent == -1).sum() == 1
    # ancestors by walking up (depth bounded by the node count)
    depth = np.zeros(nn, int)
    for v in range(nn):
        u, d = v, 0
        while parent[u] >= 0:
            u, d = parent[u], d + 1
            assert d <= nn
        depth[v] = d
    pos = np.empty(N, np.int64)
    pos[new2old] = np.arange(N)
    # each node's unknowns are contiguous in the order, a node after its subtree
    order_nodes = node_of[new2old]
    changes = np.flatnonzero(np.diff(order_nodes)) + 1
    runs = np.split(order_nodes, changes)
    assert len({r[0] for r in runs}) == len(runs)
    first = {r[0]: s for r, s in zip(runs, np.concatenate([[0], changes]))}
    for v in first:
        if parent[v] >= 0 and parent[v] in first:
            assert first[v] < first[parent[v]]

    def is_anc(a, b):  # a is b or an ancestor of b
        while b >= 0 and depth[b] >= depth[a]:
            if b == a:
                return True
            b = parent[b]
        return False

    rows = np.repeat(np.arange(N), np.diff(rp))
    e = rows < ci
    u, v = rows[e], ci[e]
    lo = np.where(pos[u] < pos[v], u, v)
    hi = np.where(pos[u] < pos[v], v, u)
    pairs = set(zip(node_of[lo].tolist(), node_of[hi].tolist()))
    for a, b in pairs:  # the later unknown's node is the earlier one's or an ancestor
        assert is_anc(b, a), (a, b)
    return new2old, node_of, parent, depth


def test_order_gram_pattern_40k():
    case = synth.large_case(3)
    p = api.Params()
    r = 2.0 * p.cutoff * np.hypot(p.sigma, p.sigma_eps)
    rp, ci = gram_csr(case.centers, r)
    assert 90 <= ci.shape[0] / case.centers.shape[0] <= 130
    new2old, node_of, parent, depth = check_order(rp, ci)
    root = int(np.flatnonzero(parent == -1)[0])
    sizes = np.bincount(node_of, minlength=parent.shape[0])
    # a 200 x 200 lattice with coupling radius 6: separators are thin bands
    assert sizes[root] <= 2500
    assert sizes.max() <= 2500
    assert depth.max() <= 16


def test_order_disconnected_and_small():
    rng = np.random.default_rng(2)
    a = rng.uniform(0, 20, size=(1500, 2))
    b = rng.uniform(0, 20, size=(1500, 2)) + np.array([100.0, 0.0])
    rp, ci = gram_csr(np.concatenate([a, b]), 3.0)
    _, node_of, parent, _ = check_order(rp, ci, leaf=256)
    root = int(np.flatnonzero(parent == -1)[0])
    assert (node_of == root).sum() == 0  # the root only joins the two components
    # isolated unknowns, a path, a complete graph, a single unknown
    check_order(*csr_from_pairs(700, np.zeros((0, 2), int)), leaf=64)
    path = np.stack([np.arange(2999), np.arange(1, 3000)], 1)
    _, node_of, parent, depth = check_order(*csr_from_pairs(3000, path), leaf=64)
    assert depth.max() <= 40
    full = np.array([(i, j) for i in range(300) for j in range(i + 1, 300)])
    check_order(*csr_from_pairs(300, full), leaf=64)
    check_order(*csr_from_pairs(1, np.zeros((0, 2), int)))


def test_order_rejects_bad_pattern():
    rp = np.array([0, 1, 2], np.int64)
    ci = np.array([0, 5], np.int32)  # column out of range
    with pytest.raises(api.RbfError):
        api.solve_order_host(rp, ci)
