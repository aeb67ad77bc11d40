"""Pins of the CPU oracle against what the paper and the mathematics fix:
worked examples, closed forms, brute force, invariants. CPU only."""
import numpy as np
import pytest

import oracle
import synth
from oracle import trace
from conftest import adj_to_csr, oracle_members, parse_adj, read_golden


def _csr_from_dense(D):
    n = D.shape[0]
    rp = np.zeros(n + 1, dtype=np.int32)
    cols = []
    for i in range(n):
        c = np.nonzero(D[i])[0]
        cols.extend(c.tolist())
        rp[i + 1] = len(cols)
    return rp, np.array(cols, dtype=np.int32)


def _random_digraph(n, p, rng, diag=True):
    D = rng.random((n, n)) < p
    np.fill_diagonal(D, diag)
    return D


def _row_struct(res, i):
    u = res.u_idx[res.u_ptr[i]:res.u_ptr[i + 1]]
    l = res.l_ridx[res.l_rptr[i]:res.l_rptr[i + 1]]
    return l.tolist(), u.tolist()


# ---- W1: the worked example (row 8) -------------------------------------

def test_w1_row8_structure():
    g = read_golden("w1_row8.txt")
    n = int(g["n"])
    adj = parse_adj(g["edges"], n)
    rp, ci = adj_to_csr(adj)
    res = oracle.symbolic(n, rp, ci)
    src = int(g["source"])
    L, U = _row_struct(res, src)
    assert L == [int(x) for x in g["L"].split(",")]
    assert U == [int(x) for x in g["U"].split(",")]
    fills = sorted(set(L + U) - set(adj[src]) - {src})
    assert fills == [int(x) for x in g["fills"].split(",")]
    # O2 and O3 agree on the whole example graph
    F = oracle.dense_from_symbolic(res)
    assert (F == oracle.ge_filled(n, rp, ci)).all()
    assert (F == oracle.path_filled(n, rp, ci)).all()


def _labels(spec):
    return {int(a): int(b) for a, b in (t.split(":") for t in spec.split(","))}


def test_w1_label_trace_and_iterations():
    g = read_golden("w1_row8.txt")
    n = int(g["n"])
    adj = parse_adj(g["edges"], n)
    src = int(g["source"])
    struct, iters, hist = trace.traverse(n, adj, src, line95=False)
    for v, lab in _labels(g["labels_iter1"]).items():
        assert hist[0][v] == lab
    for v, lab in _labels(g["labels_iter2"]).items():
        assert hist[1][v] == lab
    assert iters == int(g["iterations"])
    s95, it95, h95 = trace.traverse(n, adj, src, line95=True)
    for v, lab in _labels(g["labels_iter2_line95"]).items():
        assert h95[1][v] == lab
    # line 9.5 changes labels, never the result
    expect = sorted([int(x) for x in g["L"].split(",")] + [int(x) for x in g["U"].split(",")])
    assert struct == expect and s95 == expect


def test_w1_edge_count():
    """edges_alg(src) = deg(src) + sum of deg(v) over the v < src reachable
    from src through vertices < src (each counted once)."""
    g = read_golden("w1_row8.txt")
    n = int(g["n"])
    adj = parse_adj(g["edges"], n)
    rp, ci = adj_to_csr(adj)
    res = oracle.symbolic(n, rp, ci)
    # reachable below 8: 1, 2, 7 directly; 0, 3, 5, 4 through them
    expect = len(adj[8]) + sum(len(adj[v]) for v in (0, 1, 2, 3, 4, 5, 7))
    assert int(res.edges[8]) == expect == 14


def _naive_parallel_fill2(adj, src, schedule):
    """PLANTED MISTAKE (Design Challenges, challenge 1; Section 4): fill2 with
    several thresholds processed at once and visit-once marks. ``schedule``
    lists (threshold, neighbour) visits in the order the threads happen to
    run; it misses fills that need a smaller threshold to arrive first."""
    visited = {src} | set(adj[src])
    struct = {src} | set(adj[src])
    for t, w in schedule:
        if w in visited:
            continue
        visited.add(w)
        if w > t:
            struct.add(w)
    return sorted(struct)


def test_a9_naive_parallel_fill2_is_rejected():
    g = read_golden("w1_row8.txt")
    n = int(g["n"])
    adj = parse_adj(g["edges"], n)
    rp, ci = adj_to_csr(adj)
    good = sorted(oracle.dense_from_symbolic(oracle.symbolic(n, rp, ci))[8].nonzero()[0].tolist())
    # threads on thresholds 1, 2 and 7; the one on 7 reaches 4 first, then
    # 2 -> 3 (fill) and 3 -> 4 finds 4 already visited.
    schedule = [(7, 4), (1, 0), (2, 3), (2, 5), (3, 4), (0, 5), (5, 3)]
    bad = _naive_parallel_fill2(adj, 8, schedule)
    assert 4 not in bad and 4 in good
    assert bad != good


# ---- W2: supernode example ----------------------------------------------

def test_w2_supernodes():
    g = read_golden("w2_supernode.txt")
    n = int(g["n"])
    urows = parse_adj(g["U"], n)
    lrows = parse_adj(g["L"], n)
    u_ptr = np.zeros(n + 1, dtype=np.int64)
    l_ptr = np.zeros(n + 1, dtype=np.int64)
    for i in range(n):
        u_ptr[i + 1] = u_ptr[i] + len(urows[i])
        l_ptr[i + 1] = l_ptr[i] + len(lrows[i])
    u_idx = np.array(sum(urows, []), dtype=np.int32)
    l_idx = np.array(sum(lrows, []), dtype=np.int32)
    ucnt = np.diff(u_ptr)
    bitmap = "".join("1" if (s > 0 and ucnt[s] == ucnt[s - 1] - 1) else "0" for s in range(4))
    assert bitmap == g["bitmap_rows0_3"]
    leaders = [s for s in range(4) if bitmap[s] == "0"]
    assert leaders == [int(x) for x in g["leaders_rows0_3"].split(",")]
    xsup, supno = oracle.supernodes(n, ucnt, l_ptr, l_idx, 128)
    xs2, sn2 = oracle.supernodes_structural(n, u_ptr, u_idx, l_ptr, l_idx, 128)
    assert (xsup == xs2).all() and (supno == sn2).all()
    groups = []
    for part in g["partition_rows0_3"].split(","):
        a, _, b = part.partition("-")
        groups.append(list(range(int(a), int(b or a) + 1)))
    for grp in groups:
        assert len(set(supno[grp].tolist())) == 1
    assert len({int(supno[grp[0]]) for grp in groups}) == len(groups)


# ---- closed forms ---------------------------------------------------------

def test_c1_tridiagonal_no_fill():
    n = 50
    D = np.eye(n, dtype=bool) | np.eye(n, k=1, dtype=bool) | np.eye(n, k=-1, dtype=bool)
    rp, ci = _csr_from_dense(D)
    res = oracle.symbolic(n, rp, ci)
    assert res.nnz_l + res.nnz_u == D.sum()


def test_c2_arrowheads():
    n = 40
    D = np.eye(n, dtype=bool)
    D[-1, :] = True
    D[:, -1] = True
    rp, ci = _csr_from_dense(D)
    res = oracle.symbolic(n, rp, ci)
    assert res.nnz_l + res.nnz_u == 3 * n - 2
    D = np.eye(n, dtype=bool)
    D[0, :] = True
    D[:, 0] = True
    rp, ci = _csr_from_dense(D)
    res = oracle.symbolic(n, rp, ci)
    assert res.nnz_l + res.nnz_u == n * n


def test_c3_5pt_envelope_fill():
    """Symmetric 5-point grid in natural order fills its envelope exactly:
    nnz(L+U) = n + 2 * sum(i - f_i), f_i the first column of row i; for
    40x40 that is 126,478."""
    m = synth.stencil(5, (40, 40), nd=False, seed=1, drop_thresh=0)
    res = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
    first = m.col_idx[m.row_ptr[:-1]]
    expect = m.n + 2 * int((np.arange(m.n) - first).sum())
    assert res.nnz_l + res.nnz_u == expect == 126478
    # every row is full from its first column to the diagonal
    for i in range(m.n):
        L, _ = _row_struct(res, i)
        assert L == list(range(int(first[i]), i))


def test_c4_c5_c6_supernode_closed_forms():
    n = 300
    D = np.eye(n, dtype=bool)
    rp, ci = _csr_from_dense(D)
    assert oracle.symbolic(n, rp, ci).nsuper == n
    D = np.ones((n, n), dtype=bool)
    rp, ci = _csr_from_dense(D)
    for M in (128, 64, 7, 0):
        r = oracle.symbolic(n, rp, ci, max_supernode=M)
        assert r.nsuper == (1 if M == 0 else -(-n // M))
    for tri in (np.tril(np.ones((n, n), dtype=bool)), np.triu(np.ones((n, n), dtype=bool))):
        rp, ci = _csr_from_dense(tri)
        assert oracle.symbolic(n, rp, ci).nsuper == n


# ---- brute force ---------------------------------------------------------

@pytest.mark.parametrize("seed", range(40))
def test_o1_o2_o3_random_tiny(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 17))
    D = _random_digraph(n, float(rng.uniform(0.05, 0.5)), rng, diag=bool(seed % 2))
    rp, ci = _csr_from_dense(D)
    res = oracle.symbolic(n, rp, ci)
    F = oracle.dense_from_symbolic(res)
    assert (F == oracle.ge_filled(n, rp, ci)).all()
    assert (F == oracle.path_filled(n, rp, ci)).all()
    adj = trace.adjacency(n, rp, ci)
    for src in range(n):
        s0, _, _ = trace.traverse(n, adj, src, line95=False)
        s1, _, _ = trace.traverse(n, adj, src, line95=True)
        assert s0 == s1 == np.nonzero(F[src])[0].tolist()


@pytest.mark.parametrize("seed", range(6))
def test_o1_o2_random_medium(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(60, 300))
    D = _random_digraph(n, 3.0 / n, rng, diag=True)
    rp, ci = _csr_from_dense(D)
    res = oracle.symbolic(n, rp, ci)
    assert (oracle.dense_from_symbolic(res) == oracle.ge_filled(n, rp, ci)).all()
    adj = trace.adjacency(n, rp, ci)
    for src in rng.choice(n, 20, replace=False):
        s, _, _ = trace.traverse(n, adj, int(src), line95=bool(seed % 2))
        L, U = _row_struct(res, int(src))
        assert s == L + U


def _family_members():
    yield synth.stencil(9, (32, 32), nd=True, seed=11)
    yield synth.stencil(9, (48, 40), nd=True, seed=12)
    yield synth.stencil(27, (8, 8, 8), nd=True, seed=13)
    yield synth.stencil(27, (10, 9, 11), nd=True, seed=14)
    yield synth.stencil(5, (30, 30), nd=False, seed=15)
    for k in (0, 1, 6, 7):
        m = synth.batch_member(k)
        if m.n <= 2500:
            yield m


@pytest.mark.parametrize("m", list(_family_members()), ids=lambda m: m.desc[:40])
def test_o1_vs_o2_generator_families(m):
    res = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
    assert (oracle.dense_from_symbolic(res) == oracle.ge_filled(m.n, m.row_ptr, m.col_idx)).all()


def test_o1_vs_o2_config1():
    m = synth.config(1)
    res = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
    assert (oracle.dense_from_symbolic(res) == oracle.ge_filled(m.n, m.row_ptr, m.col_idx)).all()
    assert 4e6 < res.edges_alg < 6e6


def test_edges_alg_by_reachability():
    """Per-row algorithmic edges equal deg(src) plus the degrees of the
    vertices below src reachable from src through vertices below src."""
    m = synth.stencil(27, (7, 6, 5), nd=True, seed=21)
    res = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
    adj = trace.adjacency(m.n, m.row_ptr, m.col_idx)
    for src in range(m.n):
        seen, stack = set(), [src]
        while stack:
            x = stack.pop()
            for w in adj[x]:
                if w < src and w not in seen:
                    seen.add(w)
                    stack.append(w)
        assert res.edges[src] == len(adj[src]) + sum(len(adj[v]) for v in seen)


# ---- invariants ----------------------------------------------------------

def test_i1_i2_pattern_and_closure():
    for m in (synth.stencil(9, (20, 20), nd=True, seed=31), synth.batch_member(3)):
        if m.n > 1500:
            continue
        res = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
        F = oracle.dense_from_symbolic(res)
        rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
        assert F[rows, m.col_idx].all()
        assert F[np.arange(m.n), np.arange(m.n)].all()
        n = m.n
        for k in range(n):
            ii = np.nonzero(F[k + 1:, k])[0] + k + 1
            jj = np.nonzero(F[k, k + 1:])[0] + k + 1
            if ii.size and jj.size:
                assert F[np.ix_(ii, jj)].all()


def _transpose_csr(n, rp, ci):
    t_ptr, t_idx = oracle.csr_to_csc(n, rp, ci)
    return t_ptr.astype(np.int32), t_idx


@pytest.mark.parametrize("m", [synth.stencil(9, (40, 30), nd=True, seed=41),
                               synth.stencil(27, (12, 12, 12), nd=True, seed=42),
                               synth.batch_member(5)], ids=lambda m: m.desc[:30])
def test_i3_transpose_duality(m):
    """filled(A^T) == filled(A)^T: the strict upper part of U(A) in CSR is
    L(A^T) in CSC, and L(A) in CSC is the strict upper part of U(A^T)."""
    a = oracle.symbolic(m.n, m.row_ptr, m.col_idx, with_supernodes=False)
    tp, ti = _transpose_csr(m.n, m.row_ptr, m.col_idx)
    b = oracle.symbolic(m.n, tp, ti, with_supernodes=False)

    def strict_u(r):
        keep = r.u_idx != np.repeat(np.arange(r.n), np.diff(r.u_ptr))
        cnt = np.diff(r.u_ptr) - 1
        ptr = np.zeros(r.n + 1, dtype=np.int64)
        np.cumsum(cnt, out=ptr[1:])
        return ptr, r.u_idx[keep]

    up, ui = strict_u(a)
    assert (up == b.l_ptr).all() and (ui == b.l_idx).all()
    up, ui = strict_u(b)
    assert (up == a.l_ptr).all() and (ui == a.l_idx).all()


def test_i4_i5_supernode_partition():
    for M in (128, 16, 5):
        for m in (synth.stencil(9, (30, 30), nd=True, seed=51), synth.batch_member(2)):
            res = oracle.symbolic(m.n, m.row_ptr, m.col_idx, max_supernode=M)
            xs = res.xsup
            assert xs[0] == 0 and xs[-1] == m.n and (np.diff(xs) > 0).all()
            for a, b in zip(xs[:-1], xs[1:]):
                assert a // M == (b - 1) // M
            assert (res.supno == np.repeat(np.arange(len(xs) - 1), np.diff(xs))).all()
            x2, s2 = oracle.supernodes_structural(m.n, res.u_ptr, res.u_idx,
                                                  res.l_rptr, res.l_ridx, M)
            assert (x2 == xs).all() and (s2 == res.supno).all()


def test_i6_monotone_in_pattern():
    m = synth.stencil(9, (25, 25), nd=True, seed=61)
    m2 = synth.band_extras(m, 300, seed=62, bw=20)
    F1 = oracle.dense_from_symbolic(oracle.symbolic(m.n, m.row_ptr, m.col_idx))
    F2 = oracle.dense_from_symbolic(oracle.symbolic(m2.n, m2.row_ptr, m2.col_idx))
    assert (F2 | F1 == F2).all() and F2.sum() > F1.sum()


def test_i7_symmetric_pattern_gives_symmetric_fill():
    m = synth.stencil(27, (9, 9, 9), nd=True, seed=71, drop_thresh=0)
    res = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
    F = oracle.dense_from_symbolic(res)
    assert (F == F.T).all()


# ---- test helpers of the oracle: the transpose and the fill count ---------

@pytest.mark.parametrize("seed", range(6))
def test_transpose_helper_against_dense(seed):
    """oracle.csr_to_csc against the dense transpose, with columns shuffled
    inside rows (the helper must still list each column's rows ascending)."""
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(1, 70))
    D = _random_digraph(n, 0.15, rng, diag=bool(seed % 2))
    rp, ci = _csr_from_dense(D)
    ci = ci.copy()
    for i in range(n):
        rng.shuffle(ci[rp[i]:rp[i + 1]])
    tp, ti = oracle.csr_to_csc(n, rp, ci)
    assert tp[0] == 0 and tp[-1] == D.sum()
    for c in range(n):
        assert ti[tp[c]:tp[c + 1]].tolist() == np.nonzero(D[:, c])[0].tolist()


def test_transpose_helper_edge_cases():
    tp, ti = oracle.csr_to_csc(0, np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert tp.tolist() == [0] and len(ti) == 0
    # empty rows and columns
    tp, ti = oracle.csr_to_csc(4, np.array([0, 0, 2, 2, 3]), np.array([3, 0, 3], np.int32))
    assert tp.tolist() == [0, 1, 1, 1, 3] and ti.tolist() == [1, 1, 3]


@pytest.mark.parametrize("seed", range(8))
def test_pattern_with_diag_nnz_brute_force(seed):
    """nnz(pattern(A) union diag) against the dense count, rows with and
    without a stored diagonal mixed."""
    rng = np.random.default_rng(600 + seed)
    n = int(rng.integers(1, 60))
    D = _random_digraph(n, 0.1, rng, diag=False)
    D[np.diag_indices(n)] = rng.random(n) < 0.5
    rp, ci = _csr_from_dense(D)
    assert oracle.pattern_with_diag_nnz(n, rp, ci) == int((D | np.eye(n, dtype=bool)).sum())


def test_fill_count_closed_forms():
    """fills = nnz(L+U) - nnz(pattern(A) union diag) (dataset table,
    "#Fill-in") on patterns whose fill is known in closed form."""
    n = 50
    tri = np.eye(n, dtype=bool) | np.eye(n, k=1, dtype=bool) | np.eye(n, k=-1, dtype=bool)
    rp, ci = _csr_from_dense(tri)
    assert oracle.fills(oracle.symbolic(n, rp, ci), rp, ci) == 0
    # the same without stored diagonal entries: U still holds the diagonal
    rp, ci = _csr_from_dense(tri & ~np.eye(n, dtype=bool))
    assert oracle.pattern_with_diag_nnz(n, rp, ci) == 3 * n - 2
    assert oracle.fills(oracle.symbolic(n, rp, ci), rp, ci) == 0
    n = 40
    arrow = np.eye(n, dtype=bool)
    arrow[0, :] = True
    arrow[:, 0] = True
    rp, ci = _csr_from_dense(arrow)
    assert oracle.fills(oracle.symbolic(n, rp, ci), rp, ci) == n * n - (3 * n - 2)
    arrow = np.eye(n, dtype=bool)
    arrow[-1, :] = True
    arrow[:, -1] = True
    rp, ci = _csr_from_dense(arrow)
    assert oracle.fills(oracle.symbolic(n, rp, ci), rp, ci) == 0
    # 40x40 5-point stencil, nothing dropped, natural order: the envelope
    # (126,478 entries) minus the stencil's own couplings, 1,600 diagonal
    # entries plus 2 * 2 * 40 * 39 neighbour pairs
    m = synth.stencil(5, (40, 40), nd=False, seed=1, drop_thresh=0)
    res = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
    assert oracle.pattern_with_diag_nnz(m.n, m.row_ptr, m.col_idx) == 1600 + 4 * 40 * 39
    assert oracle.fills(res, m.row_ptr, m.col_idx) == 126478 - 7840


def test_oracle_members_helper_matches_single_calls():
    """The test helper that runs O1 on a block-diagonal concatenation of many
    matrices gives every matrix's own result."""
    mats = [synth.batch_member(k) for k in (0, 1, 7, 4095)]
    for m, a in zip(mats, oracle_members(mats)):
        b = oracle.symbolic(m.n, m.row_ptr, m.col_idx)
        assert np.array_equal(a.u_ptr, b.u_ptr) and np.array_equal(a.u_idx, b.u_idx)
        assert np.array_equal(a.l_ptr, b.l_ptr) and np.array_equal(a.l_idx, b.l_idx)
        assert np.array_equal(a.xsup, b.xsup) and np.array_equal(a.supno, b.supno)
        assert a.edges_alg == b.edges_alg
