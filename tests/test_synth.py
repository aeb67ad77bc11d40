"""The seeded input generator: orderings, drop rule, fingerprints. CPU only."""
import os

import numpy as np
import pytest

import synth
from conftest import GOLDEN


@pytest.mark.parametrize("dims", [(7, 5, 1), (40, 40, 1), (9, 8, 7), (64, 3, 2)])
def test_nd_is_permutation(dims):
    r = synth.order(*dims, nd=True)
    assert sorted(r.tolist()) == list(range(int(np.prod(dims))))


def test_nd_separator_is_last():
    """The top-level separator of a 2D grid is numbered last."""
    nx, ny = 9, 7
    r = synth.order(nx, ny, 1, nd=True).reshape(ny, nx)
    # longest axis is x (9): cut at x = 4
    assert sorted(r[:, 4].tolist()) == list(range(nx * ny - ny, nx * ny))


@pytest.mark.parametrize("kind,dims", [(5, (12, 9)), (9, (10, 11)), (7, (5, 6, 4)), (27, (5, 5, 5))])
def test_nd_is_symmetric_permutation_of_natural(kind, dims):
    """Dropping is keyed by grid coordinates, so the ND matrix equals
    P A P^T of the natural-order matrix."""
    a = synth.stencil(kind, dims, nd=False, seed=7)
    b = synth.stencil(kind, dims, nd=True, seed=7)
    d3 = dims if len(dims) == 3 else dims + (1,)
    rank = synth.order(*d3, nd=True)
    A = set()
    for i in range(a.n):
        for j in a.col_idx[a.row_ptr[i]:a.row_ptr[i + 1]]:
            A.add((int(rank[i]), int(rank[j])))
    B = set()
    for i in range(b.n):
        for j in b.col_idx[b.row_ptr[i]:b.row_ptr[i + 1]]:
            B.add((i, int(j)))
    assert A == B


def test_drop_rate_and_nonsymmetry():
    m = synth.stencil(27, (20, 20, 20), nd=True, seed=3)
    full = synth.stencil(27, (20, 20, 20), nd=True, seed=3, drop_thresh=0)
    off = m.nnz - m.n
    off_full = full.nnz - full.n
    assert abs(1 - off / off_full - 0.2) < 0.01
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    E = set(zip(rows.tolist(), m.col_idx.tolist()))
    matched = sum((j, i) in E for (i, j) in E if i != j)
    assert 0.75 < matched / off < 0.85  # about 0.8 of kept entries are matched


def test_rows_sorted_with_diagonal():
    for m in (synth.config(1), synth.batch_member(1)):
        for i in range(m.n):
            c = m.col_idx[m.row_ptr[i]:m.row_ptr[i + 1]]
            assert (np.diff(c) > 0).all() and i in c


def test_fingerprints():
    want = {}
    with open(os.path.join(GOLDEN, "fingerprints.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, n, nnz, h = line.split()
            want[name] = (int(n), int(nnz), h)
    for name, (n, nnz, h) in want.items():
        if name.startswith("config"):
            m = synth.config(int(name[6:]))
        else:
            m = synth.batch_member(int(name[5:]))
        assert (m.n, m.nnz, synth.fingerprint(m)) == (n, nnz, h), name


def test_batch_sizes_and_trace():
    ns = [synth.grid_2d(200 + (synth.sm64((4 << 32) + k) >> 32) % 4801) for k in range(0, 64, 2)]
    assert all(a * b >= 190 for a, b in ns)
    tr = synth.serve_trace()
    assert 11000 < len(tr) < 13000
    ns = np.array([r.n_req for r in tr])
    assert ns.min() >= 1000 and ns.max() <= 1000000
    assert abs(np.median(np.log10(ns)) - 4.5) < 0.1
