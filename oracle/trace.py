"""Plain simulation of the paper's fine-grained traversal for one source
(Section 4, the parallel algorithm and its worked example) -- ORACLE, test
infrastructure only.

Used to pin the reading of the method on the worked example: the label
values after each iteration, the iteration count, and the effect of the
optional "line 9.5" check. Frontiers of one iteration are processed one
after another in queue order, which is one legal schedule of the parallel
iteration.

Steps, in the paper's order and notation:

* init: every neighbour of ``src`` gets maxId = 0 and fill = src (it is an
  original entry of row src); neighbours smaller than src form the first
  frontier queue. Every other vertex has maxId = |V| ("not reached").
* each iteration, for every frontier f and neighbour w of f:
  (line 9.5, optional) skip w if fill(w) == src;
  newMaxId = max(maxId(f), f);
  if newMaxId lowers maxId(w) (the atomic minimum succeeds):
     if fill(w) != src:
        if newMaxId < w: fill(w) = src and w joins L(src,:) or U(src,:)
        if w < src: w joins the next frontier queue.
* stop when the next frontier queue is empty.
"""
from __future__ import annotations


def traverse(n, adj, src, line95=False):
    """Returns (struct_sorted, iterations, label_history) where
    label_history[k] is the maxId array after iteration k+1."""
    max_id = [n] * n
    fill = [-1] * n
    struct = {src}
    fill[src] = src
    frontier = []
    for w in adj[src]:
        if w == src:
            continue
        max_id[w] = 0
        fill[w] = src
        struct.add(w)
        if w < src:
            frontier.append(w)
    iterations = 0
    history = []
    while frontier:
        iterations += 1
        nxt = []
        for f in frontier:
            for w in adj[f]:
                if w == src:
                    continue
                if line95 and fill[w] == src:
                    continue
                new_max = max(max_id[f], f)
                if new_max < max_id[w]:
                    max_id[w] = new_max
                    if fill[w] != src:
                        if new_max < w:
                            fill[w] = src
                            struct.add(w)
                        if w < src:
                            nxt.append(w)
        frontier = nxt
        history.append(list(max_id))
    return sorted(struct), iterations, history


def adjacency(n, row_ptr, col_idx):
    return [list(col_idx[row_ptr[i]:row_ptr[i + 1]]) for i in range(n)]
