"""Colour orderings for the incomplete factorisation.

The paper does not state the ILU(0) ordering (section "Solution Update" only says the
pattern of L and U is that of A).  An ordering here is given as colour classes
C_0 .. C_{m-1}: independent sets of cells, taken in ascending colour; within a class the
order does not matter because no two cells of one class are coupled.  A solver's
ordering is an *input* to the oracle so its iterates can be compared with any solver
that exports its colouring.  The helpers below produce valid orderings for standalone
use; they are not meant to match any other implementation's choice.
"""
from collections import deque
import numpy as np


def adjacency(n, edges):
    adj = [[] for _ in range(n)]
    for a, b in np.asarray(edges):
        adj[int(a)].append(int(b))
        adj[int(b)].append(int(a))
    return adj


def greedy_colouring(n, edges):
    """First-fit colouring visiting cells by ascending id (smallest free colour)."""
    adj = adjacency(n, edges)
    col = -np.ones(n, np.int64)
    for i in range(n):
        used = {int(col[k]) for k in adj[i] if col[k] >= 0}
        c = 0
        while c in used:
            c += 1
        col[i] = c
    return col


def bipartite_colouring(n, edges):
    """Two-colouring by breadth-first search from the lowest uncoloured id, or None if
    the cell graph has an odd cycle."""
    adj = adjacency(n, edges)
    col = -np.ones(n, np.int64)
    for s in range(n):
        if col[s] >= 0:
            continue
        col[s] = 0
        dq = deque([s])
        while dq:
            i = dq.popleft()
            for k in adj[i]:
                if col[k] < 0:
                    col[k] = 1 - col[i]
                    dq.append(k)
                elif col[k] == col[i]:
                    return None
    return col


def natural_colouring(n):
    """One cell per class, ascending id: the natural (sequential) ILU ordering."""
    return np.arange(n, dtype=np.int64)


def is_valid(colour, edges):
    e = np.asarray(edges)
    return bool(np.all(colour[e[:, 0]] != colour[e[:, 1]]))


def has_triangle(n, edges):
    adj = [set(a) for a in adjacency(n, edges)]
    for a, b in np.asarray(edges):
        if adj[int(a)] & adj[int(b)]:
            return True
    return False
