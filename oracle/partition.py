"""Groups and windows of the sweeps (Sec. 3 and the implementation notes of Sec. 4.2).

Test infrastructure only (see ``oracle/__init__.py``).

Along a swept axis the nodes 1..first form group 0 (the boundary-PML layers, handled as
one block, Sec. 3); the remaining nodes are cut into consecutive groups of d layers ("several
layers are processed together", Sec. 4.2), the last one possibly shorter.  Group 0's
auxiliary problem is the group itself with the boundary profile; group g >= 1 is padded with
p moving-PML nodes below it (Sec. 4.2 allows p != b).

Pinned through the degenerate partitions in tests/test_oracle_sweep.py (one group equal to
the whole axis reproduces an exact solve).
"""


def groups(n, first, d):
    """List of (first_node, last_node) per group, 1-based and inclusive."""
    assert 1 <= first <= n and d >= 1
    out = [(1, first)]
    k = first + 1
    while k <= n:
        out.append((k, min(k + d - 1, n)))
        k += d
    return out


def window(G, g, p):
    """(w0, w1, first_phys) of the auxiliary problem of group g.

    first_phys is None for group 0 (no moving PML) and the group's first node otherwise.
    """
    a, e = G[g]
    if g == 0:
        return a, e, None
    assert a - p >= 1, "moving PML would leave the domain"
    return a - p, e, a
