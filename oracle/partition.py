"""Groups and windows of the sweeps (Sec. 3 and the implementation notes of Sec. 4.2).

Test infrastructure only (see ``oracle/__init__.py``).

Along a swept axis the nodes 1..first form group 0 (the boundary-PML layers, handled as
one block, Sec. 3); the remaining nodes are cut into consecutive groups of d layers ("several
layers are processed together", Sec. 4.2), the last one possibly shorter.  Group 0's
auxiliary problem is the group itself with the boundary profile; group g >= 1 is padded with
p moving-PML nodes below it (Sec. 4.2 allows p != b).

Two fronts (x3 only; Sec. 4.2 note 3 and the experiments of Sec. 5): the axis is swept from
both faces.  The b boundary-PML layers at each face form the first and the last group, the
interior is cut into groups of d; the groups below the middle group are eliminated upwards
(auxiliary problem padded with p moving-PML nodes below, as for one front), those above it
downwards (padded with p nodes above, the mirror image), and the middle group last, padded on
both sides.

Pinned through the degenerate partitions in tests/test_oracle_sweep.py (one group equal to
the whole axis reproduces an exact solve) and, for two fronts, through the mirror symmetry of
the preconditioner under x3 -> 1 - x3.
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


def groups_two_fronts(n, b, d):
    """Groups of the two-front sweep: boundary layers 1..b, interior groups of d from node
    b+1 (the last possibly shorter), boundary layers n-b+1..n."""
    assert 1 <= b and 2 * b + 1 <= n and d >= 1
    out = [(1, b)]
    k = b + 1
    while k <= n - b:
        out.append((k, min(k + d - 1, n - b)))
        k += d
    out.append((n - b + 1, n))
    return out


def window_fronts(G, g, p, fronts):
    """(w0, w1, first_phys, last_phys) of the auxiliary problem of group g: the window and the
    nodes strictly below first_phys / above last_phys that carry moving PML (None: none on
    that side).  One front: group 0 bare, the others padded below.  Two fronts: the first
    and last groups bare, groups below the middle one padded below, above it padded above,
    the middle group (index len(G) // 2) padded on both sides."""
    a, e = G[g]
    if fronts == 1:
        w0, w1, first = window(G, g, p)
        return w0, w1, first, None
    mid = len(G) // 2
    if g == 0 or g == len(G) - 1:
        return a, e, None, None
    if g < mid:
        return a - p, e, a, None
    if g > mid:
        return a, e + p, None, e
    return a - p, e + p, a, e
