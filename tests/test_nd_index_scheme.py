"""Host-side check of the index scheme of the GPU nested-dissection line solver (block cyclic
reduction in x1; helm_set_line_solver).  The setup's and the solve's enumerations are replayed
in numpy on random block tridiagonal lines with scalar x1-couplings (the structure of every
line problem, Sec. 3): the blocks of each level, the remaining blocks each level updates, the
items each half of a line solve takes per phase, and the factor offsets (block i's matrices
from 3 i - 2 popcount(i) on).  The replay must reproduce a dense solve, every factor slot must
be written once and read only after it is written, and no phase may write a block another item
of the same phase reads.  It checks the enumeration, not the kernels' arithmetic (the GPU
parity tests do that against the oracle)."""
import numpy as np
import pytest


def popc(i):
    return bin(i).count("1")


def nd_first(i):
    return 3 * i - 2 * popc(i)


def test_offsets_are_prefix_sums_of_the_matrix_counts():
    # block i holds 2 tz(i + 1) + 1 matrices (tz: trailing zero bits)
    tz = lambda x: (x & -x).bit_length() - 1
    acc = 0
    for i in range(1, 600):
        acc += 2 * tz(i) + 1
        assert nd_first(i) == acc


def replay(n, B, rng):
    k = (n + 1).bit_length() - 1
    assert (1 << k) == n + 1
    D = [rng.standard_normal((B, B)) + 1j * rng.standard_normal((B, B)) + 4 * np.eye(B) for _ in range(n)]
    lc = rng.standard_normal(n) + 1j * rng.standard_normal(n)   # K_{i,i-1} = l_i I
    uc = rng.standard_normal(n) + 1j * rng.standard_normal(n)   # K_{i,i+1} = u_i I
    K = np.zeros((n * B, n * B), complex)
    for i in range(n):
        K[i * B:(i + 1) * B, i * B:(i + 1) * B] = D[i]
        if i > 0:
            K[i * B:(i + 1) * B, (i - 1) * B:i * B] = lc[i] * np.eye(B)
        if i < n - 1:
            K[i * B:(i + 1) * B, (i + 1) * B:(i + 2) * B] = uc[i] * np.eye(B)
    F = [None] * nd_first(n)

    def put(idx, M):
        assert 0 <= idx < len(F) and F[idx] is None, idx
        F[idx] = M

    def get(idx):
        assert 0 <= idx < len(F) and F[idx] is not None, idx
        return F[idx]

    # setup: per level, invert its blocks e = (2 j + 1) 2^lev - 1, then (lev >= 1) G and H,
    # then for the remaining r = 2 (m + 1) 2^lev - 1: P, Q, and the reduced D, L, U
    Wd, Wl, Wu = list(D), [None] * n, [None] * n
    for lev in range(k):
        nelim = 1 << (k - 1 - lev)
        for j in range(nelim):
            e = (2 * j + 1) * (1 << lev) - 1
            put(nd_first(e), np.linalg.inv(Wd[e]))
        if lev == k - 1:
            break
        nrem = nelim - 1
        if lev == 0:
            for x in range(nrem):
                r = 2 * x + 1
                I1, I2 = get(nd_first(r - 1)), get(nd_first(r + 1))
                Wd[r] = Wd[r] - lc[r] * uc[r - 1] * I1 - uc[r] * lc[r + 1] * I2
                Wl[r] = -lc[r] * lc[r - 1] * I1 if r - 2 >= 0 else np.zeros((B, B))
                Wu[r] = -uc[r] * uc[r + 1] * I2 if r + 2 <= n - 1 else np.zeros((B, B))
        else:
            for j in range(nelim):
                e = (2 * j + 1) * (1 << lev) - 1
                f = nd_first(e)
                put(f + 1, get(f) @ Wl[e])
                put(f + 2, get(f) @ Wu[e])
            Wl2, Wu2 = list(Wl), list(Wu)
            s = 1 << lev
            for m in range(nrem):
                r = 2 * (m + 1) * s - 1
                f1, f2 = nd_first(r - s), nd_first(r + s)
                pr = nd_first(r) + 3 + 2 * (lev - 1)
                assert pr + 1 < (nd_first(r + 1) if r + 1 < n else len(F))
                put(pr, Wl[r] @ get(f1))
                put(pr + 1, Wu[r] @ get(f2))
                Wd[r] = Wd[r] - Wl[r] @ get(f1 + 2) - Wu[r] @ get(f2 + 1)
                Wl2[r] = -Wl[r] @ get(f1 + 1)
                Wu2[r] = -Wu[r] @ get(f2 + 2)
            Wl, Wu = Wl2, Wu2
    # the middle block needs no G, H (no neighbours at its level): the only empty slots
    assert [i for i, M in enumerate(F) if M is None] == [nd_first(n // 2) + 1, nd_first(n // 2) + 2]

    # solve: half 0 owns blocks 0 .. mid - 1 and the middle block's reduction from below,
    # half 1 blocks mid + 1 .. n - 1 and the reduction from above (its own copy of the middle)
    b = [rng.standard_normal(B) + 1j * rng.standard_normal(B) for _ in range(n)]
    mid = n // 2
    vec = [dict(enumerate(b)), {}]
    vec[0] = {i: b[i] for i in range(0, mid + 1)}
    vec[1] = {i: b[i] for i in range(mid + 1, n)}
    vec[1][mid] = np.zeros(B, complex)

    def phase(items, h):
        reads, writes = set(), []
        for rd, wr, fn in items:
            reads |= set(rd)
            writes.append((wr, fn))
        ws = [w for w, _ in writes]
        assert len(set(ws)) == len(ws)
        for w, _ in writes:       # a block written in a phase is read only by its own item
            assert sum(w in rd for rd, _, _ in items) <= 1
        out = [(w, fn()) for w, fn in writes]
        for w, v in out:
            vec[h][w] = v

    for l in range(k - 1):
        s, mh = 1 << l, 1 << (k - 2 - l)
        for h in (0, 1):
            m0, ny, o0 = (mh if h else 1), (2 * mh if l >= 2 else 0), (4 * mh + 1 if h else 1)
            items = []
            for t in range(mh + ny):
                if t < mh:
                    r = (m0 + t) * 2 * s - 1
                    assert r == mid or (h == 0) == (r < mid)

                    def fn(r=r, h=h, l=l, s=s):
                        acc = vec[h][r].copy()
                        if r != mid or not h:
                            M = lc[r] * get(nd_first(r - 1)) if l == 0 else get(nd_first(r) + 3 + 2 * (l - 1))
                            acc = acc - M @ vec[h][r - s]
                        if r != mid or h:
                            M = uc[r] * get(nd_first(r + 1)) if l == 0 else get(nd_first(r) + 4 + 2 * (l - 1))
                            acc = acc - M @ vec[h][r + s]
                        return acc
                    items.append(([r - s, r + s, r], r, fn))
                else:
                    e = (o0 + 2 * (t - mh)) * (s >> 1) - 1
                    assert ((e + 1) & -(e + 1)) == s >> 1 and (h == 0) == (e < mid)
                    items.append(([e], e, lambda e=e, h=h: get(nd_first(e)) @ vec[h][e]))
            phase(items, h)
    total = vec[0][mid] + vec[1][mid]
    xm = get(nd_first(mid)) @ total
    for h in (0, 1):
        vec[h][mid] = xm
        if k >= 3:
            e = (3 if h else 1) * (1 << (k - 2)) - 1
            vec[h][e] = get(nd_first(e)) @ vec[h][e]
    for l in range(k - 2, -1, -1):
        s, ne = 1 << l, 1 << (k - 2 - l)
        for h in (0, 1):
            o0 = 2 * ne + 1 if h else 1
            items = []
            for t in range(ne):
                e = (o0 + 2 * t) * s - 1
                assert ((e + 1) & -(e + 1)) == s and (h == 0) == (e < mid)

                def fn(e=e, h=h, l=l, s=s):
                    hl, hu = e - s >= 0, e + s <= n - 1
                    if l >= 1:
                        acc = vec[h][e].copy()
                        if hl:
                            acc = acc - get(nd_first(e) + 1) @ vec[h][e - s]
                        if hu:
                            acc = acc - get(nd_first(e) + 2) @ vec[h][e + s]
                        return acc
                    v = vec[h][e].copy()
                    if hl:
                        v = v - lc[e] * vec[h][e - 1]
                    if hu:
                        v = v - uc[e] * vec[h][e + 1]
                    return get(nd_first(e)) @ v
                items.append(([e - s, e + s, e], e, fn))
            phase(items, h)
    x = np.concatenate([vec[0][i] if i <= mid else vec[1][i] for i in range(n)])
    ref = np.linalg.solve(K, np.concatenate(b))
    return np.linalg.norm(x - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("n", [3, 7, 15, 31, 63])
@pytest.mark.parametrize("B", [1, 4])
def test_replayed_solve_equals_a_dense_solve(n, B):
    err = replay(n, B, np.random.default_rng(n * 10 + B))
    assert err < 1e-9, err
