"""CPU model of the coarse factorisation's level schedule (the launch order
of the block-sparse Cholesky, not the library's code): block columns of
equal height in the elimination tree of the tile pattern are factored
together, levels go in groups whose updates of later columns are applied
once per group ("thin" updates for the group's own later columns after
each level).  On random patterns closed under block elimination the model
must reproduce numpy's Cholesky factor, and every (tile, column) product
must be applied exactly once.  The GPU tests check the library's schedule
against its panel-step schedule on the same matrix."""
import numpy as np
import pytest


def _symbolic_fill(pat):
    nb = pat.shape[0]
    for k in range(nb):
        pat[k, k] = 1
        rows = [i for i in range(k + 1, nb) if pat[i, k]]
        for a in range(len(rows)):
            for b in range(a + 1):
                pat[rows[a], rows[b]] = 1
    return pat


def _dissection_pattern(nb, rng):
    pat = np.zeros((nb, nb), np.uint8)

    def rec(lo, hi):
        if hi - lo <= 3:
            for i in range(lo, hi):
                pat[i, lo:i + 1] = 1
            return
        s = max(1, (hi - lo) // 5)
        m = lo + (hi - lo - s) // 2
        rec(lo, m)
        rec(m, hi - s)
        for i in range(hi - s, hi):
            for j in range(lo, i + 1):
                if rng.random() < 0.3 or j >= hi - s:
                    pat[i, j] = 1
    rec(0, nb)
    return _symbolic_fill(pat)


def _schedule(F, group):
    """Launch lists: per level its columns; update launches (after_level,
    {(ti, tj): [k, ...]})."""
    nb = F.shape[0]
    R = {k: [i for i in range(k + 1, nb) if F[i, k]] for k in range(nb)}
    height = [0] * nb
    for j in range(nb):
        if R[j]:
            height[R[j][0]] = max(height[R[j][0]], height[j] + 1)
    nl = max(height) + 1
    by = [[j for j in range(nb) if height[j] == h] for h in range(nl)]
    launches = []
    for h0 in range(0, nl, group):
        h1 = min(nl, h0 + group)
        for h in range(h0, h1 - 1):
            d = {}
            for k in by[h]:
                for ai, a in enumerate(R[k]):
                    for b in R[k][:ai + 1]:
                        if height[b] < h1:
                            d.setdefault((a, b), []).append(k)
            launches.append((h, d))
        d = {}
        for h in range(h0, h1):
            for k in by[h]:
                for ai, a in enumerate(R[k]):
                    for b in R[k][:ai + 1]:
                        if height[b] >= h1:
                            d.setdefault((a, b), []).append(k)
        launches.append((h1 - 1, d))
    return R, by, launches


@pytest.mark.parametrize("group", [1, 3, 8])
def test_level_schedule_reproduces_cholesky(group):
    rng = np.random.default_rng(group)
    NB = 3
    for trial in range(8):
        nb = int(rng.integers(5, 45))
        if trial % 3:
            F = _dissection_pattern(nb, rng)
        else:
            F = _symbolic_fill((rng.random((nb, nb)) < 0.08).astype(np.uint8) * np.tri(nb, dtype=np.uint8))
        n = nb * NB
        mask = np.kron(np.maximum(F, F.T), np.ones((NB, NB)))
        M = rng.standard_normal((n, n))
        A = (M @ M.T) * mask + n * np.eye(n)
        R, by, launches = _schedule(F, group)
        got = sorted((k, a, b) for _, d in launches for (a, b), ks in d.items() for k in ks)
        want = sorted((k, a, b) for k in range(nb) for ai, a in enumerate(R[k]) for b in R[k][:ai + 1])
        assert got == want
        blk = lambda i, j: (slice(i * NB, (i + 1) * NB), slice(j * NB, (j + 1) * NB))
        W = A.copy()
        u = 0
        for h, cols in enumerate(by):
            for k in cols:
                W[blk(k, k)] = np.linalg.cholesky(W[blk(k, k)])
            for k in cols:
                for i in R[k]:
                    W[blk(i, k)] = np.linalg.solve(W[blk(k, k)], W[blk(i, k)].T).T
            while u < len(launches) and launches[u][0] == h:
                for (a, b), ks in launches[u][1].items():
                    acc = W[blk(a, b)].copy()
                    for k in ks:
                        acc -= W[blk(a, k)] @ W[blk(b, k)].T
                    W[blk(a, b)] = acc
                u += 1
        assert u == len(launches)
        L = np.tril(W * np.kron(F, np.ones((NB, NB))))
        ref = np.linalg.cholesky(A)
        assert np.abs(L - ref).max() <= 1e-10 * np.abs(ref).max()
