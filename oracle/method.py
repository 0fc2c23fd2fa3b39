"""Pure-Python forms of the paper's own algorithms -- test infrastructure only.

These are written from the paper's descriptions (not its listings line by
line) for small cross-checks: they show that the method, read as recorded in
the design notes, reaches exactly the set the oracle enumerates.  They share
no code with the HIP path.  All lists are Python lists of tuples.

Readings taken where the paper is silent or garbled:
  * Alg 2.8 starts its element loop at m = 1 (starting at 0 would overwrite
    F[0] = [0] with an empty list).
  * Alg 2.9 keeps ge[m][i] = |Z_{>=i}(m)|, with ge[0] = [1, ..., 1]; in the
    descending lists Z_{>=i}(m) is the tail that starts after the rows whose
    first nonzero coordinate lies left of i.
  * Alg 3.1 / 3.2 scan only coordinates 1..d-1 for the rightmost nonzero one;
    p = n - phi(a) is formed right after a_i is decremented, for both branches;
    the memo covers p < topOfMemo.
  * The stream starts from the candidate (floor(n/g_1) + 1, 0, ..., 0) with
    wasValid false; for d = 1 the single row is handled directly.
"""
from __future__ import annotations


def incr(a: tuple, i: int) -> tuple:
    """incr_i of Def 2.1 (0-based i): add one to coordinate i."""
    b = list(a)
    b[i] += 1
    return tuple(b)


def lex_lists_up_to(n: int, g) -> list:
    """Alg 2.8: F[m] for m = 0..n, each list in descending lexicographic order.

    F[m] is the concatenation over i = 1..d (in that order) of incr_i applied
    to the rows of F[m - g_i] that are zero left of coordinate i (Lemma 2.3,
    Lemma 2.6 and Cor 2.7).
    """
    d = len(g)
    F = [[] for _ in range(n + 1)]
    F[0] = [tuple([0] * d)]
    for m in range(1, n + 1):
        Z = []
        for i in range(d):
            if m - g[i] >= 0:
                Z.extend(incr(a, i) for a in F[m - g[i]] if all(a[j] == 0 for j in range(i)))
        F[m] = Z
    return F


def lex_lists_factorizationwise(n: int, g) -> list:
    """Alg 2.9: the same lists built from saved cardinalities, by block copies.

    For each m and i, the rows of Z_{>=i}(m - g_i) form one contiguous run of
    the descending list Z(m - g_i): it starts after the rows whose first
    nonzero coordinate lies left of i, and its length is ge[m - g_i][i].  The
    copy-and-increment of that run is the i-th block of Z(m) (Section 2.3).
    """
    d = len(g)
    Z = [[] for _ in range(n + 1)]
    Z[0] = [tuple([0] * d)]
    ge = [[0] * d for _ in range(n + 1)]
    ge[0] = [1] * d
    for m in range(1, n + 1):
        out = []
        for i in range(d):
            src = m - g[i]
            if src < 0:
                continue
            length = ge[src][i]
            start = len(Z[src]) - length  # rows supported left of i come first
            out.extend(incr(a, i) for a in Z[src][start:start + length])
        Z[m] = out
        # |Z_{>=i}(m)| = sum over j >= i of |Z_{=j}(m)|, and |Z_{=j}(m)| is the
        # length of block j just copied.
        blocks = []
        for i in range(d):
            src = m - g[i]
            blocks.append(ge[src][i] if src >= 0 else 0)
        for i in range(d):
            ge[m][i] = sum(blocks[i:])
    return Z


def _phi(a, g) -> int:
    return sum(x * y for x, y in zip(a, g))


def next_candidate_stream(n: int, g, memo=None, memo_dim: int = 0, top: int = 0):
    """Alg 3.1 (memo_dim == 0) or Alg 3.2 (memo_dim >= 1), run as one stream
    over the whole set (no lower bound), returning rows in the order emitted
    (descending).  memo[p] must hold Z(p; g_{d-memo_dim+1..d}) in descending
    order for p < top.
    """
    d = len(g)
    if d == 1:
        return [(n // g[0],)] if n % g[0] == 0 else []
    out = []
    a = [n // g[0] + 1] + [0] * (d - 1)
    was_valid = False
    while True:
        # Rightmost nonzero among coordinates 1..d-1 (1-based), i.e. 0..d-2.
        i = -1
        for j in range(d - 1):
            if a[j] > 0:
                i = j
        if i < 0:
            break
        a[d - 1] = 0
        a[i] -= 1
        p = n - _phi(a, g)
        lead = d - memo_dim  # coordinates 0..lead-1 are leading
        if memo_dim >= 1 and i == lead - 1 and p < top:
            for tail in memo[p]:
                out.append(tuple(a[:lead]) + tuple(tail))
            was_valid = False
        else:
            m, r = divmod(p, g[i + 1])
            was_valid = r == 0
            if r != 0:
                m += 1
            a[i + 1] = m
            if was_valid:
                out.append(tuple(a))
    return out
