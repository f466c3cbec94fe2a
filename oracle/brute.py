"""Exact brute force over all global alignments (test infrastructure only).

Enumerates every monotone lattice path from (0,0) to (n,m) with steps DIAG
(1,1), UP (1,0) and LEFT (0,1) -- the D(n,m) Delannoy paths -- and scores each
as the sum of S over its DIAG cells plus g per gap step, in exact rational
arithmetic.  This is the plain definition of the optimum the NW recurrence of
Sec. 5.1 (Figs. 1-2, eq. (1)) computes, with no recurrence at all.

Among equal-scoring optima it picks the one the UP > LEFT > DIAG traceback
picks: the path whose move sequence, read from (n,m) back to (0,0), is
lexicographically greatest with UP > LEFT > DIAG.
"""
from __future__ import annotations

from fractions import Fraction

UP, LEFT, DIAG = "U", "L", "D"
_RANK = {UP: 2, LEFT: 1, DIAG: 0}


def paths(n: int, m: int):
    """Yield every path as a tuple of moves in forward order."""
    out = []

    def rec(i, j, acc):
        if i == n and j == m:
            out.append(tuple(acc))
            return
        if i < n and j < m:
            acc.append(DIAG); rec(i + 1, j + 1, acc); acc.pop()
        if i < n:
            acc.append(UP); rec(i + 1, j, acc); acc.pop()
        if j < m:
            acc.append(LEFT); rec(i, j + 1, acc); acc.pop()

    rec(0, 0, [])
    return out


def delannoy(n: int, m: int) -> int:
    D = [[1] * (m + 1) for _ in range(n + 1)]
    for i in range(1, n + 1):
        for j in range(1, m + 1):
            D[i][j] = D[i - 1][j] + D[i][j - 1] + D[i - 1][j - 1]
    return D[n][m]


def path_score(moves, S, g):
    i = j = 0
    tot = Fraction(0)
    diag = []
    for mv in moves:
        if mv == DIAG:
            tot += Fraction(S[i][j])
            diag.append((i, j))
            i += 1; j += 1
        elif mv == UP:
            tot += Fraction(g)
            i += 1
        else:
            tot += Fraction(g)
            j += 1
    return tot, diag


def best_alignment(S, g, n=None, m=None):
    """Exact optimum: (score as Fraction, DIAG cells of the chosen optimal path,
    number of optimal paths).  ``best_alignment.last_moves`` holds the chosen
    path's full move sequence (forward order)."""
    if n is None:
        n = len(S)
    if m is None:
        m = len(S[0]) if n else 0
    best = None
    best_key = None
    best_diag = None
    best_moves = None
    count = 0
    for moves in paths(n, m):
        sc, diag = path_score(moves, S, g)
        key = tuple(_RANK[x] for x in reversed(moves))
        if best is None or sc > best:
            best, best_key, best_diag, best_moves, count = sc, key, diag, moves, 1
        elif sc == best:
            count += 1
            if key > best_key:
                best_key, best_diag, best_moves = key, diag, moves
    best_alignment.last_moves = best_moves
    return best, best_diag, count
