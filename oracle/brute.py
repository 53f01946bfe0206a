"""Brute-force enumeration of every alignment of two short sequences -- TEST INFRASTRUCTURE ONLY.

An alignment is a monotone path of moves M (q_i against s_j), I (q_i against a
gap) and D (s_j against a gap) through the (n+1) x (m+1) grid.  Its score is
the sum of sigma over its M columns plus go + k*ge for every maximal run of k
I moves or k D moves (the affine gap model of Sec. III-A; go = 0 is the linear
model of Eqs. (2)-(3)).  Which paths count depends on the mode (Sec. III-A):

  global : from (0,0) to (n,m);
  local  : from any cell to any cell below/right of it, the empty path included;
  semi   : from a cell on row 0 or column 0, through cells with i, j >= 1 only,
           to a cell on row n or column m (the empty path when the start cell
           already is such a cell).

No dynamic programming is used: every path is generated and scored, so this
pins the oracle's recurrence, initialisation and optimum rules independently.

The canonical optimal alignment is picked by the stated conventions: among
optimal paths, the end cell with the smallest i, then the smallest j; then the
lexicographically smallest *backward choice string*.  Walking a path backward
from its end, the choices are: in the no-gap state  stop < M < enter-I-run <
enter-D-run; inside a gap run  open (the run ends here) < extend.  With go = 0
runs do not matter to the score, so each gap move is its own run of length 1.
"""
from __future__ import annotations

import sys
from dataclasses import dataclass
from typing import List, Sequence, Tuple

GLOBAL, LOCAL, SEMIGLOBAL = 0, 1, 2
OP_M, OP_I, OP_D = 0, 1, 2


@dataclass
class BruteResult:
    score: int
    q_begin: int
    q_end: int
    s_begin: int
    s_end: int
    cigar: List[Tuple[int, int]]
    n_paths: int  # number of paths scored
    n_optimal: int


def _choice_string(moves: Sequence[int], go: int) -> Tuple[int, ...]:
    toks: List[int] = []
    k = len(moves) - 1
    while k >= 0:
        op = moves[k]
        if op == OP_M:
            toks.append(1)
            k -= 1
            continue
        run = 0
        while k >= 0 and moves[k] == op:
            run += 1
            k -= 1
        enter = 2 if op == OP_I else 3
        if go == 0:
            for _ in range(run):
                toks.extend((enter, 0))
        else:
            toks.append(enter)
            toks.extend([1] * (run - 1))
            toks.append(0)
    toks.append(0)  # stop
    return tuple(toks)


def _runs(moves: Sequence[int]) -> List[Tuple[int, int]]:
    out: List[Tuple[int, int]] = []
    for op in moves:
        if out and out[-1][1] == op:
            out[-1] = (out[-1][0] + 1, op)
        else:
            out.append((1, op))
    return out


def brute_align(mode: int, sigma, go: int, ge: int, q: Sequence[int], s: Sequence[int]) -> BruteResult:
    n, m = len(q), len(s)
    q = [int(x) for x in q]
    s = [int(x) for x in s]
    sig = [[int(sigma[a][b]) for b in range(len(sigma))] for a in range(len(sigma))]

    best = None
    optimal: List[Tuple[Tuple[int, int], Tuple[int, int], Tuple[int, ...]]] = []
    counter = [0]
    moves: List[int] = []

    def is_end(i: int, j: int) -> bool:
        if mode == GLOBAL:
            return i == n and j == m
        if mode == LOCAL:
            return True
        return i == n or j == m

    def allowed(i: int, j: int) -> bool:
        if i > n or j > m:
            return False
        if mode == SEMIGLOBAL:
            return i >= 1 and j >= 1
        return True

    def visit(start, i, j, score, last):
        nonlocal best, optimal
        if is_end(i, j):
            counter[0] += 1
            if best is None or score > best:
                best = score
                optimal = [(start, (i, j), tuple(moves))]
            elif score == best:
                optimal.append((start, (i, j), tuple(moves)))
        # M
        if allowed(i + 1, j + 1):
            moves.append(OP_M)
            visit(start, i + 1, j + 1, score + sig[q[i]][s[j]], OP_M)
            moves.pop()
        # I (consumes q_{i+1})
        if allowed(i + 1, j):
            moves.append(OP_I)
            visit(start, i + 1, j, score + (ge if last == OP_I else go + ge), OP_I)
            moves.pop()
        # D (consumes s_{j+1})
        if allowed(i, j + 1):
            moves.append(OP_D)
            visit(start, i, j + 1, score + (ge if last == OP_D else go + ge), OP_D)
            moves.pop()

    if mode == GLOBAL:
        starts = [(0, 0)]
    elif mode == LOCAL:
        starts = [(i, j) for i in range(n + 1) for j in range(m + 1)]
    else:
        starts = [(0, j) for j in range(m + 1)] + [(i, 0) for i in range(1, n + 1)]
    old = sys.getrecursionlimit()
    sys.setrecursionlimit(max(old, 10 * (n + m + 10)))
    try:
        for st in starts:
            visit(st, st[0], st[1], 0, -1)
    finally:
        sys.setrecursionlimit(old)

    end = min(e for (_, e, _) in optimal)
    cands = [(_choice_string(mv, go), st, mv) for (st, e, mv) in optimal if e == end]
    cands.sort(key=lambda t: t[0])
    _, st, mv = cands[0]
    return BruteResult(best, st[0], end[0], st[1], end[1], _runs(mv), counter[0], len(optimal))
