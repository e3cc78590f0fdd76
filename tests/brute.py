"""Exhaustive enumeration of alignments, used to pin the oracle.

Independent of both the oracle and the GPU library: it lists every
alignment (every string of M, I and D operations with its start in the
window) between short sequences and scores each one directly from the
affine-gap definition -- a maximal run of L insertions or deletions costs
o + L*e, an aligned pair scores a if the bases are equal, b otherwise.
Nothing here evaluates a DP recurrence.

Semi-global alignments use the whole read against any substring of the
window; local alignments use any substrings of both (plus the empty
alignment, score 0).  From the set of optimal alignments it derives
  * the optimal score,
  * every optimal end cell, and the tie-broken one (smallest window
    column, then smallest read row),
  * the canonical alignment that the traceback priorities select: walking
    backwards from the end cell, prefer stopping > match > deletion >
    insertion, and inside a gap prefer opening it here > extending it.
    Among optimal alignments this is the lexicographically smallest
    sequence of those backward decisions.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

OP_M, OP_I, OP_D = 0, 1, 2


@lru_cache(maxsize=None)
def op_strings(a: int, b: int):
    """Every op string consuming a read bases (M, I) and b window bases (M, D)."""
    if a == 0 and b == 0:
        return ((),)
    out = []
    if a > 0 and b > 0:
        out += [s + (OP_M,) for s in op_strings(a - 1, b - 1)]
    if a > 0:
        out += [s + (OP_I,) for s in op_strings(a - 1, b)]
    if b > 0:
        out += [s + (OP_D,) for s in op_strings(a, b - 1)]
    return tuple(out)


@lru_cache(maxsize=None)
def path_table(a: int, b: int):
    """(ops, P, runs, gaps): P[k, qi*b+rj] = 1 if path k aligns q[qi] with r[rj]."""
    ops = op_strings(a, b)
    P = np.zeros((len(ops), max(a * b, 1)), dtype=np.float64)
    runs = np.zeros(len(ops), dtype=np.float64)
    gaps = np.zeros(len(ops), dtype=np.float64)
    for k, s in enumerate(ops):
        qi = rj = 0
        prev = None
        for op in s:
            if op == OP_M:
                P[k, qi * b + rj] = 1.0
                qi += 1
                rj += 1
            else:
                gaps[k] += 1
                if op != prev:
                    runs[k] += 1
                if op == OP_I:
                    qi += 1
                else:
                    rj += 1
            prev = op
    return ops, P, runs, gaps


def _subst(Qs, Rs, sc):
    """(N, a*b) substitution scores for read pieces Qs (N,a) and window pieces Rs (N,b)."""
    a_, b_ = sc[0], sc[1]
    eq = Qs[:, :, None] == Rs[:, None, :]
    return np.where(eq, float(a_), float(b_)).reshape(len(Qs), -1)


def _path_scores(Qs, Rs, sc):
    """(N, n_paths) score of every path for every pair of pieces."""
    a, b = Qs.shape[1], Rs.shape[1]
    ops, P, runs, gaps = path_table(a, b)
    gap_cost = sc[2] * runs + sc[3] * gaps
    if a * b == 0:
        return np.broadcast_to(-gap_cost, (len(Qs), len(ops)))
    return _subst(Qs, Rs, sc) @ P.T - gap_cost


def _combos(mode, m, n):
    """(read piece, window piece) ranges: ((qa, ql), (s, bl)), end cell (qa+ql, s+bl)."""
    if mode == 0:
        for s in range(n + 1):
            for bl in range(n - s + 1):
                yield (0, m), (s, bl)
    else:
        for qa in range(m):
            for ql in range(1, m - qa + 1):
                for s in range(n):
                    for bl in range(1, n - s + 1):
                        yield (qa, ql), (s, bl)


def best_batch(Q, R, mode, sc):
    """Optimal score and tie-broken end cell for N pairs of equal lengths.

    Q: (N, m) codes, R: (N, n) codes.  Returns (score, end_i, end_j) arrays.
    """
    N, m = Q.shape
    n = R.shape[1]
    best = np.full(N, -np.inf)
    bi = np.zeros(N, np.int64)
    bj = np.zeros(N, np.int64)
    if mode == 1:
        best[:] = 0.0  # the empty alignment at (0, 0)
    for (qa, ql), (s, bl) in _combos(mode, m, n):
        v = _path_scores(Q[:, qa:qa + ql], R[:, s:s + bl], sc).max(axis=1)
        ei, ej = qa + ql, s + bl
        better = v > best
        tie = (v == best) & ((ej < bj) | ((ej == bj) & (ei < bi)))
        if mode == 1:
            # the empty alignment (0,0) precedes every cell in the tie order
            tie &= ~((bi == 0) & (bj == 0))
        upd = better | tie
        best = np.where(upd, v, best)
        bi = np.where(upd, ei, bi)
        bj = np.where(upd, ej, bj)
    return best.astype(np.int64), bi, bj


def optimal_end_cells(q, r, mode, sc):
    """Set of all end cells of optimal alignments for one pair (and the score)."""
    q = np.asarray(q)[None, :]
    r = np.asarray(r)[None, :]
    m, n = q.shape[1], r.shape[1]
    vals = {}
    for (qa, ql), (s, bl) in _combos(mode, m, n):
        v = _path_scores(q[:, qa:qa + ql], r[:, s:s + bl], sc).max()
        cell = (qa + ql, s + bl)
        vals[cell] = max(vals.get(cell, -np.inf), v)
    if mode == 1:
        vals[(0, 0)] = max(vals.get((0, 0), -np.inf), 0.0)
    best = max(vals.values())
    return int(best), {c for c, v in vals.items() if v == best}


def decisions(ops, forced_lead_ins):
    """Backward decision sequence of an alignment, for the canonical order.

    In the match state the choices rank stop(0) < M(1) < D(2) < I(3); inside a
    gap, open-here(0) < extend(1).  A semi-global alignment that starts at
    window column 0 with an insertion run walks that run without choices.
    """
    toks = []
    lead = 0
    if forced_lead_ins:
        while lead < len(ops) and ops[lead] == OP_I:
            lead += 1
    k = len(ops)
    while k > lead:
        op = ops[k - 1]
        if op == OP_M:
            toks.append(1)
            k -= 1
            continue
        L = 0
        while k - L > lead and ops[k - 1 - L] == op:
            L += 1
        toks.append(2 if op == OP_D else 3)
        toks += [1] * (L - 1) + [0]
        k -= L
    toks.append(0)  # stop, or the forced column-0 insertion run then stop
    return tuple(toks)


def canonical(q, r, mode, sc):
    """Score, end cell, start cell and run-length CIGAR the traceback must give."""
    q = np.asarray(q)
    r = np.asarray(r)
    m, n = len(q), len(r)
    Qb = q[None, :]
    Rb = r[None, :]
    score, bi, bj = (int(x[0]) for x in best_batch(Qb, Rb, mode, sc))
    if mode == 1 and bi == 0 and bj == 0:
        return score, (0, 0), (0, 0), []
    cands = []
    for (qa, ql), (s, bl) in _combos(mode, m, n):
        if (qa + ql, s + bl) != (bi, bj):
            continue
        ops, _, _, _ = path_table(ql, bl)
        v = _path_scores(Qb[:, qa:qa + ql], Rb[:, s:s + bl], sc)[0]
        for k in np.nonzero(v == score)[0]:
            toks = decisions(ops[k], forced_lead_ins=(mode == 0 and s == 0))
            cands.append((toks, qa, s, ops[k]))
    cands.sort(key=lambda c: c[0])
    _, qa, s, ops = cands[0]
    runs = []
    for op in ops:
        if runs and runs[-1][1] == op:
            runs[-1][0] += 1
        else:
            runs.append([1, op])
    return score, (bi, bj), (qa, s), ["%d%s" % (L, "MID"[op]) for L, op in runs]


def rescore(q, r, read_start, ref_start, cigar_ops, sc):
    """Score of a CIGAR (list of (len, op)) placed at the given starts; also the end cell."""
    a_, b_, o, e = sc
    i, j = read_start, ref_start
    total = 0
    for L, op in cigar_ops:
        if op == OP_M:
            for _ in range(L):
                total += a_ if q[i] == r[j] else b_
                i += 1
                j += 1
        elif op == OP_I:
            total -= o + L * e
            i += L
        else:
            total -= o + L * e
            j += L
    return total, i, j


def enumerate_at_least(q, r, mode, sc, floor):
    """Every alignment scoring >= floor, by depth-first search (exhaustive).

    The search cuts a branch only when even matching every remaining base
    could not reach ``floor``, so no alignment at or above it is missed.
    Alignments that open with a gap (and, semi-global, end with a deletion)
    are never optimal, so they are not extended.  Returns a list of
    (score, start_i, start_j, end_i, end_j, ops).
    """
    a, b, o, e = sc
    q = [int(x) for x in q]
    r = [int(x) for x in r]
    m, n = len(q), len(r)
    out = []

    def dfs(i, j, score, ops, si, sj):
        prev = ops[-1] if ops else None
        if mode == 0 and i == m:
            if score >= floor:
                out.append((score, si, sj, i, j, tuple(ops)))
            return
        if mode == 1 and prev == OP_M and score >= floor:
            out.append((score, si, sj, i, j, tuple(ops)))
        rem = (m - i) if mode == 0 else min(m - i, n - j)
        if score + a * rem < floor:
            return
        if i < m and j < n:
            ops.append(OP_M)
            dfs(i + 1, j + 1, score + (a if q[i] == r[j] else b), ops, si, sj)
            ops.pop()
        if mode == 1 and not ops:
            return
        if i < m:
            ops.append(OP_I)
            dfs(i + 1, j, score - (e if prev == OP_I else o + e), ops, si, sj)
            ops.pop()
        if j < n and (mode == 1 or ops):
            ops.append(OP_D)
            dfs(i, j + 1, score - (e if prev == OP_D else o + e), ops, si, sj)
            ops.pop()

    if mode == 0:
        for s in range(n + 1):
            dfs(0, s, 0, [], 0, s)
    else:
        for i0 in range(m):
            for j0 in range(n):
                dfs(i0, j0, 0, [], i0, j0)
        if floor <= 0:
            out.append((0, 0, 0, 0, 0, ()))
    return out


def canonical_at_least(q, r, mode, sc, floor):
    """Like canonical(), by bounded exhaustive search; needs floor <= the optimum."""
    alns = enumerate_at_least(q, r, mode, sc, floor)
    if not alns:
        return None
    best = max(x[0] for x in alns)
    opt = [x for x in alns if x[0] == best]
    ei, ej = min(((x[3], x[4]) for x in opt), key=lambda c: (c[1], c[0]))
    if mode == 1 and (ei, ej) == (0, 0):
        return best, (0, 0), (0, 0), []
    cands = sorted((decisions(x[5], mode == 0 and x[2] == 0), x) for x in opt if (x[3], x[4]) == (ei, ej))
    x = cands[0][1]
    runs = []
    for op in x[5]:
        if runs and runs[-1][1] == op:
            runs[-1][0] += 1
        else:
            runs.append([1, op])
    return best, (ei, ej), (x[1], x[2]), ["%d%s" % (L, "MID"[op]) for L, op in runs]


# ---------------------------------------------------------------------------
# Extension mode: every alignment starts at the anchor (0, 0) with score h0 and
# ends at any cell (i, j); its score is h0 plus the path score (a leading gap
# at the anchor is an ordinary gap run).  The best early end is the largest
# score over (0, 0) and the cells with i, j >= 1 (ties: smallest j, then
# smallest i); the best end-to-end end is the largest over row m (ties:
# smallest j).  The read is aligned to its end when that scores at least the
# early end minus the clipping penalty.


def ext_end_scores(q, r, sc, h0):
    """{(i, j): best score of an anchored alignment ending at (i, j)}."""
    q = np.asarray(q)[None, :]
    r = np.asarray(r)[None, :]
    m, n = q.shape[1], r.shape[1]
    vals = {}
    for i in range(m + 1):
        for j in range(n + 1):
            vals[(i, j)] = h0 + float(_path_scores(q[:, :i], r[:, :j], sc).max())
    return vals


def ext_best(q, r, sc, h0, clip):
    """(score, (end_i, end_j)) chosen by the extension rules."""
    m, n = len(q), len(r)
    vals = ext_end_scores(q, r, sc, h0)
    lbest, lcell = float(h0), (0, 0)
    for j in range(1, n + 1):
        for i in range(1, m + 1):
            if vals[(i, j)] > lbest:
                lbest, lcell = vals[(i, j)], (i, j)
    gbest, gcell = vals[(m, 0)], (m, 0)
    for j in range(1, n + 1):
        if vals[(m, j)] > gbest:
            gbest, gcell = vals[(m, j)], (m, j)
    if gbest >= lbest - clip:
        return int(gbest), gcell
    return int(lbest), lcell


def decisions_ext(ops):
    """Backward decisions of an anchored alignment: a leading run of one gap
    kind is walked without choices once the walk reaches row 0 or column 0."""
    lead = 0
    if ops and ops[0] != OP_M:
        while lead < len(ops) and ops[lead] == ops[0]:
            lead += 1
    toks = []
    k = len(ops)
    while k > lead:
        op = ops[k - 1]
        if op == OP_M:
            toks.append(1)
            k -= 1
            continue
        L = 0
        while k - L > lead and ops[k - 1 - L] == op:
            L += 1
        toks.append(2 if op == OP_D else 3)
        toks += [1] * (L - 1) + [0]
        k -= L
    return tuple(toks)


def canonical_ext(q, r, sc, h0, clip):
    """Score, end cell and run-length CIGAR the extension traceback must give
    (the start is always the anchor (0, 0))."""
    q = np.asarray(q)
    r = np.asarray(r)
    score, (bi, bj) = ext_best(q, r, sc, h0, clip)
    ops, _, _, _ = path_table(bi, bj)
    v = h0 + _path_scores(q[None, :bi], r[None, :bj], sc)[0]
    cands = sorted((decisions_ext(ops[k]), ops[k]) for k in np.nonzero(v == score)[0])
    runs = []
    for op in cands[0][1]:
        if runs and runs[-1][1] == op:
            runs[-1][0] += 1
        else:
            runs.append([1, op])
    return score, (bi, bj), ["%d%s" % (L, "MID"[op]) for L, op in runs]
