"""Independent model of the tiled right-looking Cholesky DAG (test side).

Derived from the paper, not from the library: the four tile operations of
Methods ("Tiled Cholesky Decomposition") with their read / read-write tile
sets, issued in the loop order of Fig. 1, with OpenMP in/inout dependency
semantics (Methods, "Implementations": a task waits for the last writer of
every tile it reads or writes, and a writer also waits for the readers since
that writer).

Work units refine tile tasks into CHOL_BLOCK-row blocks, exactly as the C ABI
documents them; their block-level read/write sets follow from the same
operation definitions.  The POTRF and TRSM tasks of a tile column are blocked
by CHOL_BLOCK-wide sub-columns: the panel of Fig. 1's step J is itself
factored right-looking with tile side CHOL_BLOCK (POTRF of the diagonal
block, TRSM of every block below it, update of the panel's later
sub-columns), after which the step's SYRK/GEMM trailing update runs with
K-depth T.  program_key gives that blocked program order.
"""
from __future__ import annotations

import math
from collections import defaultdict

BLK = 128
POTRF, TRSM, UPDATE, PANEL = 0, 1, 2, 3


class Geom:
    def __init__(self, n: int, T: int):
        self.n, self.T = n, T
        self.M = math.ceil(n / T)
        self.SB = math.ceil(min(T, n) / BLK)
        self.SBL = math.ceil((n - (self.M - 1) * T) / BLK)

    def tdim(self, I):
        return min(self.T, self.n - I * self.T)

    def sb(self, I):
        return self.SBL if I == self.M - 1 else self.SB

    def gid(self, I, a):
        return I * self.SB + a

    @property
    def NRB(self):
        return (self.M - 1) * self.SB + self.SBL

    def split(self, r):
        return r // self.SB, r % self.SB


# --------------------------------------------------------------- tile level
def tile_tasks(M: int):
    """Tile tasks of Fig. 1 in program order: (kind, J, I, K, reads, writes)."""
    out = []
    for J in range(M):
        out.append(("POTRF", J, J, J, [], [(J, J)]))
        for I in range(J + 1, M):
            out.append(("TRSM", J, I, J, [(J, J)], [(I, J)]))
        for I in range(J + 1, M):
            out.append(("SYRK", J, I, I, [(I, J)], [(I, I)]))
            for K in range(J + 1, I):
                out.append(("GEMM", J, I, K, [(I, J), (K, J)], [(I, K)]))
    return out


def dependency_edges(tasks):
    """Edges (p, q), p before q, from in/inout semantics on tiles."""
    last_writer = {}
    readers = defaultdict(list)
    edges = set()
    for q, (_, _, _, _, reads, writes) in enumerate(tasks):
        for t in reads:
            if t in last_writer:
                edges.add((last_writer[t], q))
        for t in writes:
            if t in last_writer:
                edges.add((last_writer[t], q))
            for r in readers[t]:
                if r != q:
                    edges.add((r, q))
        for t in reads:
            readers[t].append(q)
        for t in writes:
            last_writer[t] = q
            readers[t] = []
    return edges


def critical_path(tasks, edges) -> int:
    succ = defaultdict(list)
    for p, q in edges:
        succ[p].append(q)
    depth = [1] * len(tasks)
    for p in range(len(tasks)):  # program order is topological
        for q in succ[p]:
            depth[q] = max(depth[q], depth[p] + 1)
    return max(depth) if depth else 0


# --------------------------------------------------------------- unit level
def unit_access(g: Geom, u):
    """Block-level (reads, writes) of a work unit {kind, J, I, a, K, b};
    a block is a pair of global block ids (row block, column block)."""
    kind, J, I, a, K, b = (int(x) for x in u)
    if kind == POTRF:
        gs = g.gid(J, a)
        return [], [(gs, gs)]
    if kind == TRSM:
        gs = g.gid(J, K)
        return [(gs, gs)], [(g.gid(I, a), gs)]
    if kind == PANEL:
        gs, gt, r = g.gid(J, K), g.gid(J, b), g.gid(I, a)
        return [(r, gs), (gt, gs)], [(r, gt)]
    ri, rk = g.gid(I, a), g.gid(K, b)
    reads = [(ri, g.gid(J, y)) for y in range(g.sb(J))] + [(rk, g.gid(J, y)) for y in range(g.sb(J))]
    return reads, [(ri, rk)]


def program_key(g: Geom, u):
    """Position of a unit in the blocked program order of Fig. 1: step J,
    then its panel sub-columns s in order (POTRF, the TRSMs below, the panel
    updates), then the step's trailing update."""
    kind, J, I, a, K, b = (int(x) for x in u)
    if kind == POTRF:
        return (J, a, 0, 0, 0)
    if kind == TRSM:
        return (J, K, 1, g.gid(I, a), 0)
    if kind == PANEL:
        return (J, K, 2, b, g.gid(I, a))
    return (J, g.SB + 1, 3, g.gid(I, a), g.gid(K, b))


def program_order_units(g: Geom):
    """All work units in the blocked program order."""
    out = []
    for J in range(g.M):
        for s in range(g.sb(J)):
            gs = g.gid(J, s)
            out.append((POTRF, J, J, s, -1, -1))
            for r in range(gs + 1, g.NRB):
                out.append((TRSM, J, *g.split(r), s, -1))
            for s2 in range(s + 1, g.sb(J)):
                for r in range(g.gid(J, s2), g.NRB):
                    out.append((PANEL, J, *g.split(r), s, s2))
        for I in range(J + 1, g.M):
            for K in range(J + 1, I + 1):
                for a in range(g.sb(I)):
                    for b in range(g.sb(K)):
                        if I == K and b > a:
                            continue
                        out.append((UPDATE, J, I, a, K, b))
    return out


def check_ticket_order(g: Geom, units):
    """Every conflicting pair of accesses to a block (at least one a write)
    must appear in ticket order as in program order.  Returns the list of
    violations (empty when the order is valid)."""
    acc = defaultdict(list)  # block -> [(program key, ticket, is_write)]
    for t, u in enumerate(units):
        key = program_key(g, u)
        reads, writes = unit_access(g, u)
        for blk in reads:
            acc[blk].append((key, t, False))
        for blk in writes:
            acc[blk].append((key, t, True))
    bad = []
    for blk, lst in acc.items():
        lst.sort()
        last_write_ticket = -1
        max_read_ticket_since = -1
        i = 0
        while i < len(lst):
            # accesses of the same tile task to one block are never in conflict
            j = i
            while j < len(lst) and lst[j][0] == lst[i][0]:
                j += 1
            group = lst[i:j]
            for key, t, w in group:
                if t < last_write_ticket:
                    bad.append((blk, key, t, "after-write"))
                if w and t < max_read_ticket_since:
                    bad.append((blk, key, t, "write-after-read"))
            writes = [t for _, t, w in group if w]
            reads = [t for _, t, w in group if not w]
            if writes:
                last_write_ticket = max(writes)
                max_read_ticket_since = -1
            if reads:
                max_read_ticket_since = max([max_read_ticket_since] + reads)
            i = j
    return bad
