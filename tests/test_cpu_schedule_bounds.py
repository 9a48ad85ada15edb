"""Host-side model of the device-memory requests of the stored-state tangent
action (the state-slab schedules) and of the element kernels' tile gather,
checked exhaustively on the CPU: every address a kernel requests lies inside
the buffer it reads.

The state of a linearisation is [E][10][Q^3] (F^-1 and mu - lambda ln J at
each Gauss point).  Thread t of a block serves element slab le = t / Q^2 and
Gauss-point column t2 = t mod Q^2; its slab pointer is
  sp = (valid ? e : 0) * 10 Q^3 + t2
and Gauss-point slab j of word k is read at sp + k Q^3 + j Q^2.  The model
enumerates the slabs each schedule requests -- the kept ones (DEPTH = 2 or 3
named buffers stepping q3 by DEPTH with the clamp min(q3 + DEPTH, Q - 1), and
the one-slab prefetch guarded by q3 + 1 < Q) and the unclamped variants of the
same schedules -- for P = 1..8, Q in {P+1, P+2}, every run length NE a block
can have, meshes with ragged last blocks and idle element slabs.  The
unclamped variants request slab Q (one buffer) or slabs Q, Q + 1 (two
buffers) in their last step and read past the element's block; for the last
element of the mesh that is past the end of the caller's state buffer, a
fault whenever the allocation ends at a page boundary.  The tile gather is
modelled the same way against [0, 3 Nn).  A last check follows the buffers
through the pipelined loop: each point reads the slab of its own index."""
import itertools

import pytest


def slabs_pipe(Q, clamp=True, depth=2):
    """Slabs requested by the schedule with `depth` named buffers, in order,
    and the slab each point of the loop consumes (buffer contents at use)."""
    cl = (lambda j: min(j, Q - 1)) if clamp else (lambda j: j)
    req = [cl(j) for j in range(depth)]    # every buffer before the forward pass
    for q3 in range(0, Q, depth):
        for b in range(depth):
            if b == 0 or Q % depth == 0 or q3 + b < Q:
                req.append(cl(q3 + b + depth))  # buffer b, after slab q3 + b is used
    return req


def pipe_uses(Q, depth):
    """(point, slab held by its buffer) for every point of the pipelined loop:
    buffer b holds the slab requested last into it."""
    cl = lambda j: min(j, Q - 1)
    held = [cl(j) for j in range(depth)]
    uses = []
    for q3 in range(0, Q, depth):
        for b in range(depth):
            if b == 0 or Q % depth == 0 or q3 + b < Q:
                uses.append((q3 + b, held[b]))
                held[b] = cl(q3 + b + depth)
    return uses


def slabs_one(Q, guard=True):
    """Slabs requested by the one-slab prefetch, in order."""
    req = [0]
    for q3 in range(Q):
        if not guard or q3 + 1 < Q:
            req.append(q3 + 1)
    return req


def slab_consumed(Q, sched):
    # every slab 0..Q-1 is requested (the schedule covers the column)
    return set(range(Q)) <= set(sched)


def state_addresses(P, Q, NE, nx, ny, nz, slabs):
    """All state word offsets requested by every thread of every block."""
    QQ, QQQ = Q * Q, Q * Q * Q
    bpr = (nx + NE - 1) // NE
    lo, hi = None, None
    for b in range(bpr * ny * nz):
        k, row = b % bpr, b // bpr
        ey, ez = row % ny, row // ny
        for t in range(NE * QQ):
            le, t2 = t // QQ, t % QQ
            ex = k * NE + le
            valid = ex < nx
            e = (ez * ny + ey) * nx + (ex if valid else 0)
            sp = (e if valid else 0) * 10 * QQQ + t2
            for j in slabs:
                for w in (0, 9):           # first and last word bound the range
                    a = sp + w * QQQ + j * QQ
                    lo = a if lo is None else min(lo, a)
                    hi = a if hi is None else max(hi, a)
    return lo, hi


def gather_addresses(P, NE, nx, ny, nz):
    """Extremes of the tile-gather indices (clamped rows and columns)."""
    n = P + 1
    Nx, Ny, Nz = nx * P + 1, ny * P + 1, nz * P + 1
    Nn = Nx * Ny * Nz
    TX = NE * P + 1
    ROWS = 3 * n * n
    bpr = (nx + NE - 1) // NE
    lo, hi = None, None
    for b in range(bpr * ny * nz):
        k, row = b % bpr, b // bpr
        ey, ez = row % ny, row // ny
        x0 = k * NE * P
        xe = Nx - x0
        assert xe >= 2
        for r, x in itertools.product(range(ROWS + 1), (0, TX - 1, TX + 3)):
            rr, xx = min(r, ROWS - 1), min(x, xe - 1)
            bb, cc, comp = rr % n, (rr // n) % n, rr // (n * n)
            g = comp * Nn + ((ez * P + cc) * Ny + (ey * P + bb)) * Nx + x0 + xx
            lo = g if lo is None else min(lo, g)
            hi = g if hi is None else max(hi, g)
    return lo, hi, 3 * Nn


ORDERS = [(P, Q) for P in range(1, 9) for Q in (P + 1, P + 2)]


@pytest.mark.parametrize("P,Q", ORDERS, ids=["P%dQ%d" % pq for pq in ORDERS])
def test_kept_state_schedules_stay_in_bounds(P, Q):
    QQ = Q * Q
    pipe, pipe3, one = slabs_pipe(Q), slabs_pipe(Q, depth=3), slabs_one(Q)
    assert slab_consumed(Q, pipe) and slab_consumed(Q, pipe3) and slab_consumed(Q, one)
    assert max(pipe) == Q - 1 and max(pipe3) == Q - 1 and max(one) == Q - 1
    for NE in range(1, max(1, 256 // QQ) + 1):
        # rows shorter, equal and longer than a block, with a ragged tail
        for nx, ny, nz in ((1, 1, 1), (NE, 1, 2), (NE + 1, 2, 1), (2 * NE + 3, 1, 1)):
            E = nx * ny * nz
            for slabs in (pipe, pipe3, one):
                lo, hi = state_addresses(P, Q, NE, nx, ny, nz, slabs)
                assert lo >= 0 and hi < E * 10 * Q ** 3, (P, Q, NE, nx, ny, nz)


@pytest.mark.parametrize("P,Q", ORDERS, ids=["P%dQ%d" % pq for pq in ORDERS])
def test_unclamped_schedules_leave_the_state_buffer(P, Q):
    # the last requests of the unclamped schedules fall past the element's
    # [10][Q^3] block: for the last element of the mesh, past the buffer end
    nx, ny, nz, NE = 3, 1, 1, 2
    E = nx * ny * nz
    end = E * 10 * Q ** 3
    for slabs in (slabs_pipe(Q, clamp=False), slabs_one(Q, guard=False)):
        _, hi = state_addresses(P, Q, NE, nx, ny, nz, slabs)
        assert hi >= end
    # at odd Q the two-buffer schedule's last step requests slab Q + 1 into
    # the buffer freed by slab Q - 1, at even Q slabs Q and Q + 1
    last = slabs_pipe(Q, clamp=False)[-1]
    assert last == Q + 1
    # words past the end (worst thread, last element): t2 + Q^2 (slab Q) or
    # t2 + 2 Q^2 (slab Q + 1) beyond 10 Q^3
    _, hi = state_addresses(P, Q, NE, nx, ny, nz, slabs_one(Q, guard=False))
    assert hi - end == Q * Q - 1


@pytest.mark.parametrize("P", range(1, 9))
def test_tile_gather_stays_in_bounds(P):
    for Q in (P + 1, P + 2):
        for NE in range(1, max(1, 256 // (Q * Q)) + 1):
            for nx, ny, nz in ((1, 1, 1), (NE + 1, 2, 1), (2 * NE + 1, 1, 2)):
                lo, hi, end = gather_addresses(P, NE, nx, ny, nz)
                assert lo >= 0 and hi < end


@pytest.mark.parametrize("depth", (2, 3))
@pytest.mark.parametrize("Q", range(2, 11))
def test_pipelined_points_read_their_own_slab(Q, depth):
    # every point q3 = 0..Q-1 runs exactly once, in order, and its buffer then
    # holds slab q3 (the clamp only repeats the last slab in requests that no
    # point consumes)
    uses = pipe_uses(Q, depth)
    assert [q for q, _ in uses] == list(range(Q))
    assert all(q == slab for q, slab in uses)
