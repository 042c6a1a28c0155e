"""CPU model of the fused batched launch's work distribution.

The launch clears one ticket, then a grid of persistent workgroups loops:
take t = fetch_add(ticket, 1); stop once t >= items; otherwise find the
dataset whose item range holds t (items are the row blocks of every dataset
in order) and encode that row block completely -- projection tiles, then
quantize -- before taking the next ticket.  No workgroup waits for another.
The model runs that loop under adversarial schedules (a residency limit with
workgroups started only as others leave, random and reversed interleavings,
one workgroup starved until the end) and checks: every row of every dataset
is encoded exactly once, every workgroup leaves after a bounded number of
tickets, and a second launch needs the clear (without it nothing is done).
"""
import itertools
import random


def layout(ns, rows):
    """(first_item, tiles_m) per dataset, as the batch planner lays them out."""
    out, items = [], 0
    for n in ns:
        t = (n + rows - 1) // rows if n > 0 else 0
        out.append((items, t))
        items += t
    return out, items


def owner(sets, t):
    d = 0
    while d + 1 < len(sets) and t >= sets[d + 1][0]:
        d += 1
    return d, t - sets[d][0]


def run_launch(ns, rows, grid, ticket, order, resident=None, rng=None):
    """One launch. `ticket` is a one-element list (the device word);
    `order` picks which runnable workgroup makes the next step."""
    sets, items = layout([n for n in ns if n > 0], rows)
    live = [n for n in ns if n > 0]
    done = [[0] * n for n in live]
    started = list(range(grid if resident is None else min(resident, grid)))
    waiting = list(range(len(started), grid))
    state = {w: "claim" for w in started}
    claims = {w: 0 for w in range(grid)}
    steps = 0
    while state:
        w = order(sorted(state), steps, rng)
        steps += 1
        assert steps < 10 * (items + grid) + 100, "a workgroup never leaves"
        t = ticket[0]
        ticket[0] += 1                 # atomic fetch-and-add
        claims[w] += 1
        if t >= items:
            del state[w]
            if waiting:                # a slot frees up: the next workgroup starts
                nw = waiting.pop(0)
                state[nw] = "claim"
            continue
        d, tm = owner(sets, t)
        for r in range(tm * rows, min((tm + 1) * rows, live[d])):
            done[d][r] += 1
    return done, claims, items


ORDERS = {
    "round_robin": lambda ws, s, rng: ws[s % len(ws)],
    "lowest_first": lambda ws, s, rng: ws[0],
    "highest_first": lambda ws, s, rng: ws[-1],
    "random": lambda ws, s, rng: rng.choice(ws),
    "starve_zero": lambda ws, s, rng: ws[1] if len(ws) > 1 else ws[0],
}


def test_every_row_once_under_adversarial_schedules():
    rng = random.Random(5)
    shapes = [[10_000, 777, 0, 99, 129], [1, 64, 65, 128], [5000], [0, 0, 300]]
    for ns, rows, grid, resident, (name, order) in itertools.product(
            shapes, (64, 128), (1, 3, 16, 1000), (None, 2), ORDERS.items()):
        ticket = [0]
        done, claims, items = run_launch(ns, rows, grid, ticket, order, resident, rng)
        for d, rows_done in enumerate(done):
            assert all(c == 1 for c in rows_done), (ns, rows, grid, name, d)
        # every workgroup that ran took at most one ticket past the end
        assert sum(claims.values()) == items + grid, (ns, rows, grid, name)
        assert ticket[0] == items + grid


def test_second_launch_needs_the_cleared_ticket():
    ns, rows, grid = [3000, 500], 128, 8
    ticket = [0]
    run_launch(ns, rows, grid, ticket, ORDERS["random"], None, random.Random(1))
    # no clear: the ticket is already past the item count, nothing is encoded
    done, _, _ = run_launch(ns, rows, grid, ticket, ORDERS["random"], None, random.Random(2))
    assert all(c == 0 for rows_done in done for c in rows_done)
    ticket[0] = 0                      # the clear kernel
    done, _, _ = run_launch(ns, rows, grid, ticket, ORDERS["random"], None, random.Random(3))
    assert all(c == 1 for rows_done in done for c in rows_done)


def test_item_layout_covers_each_dataset():
    for ns in ([1, 2, 3], [128, 129, 255, 256], [1_000_000, 12_345]):
        for rows in (64, 128):
            sets, items = layout(ns, rows)
            seen = [0] * sum(ns)
            base = [0] + list(itertools.accumulate(ns))
            for t in range(items):
                d, tm = owner(sets, t)
                for r in range(tm * rows, min((tm + 1) * rows, ns[d])):
                    seen[base[d] + r] += 1
            assert all(c == 1 for c in seen)
