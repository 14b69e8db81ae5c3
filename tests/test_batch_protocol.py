"""CPU model of the batched kernel's work protocol (host logic, no GPU).

Persistent workgroups take tasks (parts of systems) from one queue in order;
the parts of a system are consecutive in the queue (largest systems first)
and wait for each other at group barriers, so a part can only finish once all
parts of its system are running.  The model checks that the protocol always
drains when every workgroup is resident at once (which the cooperative launch
guarantees) and a system never has more parts than the grid has workgroups,
and that it can stall when fewer workgroups are resident than a system has
parts (the case the cooperative launch rules out).  It also checks the LDS
bytes of every workgroup shape the autotuner may pick against the 160 KiB of
LDS per workgroup at the batched workloads' sizes.
"""

import math
import random

import pytest

PART_ROWS = 16384
MAX_PARTS = 256
RED = 5  # values per group reduction: four window dots and a norm
SKETCH_PARTS = 4
CANDS = [(512, 4), (256, 4), (512, 2), (1024, 2), (1024, 4), (1024, 1)]


def make_tasks(ns, CH, G):
    """The queue as the host builds it: largest systems first, each split into
    P parts of whole chunks (P <= grid)."""
    tasks = []
    for i in sorted(range(len(ns)), key=lambda i: -ns[i]):
        nchs = math.ceil(ns[i] / CH)
        P = max(1, min(math.ceil(ns[i] / PART_ROWS), nchs, MAX_PARTS, G))
        tasks += [(i, q, P) for q in range(P)]
    return tasks


def drains(tasks, resident):
    """True if `resident` workgroups running the queue protocol finish every
    task: a free workgroup takes the next task; a system's parts finish
    together once all of them are held."""
    pos = 0
    held = {}  # system -> parts held
    free = resident
    done = 0
    while done < len(tasks):
        progressed = False
        while free and pos < len(tasks):  # free workgroups take tasks in queue order
            sid, _, P = tasks[pos]
            held[sid] = held.get(sid, 0) + 1
            pos += 1
            free -= 1
            progressed = True
        for sid in [s for s, h in held.items() if h == tasks_parts(tasks, s)]:
            free += held.pop(sid)
            done += tasks_parts(tasks, sid)
            progressed = True
        if not progressed:
            return False
    return True


def tasks_parts(tasks, sid):
    for s, _, P in tasks:
        if s == sid:
            return P
    raise KeyError(sid)


@pytest.mark.parametrize("seed", range(20))
def test_queue_drains_when_all_workgroups_are_resident(seed):
    rng = random.Random(seed)
    G = rng.choice([64, 256, 512, 1024])
    ns = [rng.randint(16384, 4 << 20) for _ in range(rng.randint(1, 300))]
    tasks = make_tasks(ns, 2048, G)
    assert max(P for _, _, P in tasks) <= G
    assert drains(tasks, G)


def test_queue_can_stall_with_fewer_resident_workgroups_than_parts():
    # one system of 64 parts behind others: with 63 resident workgroups the
    # parts held can never all run together
    ns = [64 * PART_ROWS] + [PART_ROWS] * 10
    tasks = make_tasks(ns, 2048, 256)
    assert not drains(tasks, 63)
    assert drains(tasks, 64)


def batch_lds_bytes(block, R, d, s, zeta):
    """LDS of one batched workgroup: one staged chunk vector (or the raw
    pattern), the reduction scratch, the sketch accumulator, the piece sums, y,
    the list starts and counters and the lists of one chunk."""
    CH = block * R
    vals = max(CH, (zeta * CH + 3) // 4)
    doubles = vals + (block // 64) * RED + RED + s + s * SKETCH_PARTS + d
    return 8 * doubles + 4 * (2 * s + 1) + 2 * zeta * CH


@pytest.mark.parametrize("block,R", CANDS)
@pytest.mark.parametrize("d,s,zeta", [(100, 200, 8), (40, 90, 8), (200, 400, 8)])
def test_every_shape_fits_lds(block, R, d, s, zeta):
    assert batch_lds_bytes(block, R, d, s, zeta) <= 160 * 1024
