"""Host check of how the FP64 pass kernel steps from one tile to the next.

A pass tile holds V chosen global bits of vec(rho); the remaining global bits are enumerated by
the tile index through a run table (maximal runs of bits outside the tile, lowest first, each
taking the next tile-index bits), and a tile's base offset is that table applied to its index.
The kernel walks each workgroup's contiguous range of tiles and forms the next base as
((base | ~M) + 1) & M, with M the union of the runs. This test builds the run table the same
way as the pass geometry does and checks that the increment reproduces the table walk, for
every tile of small states and for random tiles of 16-qubit ones."""
import random

import pytest

MASK64 = (1 << 64) - 1


def runs_of(nb, vmask):
    """Maximal runs of global bits outside vmask, lowest first: (src, len, dst)."""
    runs, src, b = [], 0, 0
    while b < nb:
        if (vmask >> b) & 1:
            b += 1
            continue
        e = b
        while e < nb and not (vmask >> e) & 1:
            e += 1
        runs.append((src, e - b, b))
        src += e - b
        b = e
    return runs


def walk(runs, tile):
    """The kernel's run-table base of a tile."""
    base = 0
    for src, ln, dst in runs:
        base |= ((tile >> src) & ((1 << ln) - 1)) << dst
    return base


def step(base, m):
    return ((base | (~m & MASK64)) + 1) & m


def random_vmask(rng, nb, v):
    return sum(1 << b for b in rng.sample(range(nb), v))


@pytest.mark.parametrize("seed", range(20))
def test_increment_matches_run_table_small(seed):
    rng = random.Random(seed)
    nb = rng.randint(6, 14)
    v = rng.randint(1, nb - 2)
    vmask = random_vmask(rng, nb, v)
    runs = runs_of(nb, vmask)
    m = 0
    for _, ln, dst in runs:
        m |= ((1 << ln) - 1) << dst
    assert m == ((1 << nb) - 1) & ~vmask
    ntiles = 1 << (nb - v)
    base = walk(runs, 0)
    assert base == 0
    for t in range(ntiles - 1):
        base = step(base, m)
        assert base == walk(runs, t + 1), (nb, vmask, t)


@pytest.mark.parametrize("seed", range(10))
def test_increment_matches_run_table_16_qubits(seed):
    # 32 global bits, a 12-bit FP64 tile: the low bits and the row/column bits of four qubits
    rng = random.Random(100 + seed)
    nb, n = 32, 16
    qubits = rng.sample(range(n), 4)
    bits = set(range(4)) | {q for q in qubits} | {q + n for q in qubits}
    low = 4
    while len(bits) < 12:
        bits.add(low)
        low += 1
    vmask = sum(1 << b for b in bits)
    runs = runs_of(nb, vmask)
    m = 0
    for _, ln, dst in runs:
        m |= ((1 << ln) - 1) << dst
    ntiles = 1 << (nb - len(bits))
    for _ in range(200):
        t = rng.randrange(ntiles - 1)
        assert step(walk(runs, t), m) == walk(runs, t + 1)
    # the contiguous range of one workgroup of a 256-workgroup grid, stepped end to end
    per = ntiles // 256
    first = rng.randrange(256) * per
    base = walk(runs, first)
    for t in range(first, first + per - 1):
        base = step(base, m)
    assert base == walk(runs, first + per - 1)
