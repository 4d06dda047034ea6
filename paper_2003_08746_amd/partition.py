"""Balanced partition of the grid into per-process blocks (Sec. 4, Alg. 1).

Along one direction, the points go to the parts so that sizes differ by at
most one and the larger parts come first.  Part p of P over N points is the
number of points n in [0, N) with n = p (mod P), that is ceil((N - p) / P):
the round-robin deal of the points, which is balanced by construction.  The same rule applies to each direction of
a process grid.  A multi-GPU run of this path would size its per-GPU shards
this way (one block per GPU, halo exchange between neighbours); one GPU runs
one such shard.
"""


def part_size(total: int, nparts: int, index: int) -> int:
    """Points of part `index` (0-based) of `nparts` along a direction of
    `total` points."""
    if total < 0 or nparts < 1 or not 0 <= index < nparts:
        raise ValueError(f"partition: total={total}, nparts={nparts}, index={index}")
    return (total - index + nparts - 1) // nparts


def part_sizes(total: int, nparts: int) -> list:
    return [part_size(total, nparts, p) for p in range(nparts)]


def part_offsets(total: int, nparts: int) -> list:
    """First point of each part (parts are contiguous, in index order)."""
    out, start = [], 0
    for s in part_sizes(total, nparts):
        out.append(start)
        start += s
    return out


def block_shape(dims, parts, index):
    """Local block extent of process `index` (one index per direction) in a
    process grid of `parts` blocks per direction over a grid of `dims` points."""
    return tuple(part_size(n, p, q) for n, p, q in zip(dims, parts, index))
