"""Many independent chains on one GPU: footprint-packed batches.

Independent Markov chains are the paper's preferred parallelism whenever
memory allows (Sec. 3).  Chains of very uneven size are packed into groups
whose per-sweep scratch fits a budget (first fit, largest first); every group
is one lc_batch, i.e. one captured launch sequence per sweep over all of its
members.  All groups use the same stream, so they share one scratch arena in
the library: device memory is the world lines of every chain plus the
scratch of the largest group.  The grid size of each group, and with
autotune_tiles its linking-tile shape, is chosen by the library's autotuner.
Results of every chain equal its alone-run bit for bit (schedule, tile shape
and grouping never change the arithmetic).
"""
from __future__ import annotations

from . import Batch, Chain, DEFAULT_GRIDS, DEFAULT_TILE_SHAPES, lc_footprint_parts


def pack(scratch: list, budget: int) -> list:
    """First-fit decreasing: groups of indices whose scratch sums stay within
    budget (a chain larger than the budget gets a group of its own)."""
    order = sorted(range(len(scratch)), key=lambda i: -scratch[i])
    groups, room = [], []
    for i in order:
        for g, r in enumerate(room):
            if scratch[i] <= r:
                groups[g].append(i)
                room[g] -= scratch[i]
                break
        else:
            groups.append([i])
            room.append(budget - scratch[i])
    return [sorted(g) for g in groups]


class BatchRunner:
    """Owns no chains: runs the given chains in footprint-packed batches."""

    def __init__(self, chains: list, scratch_budget: int, stream=None):
        self.chains = list(chains)
        self.scratch = [lc_footprint_parts(c.L, c.S, c.beta)[1] for c in self.chains]
        self.groups = pack(self.scratch, int(scratch_budget))
        self.batches = []
        for g in self.groups:
            b = Batch(stream)
            for i in g:
                b.add(self.chains[i])
            self.batches.append(b)
        self.grids = [0] * len(self.batches)

    def autotune(self, grids=DEFAULT_GRIDS, trial_sweeps: int = 1) -> list:
        """Choose each group's grid size; the trial sweeps advance every chain
        by len(grids) * (trial_sweeps + 1) unaccumulated sweeps."""
        out = []
        for k, b in enumerate(self.batches):
            best, ms = b.autotune(grids, trial_sweeps)
            self.grids[k] = best
            out.append((best, ms))
        return out

    def autotune_tiles(self, shapes=DEFAULT_TILE_SHAPES, grids=DEFAULT_GRIDS,
                       trial_sweeps: int = 1) -> list:
        """Choose each group's (tile shape, grid) pair; every chain advances by
        len(shapes) * len(grids) * (trial_sweeps + 1) unaccumulated sweeps.
        Returns [(shape, grid, ms per sweep)] per group."""
        out = []
        for k, b in enumerate(self.batches):
            shape, grid, ms = b.autotune_tiles(shapes, grids, trial_sweeps)
            self.grids[k] = grid
            out.append((shape, grid, ms))
        return out

    def update(self, n_sweeps: int = 1, accumulate: bool = True):
        for b in self.batches:
            b.update(n_sweeps, accumulate)

    def close(self):
        for b in self.batches:
            b.close()
        self.batches = []
