"""CPU check of the block-Jacobi kernels' index arithmetic (no GPU).

Restates, lane by lane, the indexing of the inversion kernel (one wave packs
G = 64 / bs diagonal blocks: lane = g bs + i, row i of block g) and of the
application kernel (groups of G blocks per wave, grid-stride over groups),
with the launch grids the host code computes, and checks that every access
stays inside its buffer: the CSR rows, the LDS tile (64 rows x 129 columns),
the LDS staging of x (64 entries per wave), the inverse storage the
workspace reserves (per wave group of G = 64 / bs blocks, bs columns of
G bs entries: Minv[grp][c][lane]) and the vectors (n rows),
for block sizes 1, 24, 42 and 64 (and 8, 64 / bs not integral for 24 and 42)
with ragged last blocks."""
import numpy as np
import pytest

WAVE, NWAVES, BJ_MAX = 64, 4, 64


def invert_accesses(n, bs):
    nblk = -(-n // bs)
    G = WAVE // bs
    grid = -(-nblk // G)  # host: (nblk + per_wave - 1) / per_wave
    minv_size = grid * bs * G * bs  # workspace: ngrp * bs * (G bs) entries
    seen_rows = np.zeros(n, bool)
    seen_minv = np.zeros(minv_size, bool)
    for bid in range(grid):
        for lane in range(WAVE):
            g = lane // bs
            i = lane - g * bs
            blk = bid * G + g
            r0 = blk * bs
            m = min(n - r0, bs) if (g < G and blk < nblk) else 0
            base = g * bs
            assert 0 <= lane < WAVE  # LDS row of the lane
            if i < m:
                r = r0 + i
                assert 0 <= r < n
                seen_rows[r] = True
                # LDS rows the lane reads in the elimination (pivot search, swaps, the pivot row)
                assert base + m - 1 < WAVE
                assert 2 * m <= 2 * BJ_MAX < 2 * BJ_MAX + 1
                for c in range(m):
                    idx = (bid * bs + c) * (G * bs) + lane
                    assert 0 <= idx < minv_size
                    assert not seen_minv[idx]
                    seen_minv[idx] = True
            if m > 0:
                assert 0 <= g < WAVE  # pivot slot
    assert seen_rows.all()
    # every stored entry of every (possibly ragged) block is written once
    expected = sum(min(bs, n - b * bs) ** 2 for b in range(nblk))
    assert seen_minv.sum() == expected
    return seen_minv


def apply_accesses(n, bs, max_grid=1 << 20, written=None):
    nblk = -(-n // bs)
    G = WAVE // bs
    ngrp = -(-nblk // G)
    grid = min(-(-ngrp // NWAVES), max_grid)
    minv_size = ngrp * bs * G * bs
    seen = np.zeros(n, bool)
    for b in range(grid):
        for wid in range(NWAVES):
            grp = b * NWAVES + wid
            while grp < ngrp:
                for lane in range(WAVE):
                    g = lane // bs
                    i = lane - g * bs
                    blk = grp * G + g
                    r0 = blk * bs
                    m = min(n - r0, bs) if (g < G and blk < nblk) else 0
                    if i < m:
                        assert 0 <= r0 + i < n
                        assert not seen[r0 + i]
                        seen[r0 + i] = True
                        for c in range(m):
                            assert 0 <= g * bs + c < WAVE  # staged x of the wave
                            idx = (grp * bs + c) * (G * bs) + lane
                            assert 0 <= idx < minv_size
                            # every inverse entry read was written by the inversion
                            assert written is None or written[idx]
                grp += grid * NWAVES
    assert seen.all()


@pytest.mark.parametrize("bs", [1, 8, 24, 42, 64])
@pytest.mark.parametrize("n", [4096, 4113, 1000, 65, 7])
def test_block_jacobi_index_bounds(n, bs):
    written = invert_accesses(n, bs)
    apply_accesses(n, bs, written=written)


def test_apply_grid_stride_with_a_capped_grid():
    # a grid smaller than the groups (the host caps it at 2^20 blocks): the
    # grid-stride loop still visits every row exactly once
    apply_accesses(5000, 8, max_grid=3)
    apply_accesses(5003, 42, max_grid=2)
