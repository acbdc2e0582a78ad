"""Host logic of the server's workspace pool: first-fit ranges with merged
free neighbours, checked against a byte map on random take/give sequences."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def test_pool_matches_byte_map():
    from paper_1701_07181_amd.serve import WorkspacePool

    A = WorkspacePool.ALIGN
    rng = np.random.default_rng(7)
    pool = WorkspacePool(64 * A, torch.device("cpu"))
    used = np.zeros(pool.size // A, dtype=bool)
    live = []
    for _ in range(2000):
        if live and (rng.random() < 0.45 or len(live) > 12):
            off, n = live.pop(int(rng.integers(len(live))))
            pool.give(off, n)
            used[off // A:(off + WorkspacePool.round(n)) // A] = False
        else:
            n = int(rng.integers(1, 12 * A))
            k = WorkspacePool.round(n) // A
            off = pool.take(n)
            # first fit: the lowest run of k free units, if any
            runs = [i for i in range(len(used) - k + 1) if not used[i:i + k].any()]
            if off is None:
                assert not runs
                continue
            assert off % A == 0 and off // A == runs[0]
            used[off // A:off // A + k] = True
            live.append((off, n))
        # free list: ascending, disjoint, merged, and equal to the map's free units
        fl = pool.free
        assert all(fl[q][0] + fl[q][1] < fl[q + 1][0] for q in range(len(fl) - 1))
        free_units = np.ones_like(used)
        free_units[:] = False
        for off, size in fl:
            free_units[off // A:(off + size) // A] = True
        assert np.array_equal(free_units, ~used)
    assert pool.free_bytes() == pool.size - int(used.sum()) * A


def test_pool_round_and_view():
    from paper_1701_07181_amd.serve import WorkspacePool

    pool = WorkspacePool(1000, torch.device("cpu"))
    assert pool.size == 1024 and WorkspacePool.round(1) == 256 and WorkspacePool.round(256) == 256
    off = pool.take(300)
    assert off == 0 and pool.view(off, 300).numel() == 300
    assert pool.take(800) is None and pool.take(512) == 512
    pool.give(0, 300)
    assert pool.free == [[0, 512]]
