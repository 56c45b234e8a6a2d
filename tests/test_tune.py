"""Host logic of the autotuner (no GPU): the shape-bucket rule documented with
ftg_tune_set, JSON persistence, and applying a table through a handle; the GPU
test tunes two shapes through the C ABI and checks the handle returns the choice."""
import pytest

from paper_2104_00897_amd import tune


def test_bucket_rule():
    # ceil(log2 x) clamped to [4, 15]
    assert [tune.bucket(x) for x in (1, 2, 16, 17, 32, 33, 1000, 1024, 1025, 32768, 10 ** 9)] == \
        [4, 4, 4, 5, 5, 6, 10, 10, 11, 15, 15]


def test_json_round_trip_and_apply():
    t = tune.TuneTable()
    t.set(0, 100, 200, 300, 3)
    t.set(0, 8192, 8192, 8192, 2)
    t.set(2, 4096, 8192, 4096, 1)
    u = tune.TuneTable.from_json(t.to_json())
    assert u.entries == t.entries
    assert u.get(0, 120, 250, 400) == 3 and u.get(0, 5000, 5000, 5000) == 2 and u.get(1, 64, 64, 64) == 0
    calls = []

    class FakeHandle:
        def tune_set(self, dt, m, n, k, tile):
            calls.append((dt, m, n, k, tile))
    u.apply(FakeHandle())
    # each call lands in the same bucket it came from
    assert sorted((dt, tune.bucket(m), tune.bucket(n), tune.bucket(k), tl) for dt, m, n, k, tl in calls) == \
        sorted((*key, v) for key, v in t.entries.items())
    with pytest.raises(ValueError):
        tune.TuneTable.from_json('{"version": 2, "entries": []}')


@pytest.mark.gpu
def test_autotune_sets_handle():
    from paper_2104_00897_amd import ftgemm
    h = ftgemm.Handle(capacity=64)
    t = tune.autotune(h, [(384, 256, 200), (1024, 1024, 512)], steps=2, warmup=1)
    for m, n, k in [(384, 256, 200), (1024, 1024, 512)]:
        assert t.get(ftgemm.F64, m, n, k) in tune.FP64_TILES
        assert h.tune_get(ftgemm.F64, m, n, k) == t.get(ftgemm.F64, m, n, k)
    t2 = tune.autotune(h, [(512, 512, 256)], dtype=ftgemm.BF16, steps=2, warmup=1)
    assert t2.get(ftgemm.BF16, 512, 512, 256) in tune.LOWP_TILES
    assert h.tune_get(ftgemm.BF16, 512, 512, 256) == t2.get(ftgemm.BF16, 512, 512, 256)
    h.close()
