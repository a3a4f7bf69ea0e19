"""Autotuner host logic (CPU): candidate space, pattern keys, cache round trip."""
import numpy as np

from paper_2306_14337_amd import autotune, binding, kktgen


def test_candidates_are_valid_options():
    for full in (False, True):
        cands = autotune.candidates(full)
        assert cands[0]["schedule"] == 2 and cands[0]["sync_mode"] == 2
        assert len({tuple(sorted(c.items())) for c in cands}) == len(cands)
        for c in cands:
            o = binding.options(**c)  # every knob is a field of the C options struct
            assert o.schedule in (1, 2)


def test_pattern_key_depends_on_pattern_only():
    p = kktgen.make_kkt(50, 3)
    k1 = autotune.pattern_key(p.n, p.rowptr, p.colind)
    k2 = autotune.pattern_key(p.n, p.rowptr.copy(), p.colind.copy())
    q = kktgen.make_kkt(50, 4)
    assert k1 == k2 and k1 != autotune.pattern_key(q.n, q.rowptr, q.colind)


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "cache.json")
    assert autotune.load_cache(path) == {}
    autotune.store_cache("abc", {"options": {"schedule": 2}, "seconds_per_step": 1e-3}, path)
    autotune.store_cache("def", {"options": {"schedule": 1}, "seconds_per_step": 2e-3}, path)
    c = autotune.load_cache(path)
    assert c["abc"]["options"] == {"schedule": 2} and c["def"]["options"] == {"schedule": 1}


def test_refinements_vary_segments_dense_block_and_kernels():
    best = autotune.candidates()[0]
    ref = autotune.refinements(best)
    assert {r.get("solve_thin_rows") for r in ref} >= {-1, 16}
    assert any(r.get("dense_tail") == -1 for r in ref)
    assert any(r.get("refactor_short_rows") == -1 for r in ref)
    assert any(r.get("refactor_long_rows") == -1 for r in ref)
    assert any(r.get("refactor_short_band") == 256 for r in ref)
    varied = ("solve_thin_rows", "dense_tail", "refactor_short_rows", "refactor_long_rows",
              "refactor_short_band")
    for r in ref:
        binding.options(**r)  # valid option fields
        assert {k: v for k, v in r.items() if k not in varied} == best
    assert autotune.refinements(dict(schedule=1, sync_mode=0)) == []


def test_batch_candidates_and_key():
    for full in (False, True):
        cands = autotune.batch_candidates(full)
        assert cands[0] == {} and len(cands) == len({repr(c) for c in cands})
        for c in cands[1:]:
            assert len(c) == 1
            binding.options(**c)  # every knob is an option field
    a = kktgen.make_kkt(50, 1)
    b = kktgen.make_kkt(80, 2)
    pa = [(a.n, a.rowptr, a.colind, None), (b.n, b.rowptr, b.colind, None)]
    k1 = autotune.batch_key(pa, [0, 1, 0])
    assert k1 == autotune.batch_key(pa, np.array([0, 1, 0]))
    assert k1 != autotune.batch_key(pa, [0, 1, 1]) and k1 != autotune.batch_key(pa[::-1], [0, 1, 0])
    assert k1 != autotune.pattern_key(a.n, a.rowptr, a.colind)
