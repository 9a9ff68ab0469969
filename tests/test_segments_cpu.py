"""The segment runner (checkpoint, resume, shards, slow-segment flag) on the
CPU, with fake executors in place of ph_perm_partial: the exact oracle's
partial sums of an integer matrix, or arbitrary doubles where only the exact
round trip through the checkpoint matters."""
import json
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_1606_05836_amd.segments import SegmentedPermanent, combine_shards

N = 9  # 2^8 Gray terms


def int_matrix(seed=3):
    rng = np.random.default_rng(seed)
    return (rng.integers(-3, 4, (N, N)) + 1j * rng.integers(-3, 4, (N, N))).astype(np.complex128)


class OracleExecutor:
    """Exact partial sums from the oracle; optionally fails at one call."""

    def __init__(self, a, fail_at=None):
        self.g, self.d = O.to_gaussian_integers(a)
        assert self.d == 1
        self.calls = []
        self.fail_at = fail_at

    def __call__(self, kb, ke):
        if self.fail_at is not None and len(self.calls) == self.fail_at:
            raise RuntimeError("device lost")
        self.calls.append((kb, ke))
        re, im = O.glynn_gray_raw(self.g, kb, ke)
        assert abs(re) < 2 ** 53 and abs(im) < 2 ** 53
        return [float(re), 0.0, float(im), 0.0]


def exact_combiner(partials):
    re = sum(Fraction(p[0]) + Fraction(p[1]) for p in partials)
    im = sum(Fraction(p[2]) + Fraction(p[3]) for p in partials)
    s = Fraction(1, 1 << (N - 1))
    return complex(float(re * s), float(im * s))


def runner(a, ex, path=None, seg=4, shard=(0, 1), fp=None, **kw):
    return SegmentedPermanent(N, "glynn", "dd", 1, seg, fp if fp is not None else a.tobytes(), ex, exact_combiner,
                              checkpoint=path, shard=shard, device="cpu-fake", **kw)


def test_uninterrupted_total_is_the_permanent():
    a = int_matrix()
    r = runner(a, OracleExecutor(a))
    assert r.nseg_total == 16
    assert r.run()
    assert r.total() == O.to_complex(O.perm_exact(a))


def test_failure_between_segments_resumes_to_the_same_bits(tmp_path):
    a = int_matrix()
    ref = runner(a, OracleExecutor(a))
    ref.run()
    path = str(tmp_path / "ck.json")
    ex = OracleExecutor(a, fail_at=5)
    r = runner(a, ex, path)
    with pytest.raises(RuntimeError, match="device lost"):
        r.run()
    st = json.load(open(path))
    assert st["next_segment"] == 5 and len(st["partials"]) == 5
    # a new process: reads the checkpoint and evaluates only the missing segments
    ex2 = OracleExecutor(a)
    r2 = runner(a, ex2, path)
    assert r2.next_segment == 5
    assert r2.run()
    assert ex2.calls[0] == (5 * 16, 6 * 16) and len(ex2.calls) == 11
    assert r2.partials == ref.partials
    assert r2.total() == ref.total()


def test_bounded_runs_and_exact_round_trip(tmp_path):
    # arbitrary doubles (subnormal, negative zero, odd mantissas) survive the checkpoint bit for bit
    rng = np.random.default_rng(9)
    vals = {i * 16: [float(x) for x in rng.standard_normal(4) * 10.0 ** rng.integers(-300, 300, 4)]
            for i in range(16)}
    vals[3 * 16][1] = 5e-324
    vals[3 * 16][2] = -0.0

    def ex(kb, ke):
        return vals[kb]

    a = int_matrix()
    path = str(tmp_path / "ck.json")
    r = runner(a, ex, path)
    assert not r.run(max_segments=3)
    for _ in range(10):
        runner(a, ex, path).run(max_segments=2)
    r = runner(a, ex, path)
    assert r.run()
    got = [p for p in r.partials]
    want = [vals[i * 16] for i in range(16)]
    assert [[x.hex() for x in p] for p in got] == [[x.hex() for x in p] for p in want]


def test_checkpoint_of_another_run_is_refused(tmp_path):
    a = int_matrix()
    path = str(tmp_path / "ck.json")
    runner(a, OracleExecutor(a), path).run(max_segments=2)
    b = int_matrix(seed=4)
    with pytest.raises(ValueError, match="another run"):
        runner(b, OracleExecutor(b), path)
    with pytest.raises(ValueError, match="another run"):
        runner(a, OracleExecutor(a), path, seg=5)
    with pytest.raises(ValueError, match="another run"):
        runner(a, OracleExecutor(a), path, shard=(1, 2))
    # a damaged file is refused too
    st = json.load(open(path))
    st["next_segment"] = 7
    json.dump(st, open(path, "w"))
    with pytest.raises(ValueError, match="next_segment"):
        runner(a, OracleExecutor(a), path)


def test_shards_join_to_the_single_run(tmp_path):
    a = int_matrix()
    ref = runner(a, OracleExecutor(a))
    ref.run()
    G = 3  # 16 segments over 3 shards: 5, 5, 6
    shards = []
    for g in range(G):
        s = runner(a, OracleExecutor(a), str(tmp_path / f"s{g}.json"), shard=(g, G))
        shards.append(s)
    sizes = [s.seg_end - s.seg_begin for s in shards]
    assert sizes == [5, 5, 6] and shards[0].seg_begin == 0 and shards[-1].seg_end == 16
    for s in reversed(shards):  # any order of completion
        s.run()
    with pytest.raises(RuntimeError):
        shards[0].total()
    assert combine_shards(shards) == ref.total()
    with pytest.raises(ValueError):
        combine_shards(shards[:2])


def test_slow_segment_is_flagged():
    a = int_matrix()
    t = [0.0]
    durations = iter([1.0, 1.1, 0.9, 1.0, 5.0, 1.0, 1.2] + [1.0] * 9)

    def clock():
        return t[0]

    ex_inner = OracleExecutor(a)

    def ex(kb, ke):
        t[0] += next(durations)
        return ex_inner(kb, ke)

    r = runner(a, ex, clock=clock)
    r.run()
    assert r.slow == [4]
    assert r.seconds[4] == 5.0


def test_bad_segment_lengths():
    a = int_matrix()
    with pytest.raises(ValueError):
        runner(a, OracleExecutor(a), seg=0)  # shorter than a chunk (2^1)
    with pytest.raises(ValueError):
        runner(a, OracleExecutor(a), seg=9)  # longer than the 2^8 terms
    with pytest.raises(ValueError):
        runner(a, OracleExecutor(a), shard=(2, 2))
    r = runner(a, OracleExecutor(a), seg=8)
    assert r.nseg_total == 1 and r.run()
    assert r.total() == O.to_complex(O.perm_exact(a))
