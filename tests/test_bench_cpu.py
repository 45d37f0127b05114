"""Host logic of bench.py: which kernel the roofline is reported for."""
import bench


def test_dominant_kernel_by_work_not_event_time():
    # the approximate kernel holds the work; the correction kernel's events span longer
    # (it waits behind the other stream), which must not make it the dominant one
    Na = [100_000 >> l for l in range(bench.LEVELS)]
    Nc = [1_000 >> l for l in range(bench.LEVELS)]
    stats = [{"estimator": 2, "fields": 1, "scheme": 1, "ms": 3.0},
             {"estimator": 1, "fields": 4, "scheme": 1, "ms": 1.0}]
    dom, ops = bench.dominant_kernel(stats, Na, Nc)
    assert dom["estimator"] == 1
    want = sum(Na[l] * (1 << l) * bench.alg_ops_per_step(1, 4, 1, l, 1) for l in range(bench.LEVELS))
    assert ops == want


def test_dominant_kernel_follows_the_work():
    # with the sample counts reversed the correction kernel holds the work
    Na = [10] * bench.LEVELS
    Nc = [100_000] * bench.LEVELS
    stats = [{"estimator": 1, "fields": 4, "scheme": 1, "ms": 5.0},
             {"estimator": 2, "fields": 1, "scheme": 1, "ms": 1.0}]
    dom, _ = bench.dominant_kernel(stats, Na, Nc)
    assert dom["estimator"] == 2


def test_alg_ops_follow_the_method_counts():
    # approximate FP32 Milstein, four 8-bit indices per word: a quarter of a Philox
    # word, the index, the fine step with the Milstein terms; level 0 adds the
    # per-path payoff and sums, levels >= 1 the coarse share
    assert bench.alg_ops_per_step(1, 4, 1, 0, 1) == 12.5 / 4 + 1.5 + 5 + 4
    assert bench.alg_ops_per_step(1, 4, 1, 3, 1) == 12.5 / 4 + 1.5 + 5 + 3 + 4 / 8
    assert bench.alg_ops_per_step(1, 1, 0, 2, 1) == 12.5 + 1.5 + 2 + 1.5 + 4 / 4
    # correction: one word, the FP64 inverse normal, both sides' steps, two payoffs
    assert bench.alg_ops_per_step(2, 1, 1, 0, 1) == 12.5 + 1.5 + 60 + 5 + 5 + 8
    # plain FP32 / FP64: the inverse normal in the plain side's precision
    assert bench.alg_ops_per_step(0, 1, 0, 0, 1) == 12.5 + 25 + 2 + 4
    assert bench.alg_ops_per_step(0, 1, 0, 0, 0) == 12.5 + 60 + 2 + 4
    # fixed point: the integer step
    assert bench.alg_ops_per_step(1, 1, 0, 1, 3) == 12.5 + 1.5 + 12 + 6.5 + 2
