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
    want = sum(Na[l] * (1 << l) * bench.alg_ops_per_step(1, 4, 1, l) for l in range(bench.LEVELS))
    assert ops == want


def test_dominant_kernel_follows_the_work():
    # with the sample counts reversed the correction kernel holds the work
    Na = [10] * bench.LEVELS
    Nc = [100_000] * bench.LEVELS
    stats = [{"estimator": 1, "fields": 4, "scheme": 1, "ms": 5.0},
             {"estimator": 2, "fields": 1, "scheme": 1, "ms": 1.0}]
    dom, _ = bench.dominant_kernel(stats, Na, Nc)
    assert dom["estimator"] == 2
