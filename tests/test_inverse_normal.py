"""The path kernels' inverse normals Z = Phi^-1((J + 1/2) 2^-32) (Section 3.1, the
exact increment of the coupled pair) against 60-digit quantiles: extreme and
central words, the central/tail switch, and random words.  FP64 within 1e-14
relative (absolute 1e-14 near u = 1/2), FP32 within 2e-7 relative / 4e-7 absolute.
The host build runs here; the device build (four-wide form, ragged tail scalar) on
the GPU, through the C ABI."""
import mpmath
import numpy as np
import pytest

import paper_2502_07123_amd as M
from oracle import normal

EXTREMES = [0, 1, 2, 3, 2**31 - 2, 2**31 - 1, 2**31, 2**31 + 1, 2**32 - 3, 2**32 - 2, 2**32 - 1]


def _words(n_random, seed=11):
    rng = np.random.default_rng(seed)
    # near the central/tail switch of both fits: 4U(1-U) around e^-5 and e^-6.25
    sw = []
    for w in (5.0, 6.25):
        us = (1 - np.sqrt(1 - np.exp(-w))) / 2
        c = int(us * 2**32)
        sw += list(range(c - 40, c + 40)) + [2**32 - 1 - j for j in range(c - 40, c + 40)]
    J = np.concatenate([np.array(EXTREMES + sw, dtype=np.uint64),
                        rng.integers(0, 2**32, size=n_random, dtype=np.uint64)])
    return J.astype(np.uint32)


def _mp_ref(J):
    out = np.empty(len(J))
    with mpmath.workdps(60):
        for i, j in enumerate(J):
            u = (mpmath.mpf(int(j)) + mpmath.mpf(0.5)) / mpmath.mpf(2) ** 32
            out[i] = float(mpmath.sqrt(2) * mpmath.erfinv(2 * u - 1))
    return out


def check_f64(Z, ref):
    err = np.abs(Z - ref)
    assert np.all(err <= 1e-14 * np.maximum(np.abs(ref), 1.0)), float((err / np.maximum(np.abs(ref), 1)).max())


def check_f32(Z, ref):
    err = np.abs(Z.astype(np.float64) - ref)
    assert np.all((err <= 2e-7 * np.abs(ref)) | (err <= 4e-7)), float(err.max())


def test_host_build_against_mpmath():
    J = _words(2000)
    ref = _mp_ref(J)
    check_f64(M.inverse_normal_host(J, "fp64"), ref)
    check_f32(M.inverse_normal_host(J, "fp32"), ref)


def test_host_build_against_oracle_many():
    # 1e5 random words against the oracle's ndtri (itself within 2e-15 of mpmath)
    J = _words(100_000, seed=12)
    ref = normal.exact_normal(J.astype(np.uint64))
    Z = M.inverse_normal_host(J, "fp64")
    assert np.all(np.abs(Z - ref) <= 1.2e-14 * np.maximum(np.abs(ref), 1.0))
    Zf = M.inverse_normal_host(J, "fp32").astype(np.float64)
    err = np.abs(Zf - ref)
    assert np.all((err <= 2e-7 * np.abs(ref)) | (err <= 4e-7))


def test_pin_catches_a_perturbed_value():
    # the tolerance is tight enough to see a 1e-13 relative slip
    J = np.array(EXTREMES, dtype=np.uint32)
    ref = _mp_ref(J)
    with pytest.raises(AssertionError):
        check_f64(M.inverse_normal_host(J, "fp64") * (1 + 1e-13), ref)


@pytest.mark.gpu
@pytest.mark.parametrize("n_random", [2000, 2001])          # a multiple of four and a ragged tail
def test_device_build_against_mpmath(n_random):
    J = _words(n_random)
    ref = _mp_ref(J)
    with M.Context(0, workspace_bytes=16 << 20) as ctx:
        check_f64(ctx.inverse_normal(J, "fp64"), ref)
        check_f32(ctx.inverse_normal(J, "fp32"), ref)


@pytest.mark.gpu
def test_device_build_against_oracle_many():
    J = _words(100_000, seed=12)
    ref = normal.exact_normal(J.astype(np.uint64))
    with M.Context(0, workspace_bytes=16 << 20) as ctx:
        Z = ctx.inverse_normal(J, "fp64")
        Zf = ctx.inverse_normal(J, "fp32").astype(np.float64)
    assert np.all(np.abs(Z - ref) <= 1.2e-14 * np.maximum(np.abs(ref), 1.0))
    err = np.abs(Zf - ref)
    assert np.all((err <= 2e-7 * np.abs(ref)) | (err <= 4e-7))
