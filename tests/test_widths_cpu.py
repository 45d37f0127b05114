"""The library's bit-width optimiser (mlmc_optimise_widths, host code) against the
oracle's Section 6 optimiser on the same error model: real widths, multiplier,
objectives, the greedy integer widths and the kernel formats derived from them,
which the library's own validation accepts."""
import numpy as np
import pytest

import paper_2502_07123_amd as M
from oracle import errmodel as em
from oracle.paths import Problem

GBM = dict(S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0)
SEED = 1234


def model_dict(m, scheme, level, q):
    return {"level": level, "scheme": 1 if scheme == "milstein" else 0, "table_bits": q,
            "n_paths": m.n_paths, "used": [int(u) for u in m.used], "e": [int(x) for x in m.e],
            "S": [float(x) for x in m.S], "R": [float(x) for x in m.R], "V_level": m.V_level,
            "mse": m.mse}


@pytest.mark.parametrize("scheme,level,rng", [("milstein", 0, False), ("milstein", 4, False),
                                              ("euler", 3, True), ("milstein", 7, True),
                                              ("euler", 0, False)])
def test_library_widths_equal_oracle(scheme, level, rng):
    q = 8
    m = em.sensitivities(Problem(scheme, **GBM), level, 4000, q, SEED)
    plan = M.optimise_widths(model_dict(m, scheme, level, q), 1e4, rng)
    opt = em.optimise(m, scheme, level, 1e4, rng)
    assert np.allclose(plan["d_real"], opt.d_real, rtol=0, atol=1e-9)
    assert plan["d_int"] == [int(x) for x in opt.d_int]
    assert abs(plan["lambda"] - opt.lam) <= 1e-9 * opt.lam
    assert abs(plan["objective"] - opt.objective) <= 1e-12 * opt.objective
    assert plan["best_uniform"] == opt.best_uniform
    assert abs(plan["objective_uniform"] - opt.objective_uniform) <= 1e-12 * opt.objective_uniform
    assert abs(plan["v_indep"] - em.v_indep(m, opt.d_int, rng)) <= 1e-12 * plan["v_indep"]
    F = em.kernel_formats(m, opt.d_int, scheme)
    fmt = {}
    for i, v in enumerate(em.VARS):
        if m.used[i]:
            assert (plan["word_bits"][i], plan["frac_bits"][i]) == F[v], v
            fmt[v] = F[v]
        else:
            assert plan["word_bits"][i] == 0 and plan["frac_bits"][i] == 0
    prob = M.make_problem(scheme, ("euro",), **GBM)
    for est in (M.EST_APPROX, M.EST_CORR):
        M.validate(prob, level, 1000, 0, M.make_precision("fixed", q, False, fmt), est)


def test_optimiser_rejects_bad_models():
    m = em.sensitivities(Problem("euler", **GBM), 2, 1000, 8, SEED)
    d = model_dict(m, "euler", 2, 8)
    with pytest.raises(M.MlmcError):
        M.optimise_widths({**d, "level": 21})
    with pytest.raises(M.MlmcError):
        M.optimise_widths(d, c_rng=0.0)
    bad = dict(d)
    bad["S"] = [float("nan")] + d["S"][1:]
    with pytest.raises(M.MlmcError):
        M.optimise_widths(bad)
