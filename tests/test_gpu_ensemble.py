"""Batched ensemble on the GPU, through the C-ABI: every case bitwise equal
to the same case run alone, the in-kernel elliptic initial condition equal to
the recipe's profile, one case against the CPU oracle, per-case failure
flags, and the full 512-case workload of mixed sizes."""
import sys

import numpy as np
import pytest

from paper_2011_00814_amd import workloads as W
from tests.parity_util import compare_states

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpe():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_00814_amd import gpe as G

    G.lib()
    return G


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mixed_cases(precision):
    # sizes spanning one / several X tiles, ragged X (70, 96) and ragged Z
    # chunks (sizes not multiples of 32); parameters from the recipe
    cases = W.ensemble_cases(6, seed=11, precision=precision, sizes=(64, 70, 96, 128))
    return cases


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_ensemble_bitwise_equals_single_runs(gpe, precision):
    cases = _mixed_cases(precision)
    _say(f"[ensemble] {len(cases)} cases {precision} sizes {[c['n'][0] for c in cases]} vs single runs")
    ens = gpe.Ensemble(cases)
    ens.run(1)   # eager
    ens.run(15)  # graph replay
    ens.synchronize()
    for i, prob in enumerate(cases):
        a = ens.case(i).state()
        assert ens.case(i).diagnostics()["step"] == 16
        s = gpe.Solver(prob, None)
        s.run(16)
        s.synchronize()
        b = s.state()
        s.close()
        for k in a:
            if a[k] is not None:
                assert np.array_equal(a[k], b[k]), (i, k)
    ens.close()


def test_autotuned_tiles_keep_results_bitwise(gpe):
    cases = _mixed_cases("fp32")
    ens = gpe.Ensemble(cases)
    rows = ens.autotune(trial_steps=2)
    ens.run(5)
    ens.synchronize()
    _say(f"[ensemble] autotuned rows {list(rows)}")
    assert all(r in (1, 2, 4, 8, 16, 32, 64, 128) or r == c["n"][1] for r, c in zip(rows, cases))
    for i, prob in enumerate(cases):
        a = ens.case(i)
        nsteps = a.diagnostics()["step"]
        s = gpe.Solver(prob, None)
        s.run(nsteps)
        s.synchronize()
        b = s.state()
        s.close()
        sa = a.state()
        for k in sa:
            if sa[k] is not None:
                assert np.array_equal(sa[k], b[k]), (i, k, nsteps)
    ens.close()


def test_ellipse_init_matches_recipe_profile(gpe):
    cases = W.ensemble_cases(3, seed=5, precision="fp64")
    ens = gpe.Ensemble(cases)
    for i, prob in enumerate(cases):
        ref = W.ensemble_state(prob)["phi"]
        assert np.max(np.abs(ens.case(i).get("phi") - ref)) < 1e-14
    ens.close()


def test_ensemble_case_against_oracle(gpe, oracle):
    cases = W.ensemble_cases(3, seed=7, precision="fp64", sizes=(64, 70))
    ens = gpe.Ensemble(cases)
    ens.run(30)
    ens.synchronize()
    for i, prob in enumerate(cases):
        _say(f"[ensemble] oracle parity case {i} n={prob['n']} dt={prob['dt']:.4g}")
        ref = oracle.run(prob, W.ensemble_state(prob), 30)
        errs, raw = compare_states(prob, ens.case(i).state(), ref)
        assert all(v <= 1e-11 for v in errs.values()), (i, errs, raw)
    ens.close()


def test_per_case_failure_flag(gpe):
    cases = W.ensemble_cases(5, seed=2, sizes=(64, 96))
    bad = dict(cases[2])
    bad["dt"] = 40.0 * bad["dt"]  # far beyond the stability estimate
    bad["allow_unstable"] = 1
    cases[2] = bad
    ens = gpe.Ensemble(cases)
    assert list(ens.finite()) == [1] * 5
    ens.run(400)
    flags = ens.finite()
    _say(f"[ensemble] flags after 400 steps: {list(flags)}")
    assert flags[2] == 0
    assert list(np.delete(flags, 2)) == [1] * 4
    with pytest.raises(gpe.GpeError):
        ens.case(2).diagnostics()
    assert ens.case(0).diagnostics()["finite"] == 1
    ens.close()


def test_full_ensemble_workload_runs(gpe):
    """512 cases of sizes 64^2 .. 256^2 (13.8 M cells): all finite after 50
    steps; phase mass conserved per case (sampled)."""
    cases = W.ensemble_cases(512, seed=0)
    ens = gpe.Ensemble(cases)
    d0 = {i: ens.case(i).diagnostics() for i in range(0, 512, 37)}
    ens.run(50)
    ens.synchronize()
    flags = ens.finite()
    _say(f"[ensemble] 512 cases, finite after 50 steps: {int(flags.sum())}")
    assert flags.sum() == 512
    for i, d in d0.items():
        d1 = ens.case(i).diagnostics()
        assert d1["step"] == 50
        assert abs(d1["mass"] - d["mass"]) / d["mass_abs0"] < 1e-6, i
    ens.close()


def test_full_ensemble_configured_length(gpe):
    """The 512-case workload over its configured 5000 steps: every per-case
    finite flag agrees with that case's own diagnostics (a sample plus every
    flagged case), all cases stay finite, and phase mass is conserved in the
    sampled cases."""
    cases = W.ensemble_cases(512, seed=0)
    ens = gpe.Ensemble(cases)
    sample = list(range(0, 512, 23))
    d0 = {i: ens.case(i).diagnostics() for i in sample}
    ens.run(5000)
    ens.synchronize()
    flags = ens.finite()
    bad = [i for i in range(512) if not flags[i]]
    _say(f"[ensemble] 512 cases, finite after 5000 steps: {int(flags.sum())}; flagged: {bad[:20]}")
    drift = 0.0
    for i in sorted(set(sample) | set(bad)):
        d1 = ens.case(i).diagnostics()
        assert d1["step"] == 5000
        assert bool(d1["finite"]) == bool(flags[i]), i
        if i in d0 and flags[i]:
            drift = max(drift, abs(d1["mass"] - d0[i]["mass"]) / d0[i]["mass_abs0"])
    _say(f"[ensemble] max relative mass drift over the sample: {drift:.2e}")
    assert not bad
    assert drift < 1e-5
    ens.close()
