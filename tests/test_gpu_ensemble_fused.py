"""The batched ensemble's persistent fused step (itokmc_ens_tuning.fused_per_cu: push,
counting sort, scatter, KMC, coupling and end of step in one launch, phases separated by
device-wide barriers) against the same ensemble run as its sequence of kernels and
against plain single contexts: every realization's particles, counts and tallies
bit-identical, in FP32 and FP64, with graph replay and without, with realizations
admitted and released while others run; the autotuner's choice of form keeps results;
a barrier that gives up is reported, not hung on."""
import os
import subprocess
import sys
import textwrap

import pytest

from test_gpu_ensemble import (TALLIES, _assert_same, _drain, _ens_state, _new_ensemble,
                               _plain_state, _run_plain, _small_realizations)

pytestmark = pytest.mark.gpu

FUSED = (1, 2, 4)


@pytest.fixture(scope="module")
def itk():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2307_01797_amd import itokmc
    itokmc.lib()
    return itokmc


def _run(itk, cfgs, fused, precision="fp32", graph=1):
    ens = _new_ensemble(itk, precision=precision)
    ens.set_tuning(fused_per_cu=fused, use_graph=graph)
    slots = [ens.admit(c, tag=i) for i, c in enumerate(cfgs)]
    done = _drain(ens)
    return ens, slots, done


def _same_runs(a, b, cfgs):
    ea, sa, da = a
    eb, sb, db = b
    for cfg, x, y in zip(cfgs, sa, sb):
        assert da[x] == db[y]
        _assert_same(_ens_state(ea, x, cfg["grid"]), _ens_state(eb, y, cfg["grid"]))
        ra, rb = ea.result(x), eb.result(y)
        for k in TALLIES:
            assert ra[k] == rb[k], (k, ra[k], rb[k])


@pytest.mark.parametrize("fused", FUSED)
def test_fused_matches_kernel_sequence_fp32(itk, fused):
    print(f"fused fp32 W={fused}", flush=True)
    cfgs = _small_realizations(6, steps=40, seed=5)
    ref = _run(itk, cfgs, 0)
    got = _run(itk, cfgs, fused)
    _same_runs(ref, got, cfgs)
    # and one realization against its plain single context
    ens, slots, _ = got
    _assert_same(_ens_state(ens, slots[2], cfgs[2]["grid"]), _plain_state(_run_plain(itk, cfgs[2])))


@pytest.mark.parametrize("fused", (1, 4))
def test_fused_matches_kernel_sequence_fp64(itk, fused):
    print(f"fused fp64 W={fused}", flush=True)
    cfgs = _small_realizations(4, steps=30, seed=9, precision="fp64")
    _same_runs(_run(itk, cfgs, 0, precision="fp64"), _run(itk, cfgs, fused, precision="fp64"), cfgs)


def test_fused_empty_pool_then_admission(itk):
    """Fused steps of an ensemble with no realizations (nothing to push, no scan tiles),
    then a realization admitted into it runs as its plain context does."""
    print("fused empty pool W=2", flush=True)
    ens = _new_ensemble(itk, slots=2, cells=1 << 20, particles=400_000)
    ens.set_tuning(fused_per_cu=2)
    ens.step(3)
    assert ens.poll() == []
    cfg = _small_realizations(1, steps=25, seed=41)[0]
    s = ens.admit(cfg)
    done = _drain(ens)
    assert done[s][2] == 25
    _assert_same(_ens_state(ens, s, cfg["grid"]), _plain_state(_run_plain(itk, cfg)))


def test_fused_without_graph(itk):
    print("fused eager W=2", flush=True)
    cfgs = _small_realizations(5, steps=30, seed=13)
    _same_runs(_run(itk, cfgs, 0), _run(itk, cfgs, 2, graph=0), cfgs)


def test_fused_with_churn(itk):
    """Realizations admitted and released while the fused step runs: a realization
    admitted mid-run equals its plain single context; a released one's blocks are
    reused by the next admission."""
    print("fused churn W=1", flush=True)
    cfgs = _small_realizations(8, steps=30, seed=21)
    ens = _new_ensemble(itk, slots=4)
    ens.set_tuning(fused_per_cu=1)
    first = [ens.admit(c) for c in cfgs[:3]]
    ens.step(7)
    ens.release(first[0])
    late = ens.admit(cfgs[3])
    ens.step(5)
    late2 = ens.admit(cfgs[4])
    _drain(ens)
    for cfg, s in ((cfgs[3], late), (cfgs[4], late2), (cfgs[1], first[1])):
        _assert_same(_ens_state(ens, s, cfg["grid"]), _plain_state(_run_plain(itk, cfg)))


def test_autotune_chooses_a_form_and_keeps_results(itk):
    print("fused autotune", flush=True)
    cfgs = _small_realizations(5, steps=50, seed=31)
    ens = _new_ensemble(itk)
    slots = [ens.admit(c) for c in cfgs]
    ens.step(2)
    best, ms = ens.autotune(rounds=2)
    assert ms > 0 and best["fused_per_cu"] in (0,) + FUSED
    assert ens.tuning() == best
    _drain(ens)
    for cfg, s in zip(cfgs, slots):
        _assert_same(_ens_state(ens, s, cfg["grid"]), _plain_state(_run_plain(itk, cfg)))


def test_fused_tuning_is_validated(itk):
    ens = _new_ensemble(itk, slots=2, cells=1 << 16, particles=100_000)
    for bad in (3, 5, -1, 8):
        with pytest.raises(itk.ItokmcError) as e:
            ens.set_tuning(fused_per_cu=bad)
        assert e.value.code == itk.EINVAL
    assert ens.tuning()["fused_per_cu"] == 0


def test_barrier_time_limit_is_reported():
    """With the wait limit forced to zero from the host, every workgroup gives up at
    its first barrier wait and returns (the kernel ends normally); the next poll reports
    the failure instead of returning events.  Runs in a child process so that the
    environment variable applies only there."""
    print("fused barrier time limit", flush=True)
    code = textwrap.dedent("""
        import sys
        sys.path.insert(0, sys.argv[1])
        sys.path.insert(0, sys.argv[1] + "/tests")
        from paper_2307_01797_amd import itokmc
        from test_gpu_ensemble import _small_realizations
        ens = itokmc.Ensemble(4, 1 << 20, 400_000)
        ens.set_tuning(fused_per_cu=1)
        for c in _small_realizations(2, steps=5, seed=3):
            ens.admit(c)
        ens.step(1)
        try:
            ens.poll()
        except itokmc.ItokmcError as err:
            assert err.code == itokmc.EHIP and "barrier" in str(err), str(err)
            print("reported", flush=True)
            sys.exit(0)
        sys.exit("no error reported")
    """)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, ITOKMC_FUSED_WAIT_US="0")
    r = subprocess.run([sys.executable, "-c", code, root], env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "reported" in r.stdout
