"""The autotuner changes launch shapes only: tuned and untuned runs agree bitwise, and the
cache file reproduces the choices without timing again."""
import sys

import numpy as np
import pytest

from paper_2210_15668_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2210_15668_amd import ferrox
    ferrox.lib()
    return ferrox


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
def test_tuned_stack_is_bitwise_unchanged_and_cached(fx, tmp_path, prec):
    spec = W.shrink_lateral(W.mfism_large(prec), 64, 64)
    P0 = W.random_P(spec, 11)
    ref = fx.Stack(spec, P0)
    ref.run_steps(5, W.DT)
    cache = str(tmp_path / "tune.txt")
    s = fx.Stack(spec, P0)
    info = s.autotune(cache)
    say(f"  levels {info.levels} timed {info.configs_timed} default {info.default_us:.1f} us "
        f"tuned {info.tuned_us:.1f} us; " + ", ".join(str(s.tune_config(l)) for l in range(info.levels)))
    assert info.levels >= 1 and info.from_cache == 0 and info.configs_timed >= info.levels
    assert info.cache_written == 1 and info.tuned_us <= info.default_us
    s.run_steps(5, W.DT)
    assert np.array_equal(s.get(fx.FIELD_P), ref.get(fx.FIELD_P))
    assert np.array_equal(s.get(fx.FIELD_PHI), ref.get(fx.FIELD_PHI))
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == info.levels and all(" -> " in ln for ln in lines)
    t = fx.Stack(spec, P0)
    again = t.autotune(cache)
    assert again.from_cache == again.levels == info.levels and again.configs_timed == 0
    assert [t.tune_config(l) for l in range(info.levels)] == [s.tune_config(l) for l in range(info.levels)]
    forced = t.autotune(cache, force=True)
    assert forced.from_cache == 0 and forced.configs_timed >= forced.levels
    t.run_steps(5, W.DT)
    assert np.array_equal(t.get(fx.FIELD_PHI), ref.get(fx.FIELD_PHI))


def test_tuned_batch_is_bitwise_unchanged(fx, tmp_path):
    inst = W.batch_instances(12, seed0=300)
    specs = [sp for sp, _ in inst]
    Ps = [P for _, P in inst]
    a = fx.Batch(specs, Ps)
    a.run(4, W.DT)
    b = fx.Batch(specs, Ps)
    info = b.autotune(str(tmp_path / "tune.txt"))
    assert info.levels >= 1 and info.configs_timed >= info.levels
    b.run(4, W.DT)
    for q in range(len(specs)):
        assert np.array_equal(a.get(q, fx.FIELD_PHI), b.get(q, fx.FIELD_PHI)), q
        assert np.array_equal(a.get(q, fx.FIELD_P), b.get(q, fx.FIELD_P)), q
