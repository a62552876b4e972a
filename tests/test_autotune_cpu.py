"""Host logic of the autotuner (paper_2307_08006_amd/autotune.py), on the CPU:
the device timings are replaced by a fixed cost model, so that what is tested
is the search (widths at the default buffer, then buffers at the best width)
and the batch check that keeps a class's choice only for a gain above the
margin."""
import numpy as np
import pytest

from paper_2307_08006_amd import autotune, synth


def _small_uneven():
    # four walkers of uneven size (13k-41k atoms: three size classes)
    spec, lam = synth.uneven(n_walkers=4, n_min=5000, n_max=60000, seed=synth.BASE_SEED + 3)
    return spec, lam


def test_batch_check_keeps_only_clear_gains(monkeypatch, tmp_path):
    spec, lam = _small_uneven()
    n = np.diff(spec.atom_offset)
    classes = [autotune.size_class(int(x)) for x in n]
    # cost model: replicas prefer width 1.12 and buffer 0.5 in every class;
    # on the batch only the largest class's choice gains (2 %), the others
    # lose a little
    largest = max(classes)

    def fake_time_knobs(sp, lm, widths, buffers, reps=4, warm_blocks=6):
        widths = np.asarray(widths, float)
        buffers = np.asarray(buffers, float)
        if sp is not spec:      # a class's replicas (the batch itself is relaxed to itself here)
            return 1.0 - 0.01 * float(np.all(widths == 1.12)) - 0.02 * float(np.all(buffers == 0.5))
        t = 1.0
        for k, cls in enumerate(classes):
            tuned = widths[k] == 1.12 and buffers[k] == 0.5
            if tuned:
                t *= 0.98 if cls == largest else 1.002
        return t

    monkeypatch.setattr(autotune, "time_knobs", fake_time_knobs)
    monkeypatch.setattr(autotune, "relax", lambda sp, lm, steps=300: sp)
    monkeypatch.setattr(autotune, "arch", lambda: "gfx950")
    cache = tmp_path / "cache.json"
    widths, buffers = autotune.tune(spec, lam, cache_path=str(cache), force=True)
    c = autotune.load_cache(str(cache))
    for k, cls in enumerate(classes):
        ent = c[autotune._key("gfx950", cls, spec.precision)]
        # the replicas' choice is recorded either way
        assert ent["replica_choice"] == {"column_width": 1.12, "prune_buffer": 0.5}
        if cls == largest:
            assert ent["accepted"] and widths[k] == 1.12 and buffers[k] == 0.5
        else:
            assert not ent["accepted"] and widths[k] == 1.0 and buffers[k] == 0.0
            assert (ent["column_width"], ent["prune_buffer"]) == (1.0, 0.0)
    # the cached knobs are what the tuner returned
    w2, b2 = autotune.cached_knobs(spec, str(cache))
    np.testing.assert_array_equal(w2, widths)
    np.testing.assert_array_equal(b2, buffers)


def test_batch_check_margin(monkeypatch, tmp_path):
    """A gain below the margin (1 %) is not kept."""
    spec, lam = _small_uneven()

    def fake_time_knobs(sp, lm, widths, buffers, reps=4, warm_blocks=6):
        widths = np.asarray(widths, float)
        if sp is not spec:
            return 1.0 - 0.01 * float(np.all(widths == 0.9))
        return 1.0 - 0.005 * float(np.sum(widths == 0.9))    # 0.5 % per class

    monkeypatch.setattr(autotune, "time_knobs", fake_time_knobs)
    monkeypatch.setattr(autotune, "relax", lambda sp, lm, steps=300: sp)
    monkeypatch.setattr(autotune, "arch", lambda: "gfx950")
    widths, buffers = autotune.tune(spec, lam, cache_path=str(tmp_path / "c.json"), force=True)
    assert np.all(widths == 1.0) and np.all(buffers == 0.0)
