"""The learned corrector end to end at a small size (fine 128^3 -> coarse 32^3,
16 training seeds, 2 held-out seeds): teacher-forced pairs from the method's
own fine runs, training on the GPU by the library's kernels, and what the
trained network gains over the plain coarse run."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def trained():
    from paper_2102_09512_amd import corrector as Cr
    from paper_2102_09512_amd import lbm

    w = Cr.Workload(n_fine=128, n_coarse=32, every=4, windows=16)
    log = lambda s: print(s, flush=True)
    pairs = Cr.generate_pairs(w, *Cr.training_seeds(16), log=log)
    assert pairs.shape[0] == 16 * w.windows
    res = Cr.train(w, pairs, epochs=100, lr=1e-3, batch=4, log=log)
    del pairs
    yield w, res
    lbm.lbm_nn_destroy(res.net)


def test_training_lowers_the_loss_and_generalises(trained):
    from paper_2102_09512_amd import corrector as Cr

    w, res = trained
    assert res.history[-1] < 0.85 * res.history[0]
    vp = Cr.generate_pairs(w, *Cr.evaluation_seeds(2), log=print)
    zero = Cr.no_correction_loss(w, vp, res.scaling[2])
    val = Cr.validation_loss(res.net, vp)
    print(f"  held-out loss {val:.4f}, without correction {zero:.4f}", flush=True)
    assert val < 0.85 * zero


def test_corrected_run_beats_the_plain_coarse_run(trained):
    """On held-out seeds the corrected 32^3 run's kinetic-energy spectrum is
    closer to the filtered 128^3 run than the plain 32^3 run's, and closer
    than the best plain run (32^3, 40^3 or 48^3) that takes no more wall time
    than the corrected run (the plain run at equal wall time)."""
    from paper_2102_09512_amd import corrector as Cr

    w, res = trained
    rows = Cr.evaluate(w, res.net, *Cr.evaluation_seeds(2), grids=[32, 40, 48], log=print)
    for r in rows:
        assert r["fine_ok"] and r["learned"]["ok"] and all(p["ok"] for p in r["plain"])
    s = Cr.summarize(rows)
    print("  summary", s, flush=True)
    assert s["learned"] < s["plain_coarse"]
    assert s["learned"] < s["plain_equal_time"]
    assert s["wins_equal_time"] == s["seeds"]
