"""What the trained warm start gains over the cold start, on held-out instances of
the batched size mix (seeds never used in training): fewer iterations to the
same tolerance at the same error against the planted low-rank part, every run
converged, no fallback."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1904_07497_amd import warmstart as ws  # noqa: E402

pytestmark = pytest.mark.gpu


def test_trained_warm_start_gains_over_cold_start():
    if not ws.MODEL_PATH.exists():
        pytest.skip("no trained warm-start model stored")
    P, hidden, sseed = ws.load_model()
    seeds = [ws.HELDOUT_BASE + 100_000 + i for i in range(64)]
    res = ws.evaluate(P, hidden, seeds, sketch_seed=sseed, chunk=64, log=lambda m: print(m, flush=True))
    s = ws.summary(res)
    print(s, flush=True)
    assert s["cold_converged"] == 64 and s["warm_converged"] == 64
    assert s["fallbacks"] == 0
    assert s["warm_iters_mean"] <= s["cold_iters_mean"] - 3.0
    assert s["err_ratio_max"] <= 1.05
    assert np.all(np.array(res["warm_iters"]) <= np.array(res["cold_iters"]))


def test_predicted_rho0_alone_gains_over_cold_start():
    """The warm start's predicted rho0 with the cold start's groups (K-means of X):
    fewer iterations on average at the same error, every run converged."""
    if not ws.MODEL_PATH.exists():
        pytest.skip("no trained warm-start model stored")
    P, hidden, sseed = ws.load_model()
    seeds = [ws.HELDOUT_BASE + 100_000 + i for i in range(64)]
    res = ws.evaluate(P, hidden, seeds, sketch_seed=sseed, chunk=64, groups="kmeans",
                      log=lambda m: print(m, flush=True))
    s = ws.summary(res)
    print(s, flush=True)
    assert s["cold_converged"] == 64 and s["warm_converged"] == 64
    assert s["fallbacks"] == 0
    assert s["warm_iters_mean"] <= s["cold_iters_mean"] - 3.0
    assert s["err_ratio_max"] <= 1.05


def test_sketch_seeded_warm_start_gains_over_cold_start():
    """The predicted rho0 with k-means++ seeds placed on the predicted centroid
    sketches and the K-means of X from those seed columns (init_embedding_refine 2):
    fewer iterations and fewer kernel steps per launch than the cold start, every run
    converged, the error against the planted part close to the cold start's."""
    if not ws.MODEL_PATH.exists():
        pytest.skip("no trained warm-start model stored")
    P, hidden, sseed = ws.load_model()
    seeds = [ws.HELDOUT_BASE + 100_000 + i for i in range(64)]
    res = ws.evaluate(P, hidden, seeds, sketch_seed=sseed, chunk=64, groups="seeds",
                      log=lambda m: print(m, flush=True))
    s = ws.summary(res)
    print(s, flush=True)
    assert s["cold_converged"] == 64 and s["warm_converged"] == 64
    assert s["fallbacks"] == 0
    assert s["warm_iters_mean"] <= s["cold_iters_mean"] - 3.0
    assert s["warm_steps"][0] < s["cold_steps"][0]
    assert s["err_ratio_median"] <= 1.02
    assert s["err_ratio_max"] <= 1.15
