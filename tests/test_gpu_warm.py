"""What the trained warm-start network gains over cold-start GaBP, on held-out
problems of the 1024 x 1024 warm-start workload (seeds never used in
training), and the cold fallback."""
import os

import pytest

from paper_2404_12968_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2404_12968_amd", "weights", "warm1024.npz")


@pytest.fixture(scope="module")
def W():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_12968_amd import warm
    return warm


@pytest.mark.parametrize("instance", [200000, 200001])
def test_trained_warm_start_cuts_iterations_and_time(W, instance):
    from paper_2404_12968_amd import gabp as G
    net = W.WarmNet.load(WEIGHTS)
    p = I.warm1024(instance=instance)
    cold = W.cold_solve(p)
    warm = W.warm_solve(net, p)
    print(instance, p.kappa, cold, warm)
    assert cold["status"] == G.GABP_OK and warm["status"] == G.GABP_OK
    assert warm["rel"] <= 1e-6
    assert warm["start"] == "warm"
    assert warm["iterations"] <= 0.7 * cold["iterations"]
    assert warm["seconds"] < cold["seconds"]


def test_untrained_network_is_caught_by_the_fallback(W):
    """A random network still ends at the right answer: the solver's residual
    test decides convergence, and the worse start is dropped at the probe."""
    from paper_2404_12968_amd import gabp as G
    net = W.WarmNet(seed=123)
    p = I.warm1024(instance=200002, n=256)
    res = W.warm_solve(net, p)
    assert res["status"] == G.GABP_OK and res["rel"] <= 1e-6
    assert res["start"] in ("warm", "cold")
    assert (res["start"] == "warm") == (res["probe_residual_warm"] <= res["probe_residual_cold"])
