"""What the trained warm start gains over the plain method (GPU, through the C ABI).

The MLP is trained on eight seeded graphs of the warm-start family (n = 10k, d = 512, k = 30,
shared mixture centres), then a larger unseen graph of the family (n = 30k) is clustered cold
and warm-started.  The gain asserted: the warm block's labels start at a lower multi-hop
conductance than the greedy start, the warm run reaches the cold run's final conductance
(within 1e-4 relative) in fewer iterations, and its labels recover the planted clusters at least
as well.  The warm block is used by the loop's own rule (its conductance is no larger).
"""
import numpy as np
import pytest

from paper_2408_05459_amd import synth, warmstart
from tests.helpers import ari

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_trained_warm_start_beats_cold_start(lib):
    exs = warmstart.make_examples(lib, 10000, list(range(5101, 5109)))
    ws, tl = warmstart.train(lib, exs, 512, 30, epochs=20, lr=1e-3, seed=0)
    assert tl.epoch_loss[-1] < 0.5 * tl.epoch_loss[0]
    net, prm = synth.make_warm_graph(30000, 5000)
    s, keep = lib.network(net)
    X = keep[-1]
    lc, ic, _ = warmstart.run(lib, s, X, net.k, prm)
    lw, iw, _ = warmstart.run(lib, s, X, net.k, prm, ws=ws)
    target = ic["best_phi"] * (1 + 1e-4)
    t_cold = warmstart.time_to_reach(ic, target)
    t_warm = warmstart.time_to_reach(iw, target)
    a_cold = ari(lc.cpu().numpy(), net.labels)
    a_warm = ari(lw.cpu().numpy(), net.labels)
    print(f"cold: phi0 {ic['phi_init_cold']:.5f} best {ic['best_phi']:.5f} at t={ic['best_t']} reach {t_cold} "
          f"ARI {a_cold:.4f}; warm: phi0 {iw['phi_init_warm']:.5f} best {iw['best_phi']:.5f} reach {t_warm} "
          f"ARI {a_warm:.4f} ({iw['init_used']})")
    assert iw["init_used"] == "warm"
    assert iw["phi_init_warm"] < ic["phi_init_cold"]
    assert t_warm is not None and t_cold is not None and t_warm < t_cold
    assert iw["best_phi"] <= target
    assert a_warm >= a_cold - 0.01
