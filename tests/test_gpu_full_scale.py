"""Full-size clustering parity: the whole GPU method (ancka_cluster, in the launch
configuration the benchmark times) against the FP64 oracle's clustering of the same workload.

The oracle's results (labels, conductance trace, stopping iteration and reason) are written by
tests/golden/make_full_scale.py, which calls only the oracle and the input generator, together
with a SHA-256 digest of the generated input; the test regenerates the input, checks the digest
and compares.  Bar: ARI(gpu, oracle) >= 0.99; best conductance within 1e-4 relative; the same
stopping iteration, reason and best iteration; every traced conductance within 1e-4 relative.
The GPU's own conductance of the oracle's labels (on the operator it builds from its own KNN
lists) must also match the oracle's value within 1e-4.
"""
import glob
import json
import os

import numpy as np
import pytest

from paper_2408_05459_amd import synth
from tests.helpers import ari

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
FILES = sorted(glob.glob(os.path.join(HERE, "golden", "full_scale", "*.json")))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("path", FILES, ids=[os.path.basename(f)[:-5] for f in FILES])
def test_full_scale_cluster_matches_oracle(lib, path):
    import torch
    from tests.golden.make_full_scale import input_digest
    meta = json.load(open(path))
    ref = np.load(path[:-5] + ".npz")["labels"].astype(np.int64)
    net, prm = synth.make_config(meta["config"], scale=meta["scale"])
    assert input_digest(net, prm) == meta["input_sha256"], "generator changed: rerun make_full_scale.py"
    p = meta["params"]
    s, keep = lib.network(net)
    params = lib.default_params(k=net.k, K=p["K"], alpha=p["alpha"], beta=p["beta"], gamma=p["gamma"],
                                tau=p["tau"], T_i=p["T_i"], T_a=p["T_a"], eps_q=p["eps_q"],
                                knn_mode=prm.knn_mode, q_dtype=prm.q_dtype)
    params.disc_max_iter = p["disc_max_iter"]
    lg, info = lib.cluster(s, params)
    lg = lg.cpu().numpy()
    a = ari(lg, ref)
    print(f"{os.path.basename(path)}: n={net.n} ARI(gpu, oracle)={a:.5f} phi gpu {info['best_phi']:.7f} oracle "
          f"{meta['best_phi']:.7f}; iterations gpu {info['iterations']} ({info['stop_reason']}) oracle "
          f"{meta['iterations']} ({meta['stop_reason']}); best t gpu {info['best_t']} oracle {meta['best_t']}; "
          f"uncertified KNN rows {info['knn_uncertified_rows']}", flush=True)
    assert a >= 0.99
    assert abs(info["best_phi"] - meta["best_phi"]) <= 1e-4 * meta["best_phi"]
    assert (info["iterations"], info["stop_reason"], info["best_t"]) == \
        (meta["iterations"], meta["stop_reason"], meta["best_t"])
    assert [t for t, _ in info["trace"]] == [t for t, _ in meta["phi_trace"]]
    for (_, pg), (_, pr) in zip(info["trace"], meta["phi_trace"]):
        assert abs(pg - pr) <= 1e-4 * pr
    # the oracle's labels scored on the GPU's own operator
    from paper_2408_05459_amd.binding import upload_attributes
    X = upload_attributes(net.X, net.x_dtype)
    idx, sim, st = lib.knn(X, p["K"], prm.knn_mode)
    del X
    op = lib.build_operator(s, idx, sim, p["K"], p["beta"], prm.q_dtype)
    del idx, sim
    phi_ref_on_gpu = op.mhc(torch.from_numpy(ref.astype(np.int32)).cuda(), net.k, p["alpha"], p["gamma"])
    assert abs(phi_ref_on_gpu - meta["best_phi"]) <= 1e-4 * meta["best_phi"]
