"""Host: the stored full-size oracle results still describe the inputs the generator makes.

Each file under tests/golden/full_scale/ records the SHA-256 of the generated input it was
computed on; a changed generator would make the GPU comparison meaningless.  Regenerating the
largest inputs takes minutes, so this checks the n = 250k graph (the benchmark family at one
tenth of its size) and the metadata of every stored result.
"""
import glob
import json
import os

import numpy as np

from paper_2408_05459_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "full_scale")


def test_stored_results_are_complete():
    files = sorted(glob.glob(os.path.join(GOLD, "*.json")))
    assert len(files) >= 4
    for f in files:
        meta = json.load(open(f))
        lab = np.load(f[:-5] + ".npz")["labels"]
        net_n = {"c2": 100_000, "c3": 500_000, "c4": 2_500_000, "c5": 1_000_000}[os.path.basename(f)[:2]]
        assert lab.shape == (int(round(net_n * meta["scale"])),)
        assert meta["stop_reason"] in ("early_stop", "converged", "max_iter")
        ts = [t for t, _ in meta["phi_trace"]]
        assert ts == sorted(ts) and ts[0] == 0 and meta["best_t"] in ts
        assert abs(dict(meta["phi_trace"])[meta["best_t"]] - meta["best_phi"]) == 0.0
        assert len(meta["input_sha256"]) == 64


def test_generator_digest_unchanged():
    from tests.golden.make_full_scale import input_digest
    meta = json.load(open(os.path.join(GOLD, "c4_scale0.1.json")))
    net, prm = synth.make_config(meta["config"], scale=meta["scale"])
    assert input_digest(net, prm) == meta["input_sha256"]
