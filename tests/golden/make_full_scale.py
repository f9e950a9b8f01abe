"""Write the oracle's clustering of a full-size synthetic workload to tests/golden/full_scale/.

Only ``oracle`` (the FP64 CPU implementation) and the seeded input generator are called;
nothing here touches the GPU library.  The GPU test ``tests/test_gpu_full_scale.py``
regenerates the same input, checks its digest, and compares the GPU clustering with the
stored result.

    python tests/golden/make_full_scale.py --config 4 --scale 0.1 [--scratch DIR]

The exact FP64 KNN of Sec. 3.1 is the long step (n^2 d multiply-adds: hours on a few
cores at n = 2.5M).  With ``--scratch`` it is computed in slices of query rows, each saved
there as it finishes, so an interrupted run resumes where it stopped; slices are keyed by
the input digest, so a changed generator never reuses them.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2408_05459_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "full_scale")


def name_of(cfg: int, scale: float) -> str:
    return f"c{cfg}_scale{scale:g}"


def input_digest(net, prm) -> str:
    """SHA-256 over everything the method reads: attributes, topology, sizes and parameters."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(net.X).tobytes())
    for a in list(net.ptrs) + list(net.idxs):
        h.update(np.ascontiguousarray(a).tobytes())
    meta = dict(kind=int(net.kind), n=int(net.n), k=int(net.k), m=int(net.m), d=int(net.d),
                x_dtype=net.x_dtype, K=prm.K, alpha=prm.alpha, beta=prm.beta, gamma=prm.gamma,
                tau=prm.tau, T_i=prm.T_i, T_a=prm.T_a, eps_q=prm.eps_q,
                disc_max_iter=prm.disc_max_iter)
    h.update(json.dumps(meta, sort_keys=True).encode())
    return h.hexdigest()


def knn_sliced(X, K, digest, scratch, rows_per_slice=65536, log=print):
    n = X.shape[0]
    idx = np.empty((n, K), dtype=np.int64)
    sim = np.empty((n, K), dtype=np.float64)
    for r0 in range(0, n, rows_per_slice):
        r1 = min(n, r0 + rows_per_slice)
        path = os.path.join(scratch, f"knn_{digest[:16]}_{r0}_{r1}.npz") if scratch else None
        if path and os.path.exists(path):
            z = np.load(path)
            idx[r0:r1], sim[r0:r1] = z["idx"], z["sim"]
            log(f"knn rows {r0}..{r1}: from {path}")
            continue
        t = time.time()
        idx[r0:r1], sim[r0:r1] = oracle.knn(X, K, rows=np.arange(r0, r1))
        if path:
            np.savez(path + ".tmp.npz", idx=idx[r0:r1], sim=sim[r0:r1])
            os.replace(path + ".tmp.npz", path)
        log(f"knn rows {r0}..{r1} of {n}: {time.time() - t:.1f} s")
    return idx, sim


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, required=True)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--scratch", default=None, help="directory for resumable KNN slices")
    a = ap.parse_args()

    def log(msg):
        print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)

    t0 = time.time()
    net, prm = synth.make_config(a.config, scale=a.scale)
    digest = input_digest(net, prm)
    log(f"{net.name}: digest {digest[:16]}")
    if a.scratch:
        os.makedirs(a.scratch, exist_ok=True)
    X = np.asarray(net.X, dtype=np.float64)
    tk = time.time()
    ki, ks = knn_sliced(X, prm.K, digest, a.scratch, log=log)
    t_knn = time.time() - tk
    _, zero = oracle.normalize_rows(X)
    del X
    tc = time.time()
    op = oracle.build_operator(net.kind, net.n, net.ptrs, net.idxs, net.m, zero, ki, ks, prm.beta)
    labels, rep = oracle.cluster(op, net.k, alpha=prm.alpha, gamma=prm.gamma, tau=prm.tau,
                                 T_i=prm.T_i, T_a=prm.T_a, eps_q=prm.eps_q,
                                 disc_max_iter=prm.disc_max_iter)
    t_cluster = time.time() - tc
    log(f"cluster: {rep.iterations} iterations, {rep.reason}, best phi {rep.best_phi:.9f} at t={rep.best_t}")

    os.makedirs(OUT, exist_ok=True)
    name = name_of(a.config, a.scale)
    np.savez_compressed(os.path.join(OUT, name + ".npz"),
                        labels=labels.astype(np.uint8 if net.k <= 255 else np.int32))
    meta = {
        "workload": net.name, "config": a.config, "scale": a.scale, "n": int(net.n), "k": int(net.k),
        "input_sha256": digest,
        "params": {"K": prm.K, "alpha": prm.alpha, "beta": prm.beta, "gamma": prm.gamma, "tau": prm.tau,
                   "T_i": prm.T_i, "T_a": prm.T_a, "eps_q": prm.eps_q, "disc_max_iter": prm.disc_max_iter},
        "iterations": int(rep.iterations), "stop_reason": rep.reason,
        "best_phi": float(rep.best_phi), "best_t": int(rep.best_t),
        "phi_trace": [[int(t), float(p)] for t, p in rep.phi_trace],
        "phi_init_cold": float(rep.phi_init_cold),
        "knn_zero_rows": int(zero.sum()),
        "oracle_seconds": {"knn": round(t_knn, 1), "operator_and_cluster": round(t_cluster, 1),
                           "total": round(time.time() - t0, 1)},
        "written_by": "tests/golden/make_full_scale.py (oracle only)",
    }
    with open(os.path.join(OUT, name + ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    log(f"wrote {name}: {json.dumps({k: meta[k] for k in ('iterations', 'stop_reason', 'best_phi')})}")


if __name__ == "__main__":
    main()
