#!/usr/bin/env python3
"""Benchmark of the clustering hot path on one MI355X.

One step = one whole clustering run through the C ABI (ancka_cluster): exact KNN graph over the
attributes (BF16 MFMA tiles + FP64 rescoring), operator build, greedy initial BCM, orthogonal
iteration with Cholesky QR, Discretize and MHC every tau iterations, early termination.  The
workload is the n = 2.5M attributed graph (50 planted clusters, power-law SBM of mean degree 30,
BF16 attributes d = 128 from a 50-component Gaussian mixture, K = 10), generated synthetically
and resident in HBM before the timed region starts.

stdout: one JSON line.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cluster wall-s at n=2.5M; KNN TFLOP/s; SpMM HBM GB/s; warm vs cold iters"
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBPS = 8000.0


def committed_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (profiles/traffic.json), or None when the kernel's source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)[kernel]
        with open(os.path.join(ROOT, t["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != t["source_sha256"]:
                return None
        return t["traffic_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def committed_mfma(pass_name: str):
    """MFMA utilisation counters of a BF16 KNN pass from the committed rocprofv3 summary
    (profiles/mfma.json), or None when the kernel source changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "mfma.json")
    try:
        with open(path) as f:
            t = json.load(f)
        with open(os.path.join(ROOT, t["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != t["source_sha256"]:
                return None
        e = t[pass_name]
        return {"mfma_util": e["mfma_util"], "clock_ghz": e["clock_ghz"], "mfma_tflops": e["mfma_tflops"]}
    except (OSError, KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmm_compulsory_bytes(info, n, L, kp, es=4):
    """Compulsory bytes of one Z = P Q: topology indices + row pointers + per-segment scales,
    KNN indices and values + row pointers, per-row self coefficient, Q read once, Z written once."""
    topo = 4 * info["nnz_topo"] + 8 * (n * L + 1) + es * n * L
    knn = (4 + es) * info["nnz_knn"] + 8 * (n + 1)
    rows = es * n
    blocks = 2 * es * n * kp
    return topo + knn + rows + blocks


def host_threads() -> int:
    """Threads the CPU legs use: the CPUs this process may run on, at most 16 (one GPU's share
    of the host)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail))


def cpu_baseline(net, prm, gpu_iters, gpu_checks, knn_rows=512, small_scale=0.02):
    """The FP64 oracle timed on a bounded sample of the workload, extrapolated to one run.

    Sample: (a) exact KNN of query rows against all n candidates: one call on `knn_rows` rows
    and one on 2 * `knn_rows` rows, with X already in FP64; their difference is the cost per
    row, the rest the once-per-call work (squared norms, threshold slice), so a full run costs
    once + per_row * n; (b) the oracle's operator build, one orthogonal iteration, one
    Discretize and one MHC on the same workload generated at `small_scale` (same
    distributions), scaled linearly in n and by the GPU run's iteration and check counts."""
    import oracle
    from paper_2408_05459_amd import synth
    from threadpoolctl import threadpool_info
    threads = host_threads()
    X = np.asarray(net.X, dtype=np.float64)
    rng = np.random.default_rng(12345)
    rows = np.sort(rng.choice(net.n, size=2 * knn_rows, replace=False))
    t0 = time.perf_counter()
    oracle.knn(X, prm.K, rows=rows[:knn_rows], threads=threads)
    t1 = time.perf_counter()
    oracle.knn(X, prm.K, rows=rows, threads=threads)
    t2 = time.perf_counter()
    per_row = ((t2 - t1) - (t1 - t0)) / knn_rows
    once = max(0.0, (t1 - t0) - per_row * knn_rows)
    t_knn = once + per_row * net.n
    del X
    small, sp = synth.make_config(4, scale=small_scale)
    _, zero = oracle.normalize_rows(small.X)
    ki, ks = oracle.knn(small.X, sp.K, threads=threads)
    t0 = time.perf_counter()
    op = oracle.build_operator(small.kind, small.n, small.ptrs, small.idxs, small.m, zero, ki, ks, sp.beta)
    t_op = time.perf_counter() - t0
    y0, _ = oracle.init_bcm(op, small.k, sp.alpha, sp.T_i)
    C = np.concatenate([np.full((small.n, 1), 1 / math.sqrt(small.n)), oracle.normalized_bcm(y0, small.k)], axis=1)
    Q = oracle.initial_q(C)
    t0 = time.perf_counter()
    Q, _ = oracle.qr_pos(oracle.apply_P(op, Q))
    t_it = time.perf_counter() - t0
    t0 = time.perf_counter()
    y, _, _, _ = oracle.discretize(Q[:, 1:])
    t_disc = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.mhc(op, y, small.k, sp.alpha, sp.gamma)
    t_mhc = time.perf_counter() - t0
    f = net.n / small.n
    total = t_knn + f * (t_op + gpu_iters * t_it + gpu_checks * (t_disc + t_mhc))
    blas = sorted({f"{i.get('internal_api')} {i.get('num_threads')} threads" for i in threadpool_info()
            if i.get("user_api") == "blas"})
    return {
        "value": round(total, 1), "unit": "s", "cores": threads, "kind": "oracle",
        "sample": (f"exact FP64 KNN of {knn_rows} and {2 * knn_rows} random query rows against all {net.n} "
                   f"candidates (X converted to FP64 beforehand), {per_row * 1e3:.2f} ms per row plus "
                   f"{once:.2f} s once per call, extrapolated to {net.n} rows on {threads} threads (one "
                   f"single-threaded BLAS product per thread); operator build + 1 orthogonal iteration + 1 "
                   f"Discretize + 1 MHC on the same workload at n={small.n} scaled x{f:.0f} and by the GPU run's "
                   f"{gpu_iters} iterations / {gpu_checks} checks (scipy sparse products single-threaded, dense "
                   f"BLAS: {', '.join(blas) or 'unknown'})"),
        "phases_s": {"knn": round(t_knn, 1), "operator": round(f * t_op, 2),
                     "iterations": round(f * gpu_iters * t_it, 2),
                     "discretize+mhc": round(f * gpu_checks * (t_disc + t_mhc), 2)},
    }


# The paper's own end-to-end times (KNN included) on its hardware: context, not a target.
PAPER_TIMES = {
    "hardware": "Intel Xeon Gold 6226R, 16 threads, 384 GB RAM (CPU); NVIDIA RTX 3090 (GPU) (Sec. 8)",
    "knn_method": "GPU: Faiss Flat below 100k nodes, IVFPQ (approximate) above; CPU: ScaNN (approximate)",
    "amazon2m_agc_s": {"cpu": 1708, "gpu": 158.9, "note": "attributed graph, about 2M nodes, the closest "
                       "analogue of the benchmarked workload"},
    "amazon_ahc_s": {"cpu": 1286, "gpu": 152.3, "note": "attributed hypergraph, 2.27M nodes"},
    "mag_pm_ahc_s": {"cpu": 1371, "gpu": 120.2, "note": "attributed hypergraph, more than 2M nodes"},
    "tweibo_agc_s": {"cpu": 1318, "gpu": 105.0},
}


def warm_vs_cold(lib, graphs: int, n_train: int, epochs: int, lr: float, n_test: int, workers: int):
    """Learned warm start on the n = 1M hypergraph of the warm-start family (d = 512, k = 30):
    train the MLP on `graphs` seeded graphs of n_train nodes (targets from the plain method's
    eigenblocks), then run the method cold and warm-started on the test graph and compare
    iterations and wall time to reach the cold run's conductance (within 1e-4 relative)."""
    import torch
    from paper_2408_05459_amd import synth, warmstart
    t0 = time.perf_counter()
    seeds = list(range(5001, 5001 + graphs))
    exs = warmstart.make_examples(lib, n_train, seeds, workers=workers, log=log)
    t_data = time.perf_counter() - t0
    ws, tl = warmstart.train(lib, exs, 512, 30, epochs=epochs, lr=lr, seed=0)
    log(f"trained on {graphs} graphs x {n_train} rows, {epochs} epochs: loss {tl.epoch_loss[0]:.4f} -> "
        f"{tl.epoch_loss[-1]:.4f} in {tl.seconds:.1f}s")
    plain_iters = float(np.mean([e.iters for e in exs]))
    del exs
    torch.cuda.empty_cache()
    t1 = time.perf_counter()
    net, prm = synth.make_warm_graph(n_test, 5000)
    log(f"generated {net.name} in {time.perf_counter() - t1:.1f}s")
    s, keep = lib.network(net)
    X = keep[-1]
    warmstart.run(lib, s, X, net.k, prm)                       # first call: kernels and workspaces warm
    lc, ic, tc = warmstart.run(lib, s, X, net.k, prm)
    lw, iw, tw = warmstart.run(lib, s, X, net.k, prm, ws=ws)
    target = ic["best_phi"] * (1 + 1e-4)
    t_cold = warmstart.time_to_reach(ic, target)
    t_warm = warmstart.time_to_reach(iw, target)
    # end-to-end time to the cold run's objective: the same runs stopped at that iteration
    to_target = {}
    for tag, t_hit, model in (("cold", t_cold, None), ("warm", t_warm, ws)):
        if t_hit is None:
            to_target[tag] = None
            continue
        _, it_, tm_ = warmstart.run(lib, s, X, net.k, prm, ws=model, T_a=t_hit)
        to_target[tag] = {"iterations": t_hit, "best_phi": it_["best_phi"], "ms": round(tm_["total"], 1)}
    from sklearn.metrics import adjusted_rand_score
    res = {
        "workload": net.name, "train_graphs": graphs, "train_n": n_train, "epochs": epochs,
        "train_loss_first_last": [round(tl.epoch_loss[0], 5), round(tl.epoch_loss[-1], 5)],
        "train_s": round(tl.seconds, 2), "train_data_s": round(t_data, 1),
        "train_plain_iters_mean": plain_iters,
        "target_phi": target,
        "to_target": to_target,
        "speedup_to_target": (round(to_target["cold"]["ms"] / to_target["warm"]["ms"], 3)
                              if to_target.get("cold") and to_target.get("warm") else None),
        "cold": {"iterations": ic["iterations"], "stop": ic["stop_reason"], "best_phi": ic["best_phi"],
                 "best_t": ic["best_t"], "iters_to_target": t_cold, "ms": {k_: round(v, 1) for k_, v in tc.items()},
                 "ari_vs_planted": round(float(adjusted_rand_score(net.labels, lc.cpu().numpy())), 4)},
        "warm": {"iterations": iw["iterations"], "stop": iw["stop_reason"], "best_phi": iw["best_phi"],
                 "best_t": iw["best_t"], "iters_to_target": t_warm, "init_used": iw["init_used"],
                 "phi_init_cold": iw["phi_init_cold"], "phi_init_warm": iw["phi_init_warm"],
                 "ms": {k_: round(v, 1) for k_, v in tw.items()},
                 "ari_vs_planted": round(float(adjusted_rand_score(net.labels, lw.cpu().numpy())), 4)},
    }
    log(f"cold: {ic['iterations']} iterations, phi {ic['best_phi']:.6f}, {tc['total']:.0f} ms; "
        f"warm: {iw['iterations']} iterations, phi {iw['best_phi']:.6f}, {tw['total']:.0f} ms")
    del keep, X, ws
    torch.cuda.empty_cache()
    return res


def gemm_reference():
    """The vendor BF16 GEMM (torch.matmul, hipBLASLt) on the same GPU, for context: large square
    products and the n x n x 128 shape of the KNN similarity product.  One JSON line."""
    import torch
    out = []
    for M, N, K, reps in ((8192, 8192, 8192, 20), (16384, 16384, 8192, 5), (32768, 32768, 128, 10),
                          (65536, 65536, 128, 5), (65536, 65536, 256, 5)):
        a = torch.randn(M, K, device="cuda", dtype=torch.bfloat16)
        b = torch.randn(N, K, device="cuda", dtype=torch.bfloat16)
        for _ in range(3):
            c = a @ b.T
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            c = a @ b.T
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out.append({"M": M, "N": N, "K": K, "ms": round(ms, 3), "tflops": round(2.0 * M * N * K / ms / 1e9, 1)})
        log(f"{M}x{N}x{K}: {ms:.3f} ms, {out[-1]['tflops']} TFLOP/s")
        del a, b, c
    print(json.dumps({"gemm_reference_bf16": out}), flush=True)


def spmm_reference(lib, cfg: int, scale: float, reps: int = 10):
    """The vendor sparse product (torch.sparse CSR @ dense, hipSPARSE) on the sparsity structure of
    the walk operator P of the benchmark graph (topology rows plus KNN rows; values do not change
    the cost), against the library's own Z = P Q on the same graph.  One JSON line."""
    import torch
    from paper_2408_05459_amd import binding, synth
    net, prm = synth.make_config(cfg, scale=scale)
    n = net.n
    s, keep = lib.network(net)
    X = binding.upload_attributes(net.X, net.x_dtype)
    idx, sim, _ = lib.knn(X, prm.K, prm.knn_mode)
    op = lib.build_operator(s, idx, sim, prm.K, prm.beta, prm.q_dtype)
    info = op.info()
    del X
    kp = net.k + 1
    Q = torch.randn((n, 64), dtype=torch.float32, device="cuda")
    Q[:, kp:] = 0
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for _ in range(3):
        op.apply(Q)
    ev[0].record()
    for _ in range(reps):
        op.apply(Q)
    ev[1].record()
    torch.cuda.synchronize()
    own_ms = ev[0].elapsed_time(ev[1]) / reps
    # structure of P: the symmetrised topology rows, then each row's KNN neighbours (both directions)
    ptr = torch.from_numpy(np.asarray(net.ptrs[0], dtype=np.int64)).cuda()
    rows_t = torch.repeat_interleave(torch.arange(n, device="cuda"), ptr[1:] - ptr[:-1])
    cols_t = torch.from_numpy(np.asarray(net.idxs[0], dtype=np.int64)).cuda()
    ki = idx.long()
    kr = torch.arange(n, device="cuda").repeat_interleave(prm.K)
    kc = ki.reshape(-1)
    ok = kc >= 0
    r_all = torch.cat([rows_t, cols_t, kr[ok], kc[ok]])
    c_all = torch.cat([cols_t, rows_t, kc[ok], kr[ok]])
    key = torch.unique(r_all * n + c_all)
    del r_all, c_all, rows_t, cols_t, kr, kc
    rr, cc = key // n, key % n
    crow = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    crow[1:] = torch.cumsum(torch.bincount(rr, minlength=n), 0)
    vals = torch.rand(key.numel(), dtype=torch.float32, device="cuda")
    P = torch.sparse_csr_tensor(crow, cc, vals, size=(n, n))
    Qd = Q[:, :kp].contiguous()
    for _ in range(3):
        Z = P @ Qd
    ev[2].record()
    for _ in range(reps):
        Z = P @ Qd
    ev[3].record()
    torch.cuda.synchronize()
    lib_ms = ev[2].elapsed_time(ev[3]) / reps
    # the same product as a weighted gather-sum per row (torch embedding_bag, mode 'sum')
    import torch.nn.functional as F
    offs = crow[:-1].contiguous()
    for _ in range(3):
        Z = F.embedding_bag(cc, Qd, offs, mode="sum", per_sample_weights=vals)
    ev[2].record()
    for _ in range(reps):
        Z = F.embedding_bag(cc, Qd, offs, mode="sum", per_sample_weights=vals)
    ev[3].record()
    torch.cuda.synchronize()
    bag_ms = ev[2].elapsed_time(ev[3]) / reps
    out = {"workload": net.name, "nnz_P_structure": int(key.numel()), "cols": kp,
           "own_spmm_ms": round(own_ms, 3), "torch_sparse_csr_ms": round(lib_ms, 3),
           "torch_embedding_bag_ms": round(bag_ms, 3),
           "own_nnz": int(info["nnz_topo"] + info["nnz_knn"]),
           "speedup_vs_sparse_csr": round(lib_ms / own_ms, 2), "speedup_vs_embedding_bag": round(bag_ms / own_ms, 2)}
    log(f"Z = P Q: library kernel {own_ms:.3f} ms, torch sparse CSR {lib_ms:.3f} ms, embedding_bag {bag_ms:.3f} ms "
        f"on {key.numel()} entries")
    print(json.dumps({"spmm_reference": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--spmm-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-warm", action="store_true", help="skip the learned warm start comparison")
    ap.add_argument("--no-ivf", action="store_true", help="skip the IVF (approximate KNN) comparison")
    ap.add_argument("--ivf-nlist", type=int, default=1024)
    ap.add_argument("--ivf-nprobe", type=int, default=32)
    ap.add_argument("--ws-graphs", type=int, default=200)
    ap.add_argument("--ws-n", type=int, default=50000)
    ap.add_argument("--ws-epochs", type=int, default=8)
    ap.add_argument("--ws-lr", type=float, default=1e-3)
    ap.add_argument("--ws-test-n", type=int, default=1000000)
    ap.add_argument("--ws-workers", type=int, default=host_threads())
    ap.add_argument("--study", default=None, metavar="OUT.json",
                    help="only run the parameter sweeps and convergence traces on the synthetic workloads "
                         "(sweep.study) and write them to OUT.json, then exit")
    ap.add_argument("--spmm-reference", action="store_true",
                    help="only time the vendor sparse product (torch sparse CSR) on the operator's structure "
                         "beside the library's Z = P Q, then exit")
    ap.add_argument("--gemm-reference", action="store_true",
                    help="only time the vendor BF16 GEMM (torch.matmul) for context, then exit")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="copy a buffer of this many MiB three times first (reference kernel for HBM counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {a.gpus}); the method's multi-GPU sharding is "
              f"described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2408_05459_amd import binding, synth

    torch.cuda.set_device(0)
    if a.gemm_reference:
        gemm_reference()
        return
    lib = binding.load()
    if a.spmm_reference:
        spmm_reference(lib, a.config, a.scale)
        return
    if a.study:
        from paper_2408_05459_amd import sweep
        t0 = time.perf_counter()
        res = sweep.study(lib, log=log)
        res["seconds"] = round(time.perf_counter() - t0, 1)
        with open(a.study, "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps({"study": a.study, "seconds": res["seconds"]}), flush=True)
        return
    if a.copy_calibration_mib > 0:
        nb = a.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nb} bytes read and {nb} bytes written per launch")
        del src, dst
    t0 = time.perf_counter()
    net, prm = synth.make_config(a.config, scale=a.scale)
    log(f"generated {net.name} in {time.perf_counter() - t0:.1f}s")
    s, keep = lib.network(net)
    params = lib.default_params(k=net.k, K=prm.K, alpha=prm.alpha, beta=prm.beta, gamma=prm.gamma, tau=prm.tau,
                                T_i=prm.T_i, T_a=prm.T_a, eps_q=prm.eps_q, knn_mode=prm.knn_mode,
                                q_dtype=prm.q_dtype)
    torch.cuda.synchronize()

    for w in range(a.warmup):
        _, info = lib.cluster(s, params)
        log(f"warmup {w}: iterations {info['iterations']} phases {info['phase_ms']}")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for st in range(a.steps):
        labels, info = lib.cluster(s, params)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / a.steps
    for i, info in enumerate(infos):
        log(f"step {i}: iterations {info['iterations']} ({info['stop_reason']}) best phi {info['best_phi']:.6f} "
            f"phases {json.dumps({k: round(v, 1) for k, v in info['phase_ms'].items()})}")
    last = infos[-1]
    from sklearn.metrics import adjusted_rand_score
    ari_planted = float(adjusted_rand_score(net.labels, labels.cpu().numpy()))

    # ---- KNN tile phase: algorithmic (unordered-pair) and executed FLOPs.  The window pass
    # scores each ordered pair of its window (both orders of a pair), the symmetric pass each
    # remaining unordered pair once.
    n, d = net.n, net.d
    tile_ms = float(np.mean([i["knn_tile_ms"] for i in infos]))
    sym_ms = float(np.mean([i["knn_sym_ms"] for i in infos]))
    window = last["knn_window"]
    sym_pairs = last["knn_sym_pairs"]
    qb = 256
    npad = -(-n // qb) * qb
    win_pairs = float(npad) * npad if window < 0 else float(npad) * (2 * window + 1) * qb
    useful = float(n) * (n - 1) * d
    executed = 2.0 * d * (win_pairs + sym_pairs)
    knn_useful_tf = useful / (tile_ms * 1e-3) / 1e12
    knn_exec_tf = executed / (tile_ms * 1e-3) / 1e12
    sym_tf = 2.0 * d * sym_pairs / (sym_ms * 1e-3) / 1e12 if sym_ms > 0 else 0.0

    # ---- SpMM Z = P Q of the iteration, timed with HIP events on the library's stream
    X = binding.upload_attributes(net.X, net.x_dtype)
    nidx, nsim, _ = lib.knn(X, prm.K, prm.knn_mode)
    op = lib.build_operator(s, nidx, nsim, prm.K, prm.beta, prm.q_dtype)
    oinfo = op.info()
    kp = net.k + 1
    ld = ((kp * 4 + 127) // 128) * 32 if kp * 4 > 128 else max(4, 1 << (kp - 1).bit_length())   # as the library pads
    Q = torch.randn((n, ld), dtype=torch.float32, device="cuda")
    for _ in range(3):
        op.apply(Q)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.spmm_reps):
        op.apply(Q)
    e1.record()
    torch.cuda.synchronize()
    spmm_ms = e0.elapsed_time(e1) / a.spmm_reps
    spmm_bytes = spmm_compulsory_bytes(oinfo, n, net.L, kp)
    spmm_gbps = spmm_bytes / (spmm_ms * 1e-3) / 1e9
    spmm_traffic = committed_traffic("spmm_kernel")
    # the same product with Q stored in BF16 (measured beside; the method keeps FP32 blocks)
    Qb = Q.to(torch.bfloat16)
    for _ in range(3):
        op.apply_bf16(Qb)
    e0.record()
    for _ in range(a.spmm_reps):
        op.apply_bf16(Qb)
    e1.record()
    torch.cuda.synchronize()
    spmm_bf16_ms = e0.elapsed_time(e1) / a.spmm_reps
    spmm_bf16_bytes = spmm_bytes - 2 * n * kp      # Q read at 2 bytes per element instead of 4
    del Qb
    # ---- IVF search (approximate) at the same size: time, recall against the exact lists above,
    # and the whole method with IVF lists against the exact run's labels
    ivf = None
    if not a.no_ivf:
        ivf = {"nlist": a.ivf_nlist, "nprobe": a.ivf_nprobe}
        lib.knn_ivf(X, prm.K, a.ivf_nlist, a.ivf_nprobe)          # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iidx, isim, ist = lib.knn_ivf(X, prm.K, a.ivf_nlist, a.ivf_nprobe)
        torch.cuda.synchronize()
        ivf["knn_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
        ivf["tile_ms"] = round(ist.tile_ms, 2)
        ivf["pairs_fraction"] = round(ist.sym_pairs / float(n) ** 2, 5)
        hits = torch.zeros((), dtype=torch.int64, device="cuda")
        for r0 in range(0, n, 1 << 18):
            a_ = iidx[r0:r0 + (1 << 18)].long()
            b_ = nidx[r0:r0 + (1 << 18)].long()
            m = (a_[:, :, None] == b_[:, None, :]) & (b_[:, None, :] >= 0)
            hits += m.any(dim=2).sum()
        ivf["recall_at_K"] = round(int(hits) / float(int((nidx >= 0).sum())), 5)
        del iidx, isim
        pi = lib.default_params(k=net.k, K=prm.K, alpha=prm.alpha, beta=prm.beta, gamma=prm.gamma, tau=prm.tau,
                                T_i=prm.T_i, T_a=prm.T_a, eps_q=prm.eps_q, knn_mode="ivf", q_dtype=prm.q_dtype)
        pi.ivf_nlist, pi.ivf_nprobe = a.ivf_nlist, a.ivf_nprobe
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        li, ii = lib.cluster(s, pi)
        torch.cuda.synchronize()
        ivf["cluster_s"] = round(time.perf_counter() - t0, 4)
        ivf["cluster_phases_ms"] = {k_: round(v, 1) for k_, v in ii["phase_ms"].items()}
        ivf["ari_vs_exact_run"] = round(float(adjusted_rand_score(labels.cpu().numpy(), li.cpu().numpy())), 5)
        ivf["best_phi"] = ii["best_phi"]
        ivf["best_phi_exact_run"] = last["best_phi"]
        ivf["iterations"] = ii["iterations"]
        log(f"IVF nlist {a.ivf_nlist} nprobe {a.ivf_nprobe}: KNN {ivf['knn_ms']} ms, recall {ivf['recall_at_K']}, "
            f"cluster {ivf['cluster_s']} s, ARI vs exact run {ivf['ari_vs_exact_run']}")
    del X, nidx, nsim, op, Q
    torch.cuda.empty_cache()

    iters = last["iterations"]
    spmm_total_ms = iters * spmm_ms
    if sym_ms > 0 and sym_ms >= spmm_total_ms:
        # the symmetric pass scores each of its pairs once: its FLOPs are all algorithmic
        roof = {"kernel": "knn_bf16_kernel, symmetric pass (similarity tiles + both rows' top-2K)",
                "bound": "mfma", "achieved": round(sym_tf, 1), "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                "frac": round(sym_tf / PEAK_BF16_TFLOPS, 4), "traffic": committed_traffic("knn_bf16_kernel_sym"),
                "counters": committed_mfma("symmetric")}
    elif tile_ms >= spmm_total_ms:
        roof = {"kernel": "knn_bf16_kernel (similarity tiles + top-2K)", "bound": "mfma",
                "achieved": round(knn_useful_tf, 1), "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                "frac": round(knn_useful_tf / PEAK_BF16_TFLOPS, 4), "traffic": committed_traffic("knn_bf16_kernel")}
    else:
        roof = {"kernel": "spmm_kernel (Z = P Q)", "bound": "hbm", "achieved": round(spmm_gbps, 1),
                "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": round(spmm_gbps / PEAK_HBM_GBPS, 4),
                "traffic": committed_traffic("spmm_kernel")}

    out = {
        "metric": METRIC,
        "value": round(ms_per_step / 1000.0, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": net.name, "n": n, "k": net.k, "d": d, "K": prm.K,
                   "nnz_topology": int(sum(int(p[-1]) for p in net.ptrs)),
                   "precision": "KNN BF16 MFMA (FP32 accumulation) + FP64 rescoring; SpMM FP32; k x k FP64",
                   "parallelism": "1 GPU"},
        "roofline": roof,
        "knn": {"tile_ms": round(tile_ms, 2), "tflops_useful": round(knn_useful_tf, 1),
                "tflops_executed": round(knn_exec_tf, 1), "frac_executed": round(knn_exec_tf / PEAK_BF16_TFLOPS, 4),
                "uncertified_rows": last["knn_uncertified_rows"], "call_ms": round(last["knn_total_ms"], 2),
                "window_blocks": window, "sym_ms": round(sym_ms, 2), "sym_pairs": sym_pairs,
                "sym_tflops": round(sym_tf, 1), "handed_over": last["knn_handed_over"],
                "mfma_counters": {p: committed_mfma(p) for p in ("bound", "window", "symmetric")},
                "rescanned": last["knn_rescanned"]},
        "spmm": {"ms": round(spmm_ms, 3), "compulsory_bytes": spmm_bytes, "gbps_compulsory": round(spmm_gbps, 1),
                 "traffic_bytes": spmm_traffic,
                 # counter bytes read and written beyond L2 per launch over this run's launch time
                 "gbps_traffic": (round(spmm_traffic / (spmm_ms * 1e-3) / 1e9, 1) if spmm_traffic else None),
                 "frac": round(spmm_gbps / PEAK_HBM_GBPS, 4),
                 "bf16_block": {"ms": round(spmm_bf16_ms, 3), "compulsory_bytes": spmm_bf16_bytes,
                                "gbps_compulsory": round(spmm_bf16_bytes / (spmm_bf16_ms * 1e-3) / 1e9, 1)},
                 "nnz_topology": oinfo["nnz_topo"],
                 "nnz_knn": oinfo["nnz_knn"], "cols": kp},
        "phases_ms": {k_: round(v, 1) for k_, v in last["phase_ms"].items()},
        "iterations": iters,
        "stop_reason": last["stop_reason"],
        "best_phi": last["best_phi"],
        "ari_vs_planted": round(ari_planted, 4),
        "ivf": ivf,
    }
    if not a.no_warm:
        out["warm_start"] = warm_vs_cold(lib, a.ws_graphs, a.ws_n, a.ws_epochs, a.ws_lr, a.ws_test_n, a.ws_workers)
    out["paper_times_context"] = PAPER_TIMES
    if not a.no_cpu_baseline:
        log("timing the oracle on a bounded sample ...")
        checks = sum(1 for t, _ in last["trace"] if t > 0)
        out["cpu_baseline"] = cpu_baseline(net, prm, iters, checks)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
