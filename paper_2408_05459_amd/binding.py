"""Thin ctypes binding of libancka (include/ancka.h).

Functions keep the C names; pointer arguments accept torch tensors (device memory) or raw
integers, host outputs are returned.  Nothing here computes any part of the method: every
step runs in the HIP library, and loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import List, Optional

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libancka.so")

ANCKA_OK, ANCKA_ERR_INVALID_ARG, ANCKA_ERR_UNSUPPORTED, ANCKA_ERR_OOM, ANCKA_ERR_HIP, ANCKA_ERR_NUMERICAL = range(6)
ANCKA_F64, ANCKA_F32, ANCKA_BF16 = 0, 1, 2
ANCKA_HYPERGRAPH, ANCKA_GRAPH, ANCKA_MULTIPLEX = 0, 1, 2
ANCKA_KNN_EXACT_F64, ANCKA_KNN_EXACT_F32, ANCKA_KNN_BF16_RESCORE, ANCKA_KNN_IVF_BF16 = 0, 1, 2, 3
ANCKA_MAX_LAYERS = 16
ANCKA_NPHASES = 7
PHASES = ["knn", "operator", "init", "iterations", "discretize", "mhc", "warm"]
STOP_REASONS = ["max_iter", "converged", "early_stop"]

DTYPE_CODE = {"f64": ANCKA_F64, "f32": ANCKA_F32, "bf16": ANCKA_BF16}
KNN_MODE = {"f64": ANCKA_KNN_EXACT_F64, "f32": ANCKA_KNN_EXACT_F32, "bf16": ANCKA_KNN_BF16_RESCORE,
            "ivf": ANCKA_KNN_IVF_BF16}


class ancka_network(C.Structure):
    _fields_ = [("kind", C.c_int32), ("L", C.c_int32), ("n", C.c_int64), ("m", C.c_int64),
                ("ptr", C.c_void_p * ANCKA_MAX_LAYERS), ("idx", C.c_void_p * ANCKA_MAX_LAYERS),
                ("nnz", C.c_int64 * ANCKA_MAX_LAYERS), ("X", C.c_void_p), ("xdtype", C.c_int32),
                ("d", C.c_int64), ("ldx", C.c_int64)]


class ancka_params(C.Structure):
    _fields_ = [("k", C.c_int32), ("K", C.c_int32), ("alpha", C.c_double), ("beta", C.c_double),
                ("gamma", C.c_int32), ("tau", C.c_int32), ("T_i", C.c_int32), ("T_a", C.c_int32),
                ("eps_q", C.c_double), ("disc_max_iter", C.c_int32), ("knn_mode", C.c_int32),
                ("q_dtype", C.c_int32), ("early_stop", C.c_int32), ("ivf_nlist", C.c_int32),
                ("ivf_nprobe", C.c_int32)]


class ancka_knn_stats(C.Structure):
    _fields_ = [("zero_rows", C.c_int64), ("uncertified_rows", C.c_int64), ("recomputed_rows", C.c_int64),
                ("tile_ms", C.c_double), ("total_ms", C.c_double), ("sym_ms", C.c_double),
                ("sym_pairs", C.c_int64), ("handed_over", C.c_int64), ("window", C.c_int32),
                ("rescanned", C.c_int32)]


class ancka_report(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("stop_reason", C.c_int32), ("best_phi", C.c_double),
                ("best_t", C.c_int32), ("init_used", C.c_int32), ("phi_init_cold", C.c_double),
                ("phi_init_warm", C.c_double), ("trace_capacity", C.c_int32), ("trace_len", C.c_int32),
                ("trace_t", C.POINTER(C.c_int32)), ("trace_phi", C.POINTER(C.c_double)),
                ("phase_ms", C.c_double * ANCKA_NPHASES), ("knn", ancka_knn_stats),
                ("disc_iters_total", C.c_int32)]


class AnckaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ancka status {status}: {msg}")
        self.status = status


_VP = C.c_void_p
_SIGS = {
    "ancka_create": (C.c_int, [C.POINTER(_VP), C.c_int32, _VP]),
    "ancka_destroy": (None, [_VP]),
    "ancka_last_error": (C.c_char_p, [_VP]),
    "ancka_default_params": (ancka_params, []),
    "ancka_device_info": (C.c_int, [_VP, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "ancka_knn": (C.c_int, [_VP, _VP, C.c_int32, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int32, _VP, _VP,
                            C.POINTER(ancka_knn_stats)]),
    "ancka_knn_ivf": (C.c_int, [_VP, _VP, C.c_int32, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int32,
                                C.c_int32, _VP, _VP, C.POINTER(ancka_knn_stats)]),
    "ancka_build_operator": (C.c_int, [_VP, C.POINTER(ancka_network), _VP, _VP, C.c_int32, C.c_int32, C.c_double,
                                       C.c_int32, C.POINTER(_VP)]),
    "ancka_op_destroy": (None, [_VP]),
    "ancka_op_info": (C.c_int, [_VP, _VP, _VP, _VP, _VP, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "ancka_apply_p": (C.c_int, [_VP, _VP, _VP, _VP, C.c_int32, C.c_int64]),
    "ancka_apply_p_bf16": (C.c_int, [_VP, _VP, _VP, _VP, C.c_int32, C.c_int64]),
    "ancka_init_bcm": (C.c_int, [_VP, _VP, C.c_int32, C.c_double, C.c_int32, _VP]),
    "ancka_initial_block": (C.c_int, [_VP, _VP, _VP, _VP, C.c_int32, _VP, C.c_int64]),
    "ancka_orth_iter": (C.c_int, [_VP, _VP, _VP, C.c_int64, C.c_int32, C.c_int32, _VP, _VP]),
    "ancka_discretize": (C.c_int, [_VP, _VP, C.c_int32, C.c_int64, C.c_int32, C.c_int64, C.c_int32, _VP, _VP, _VP,
                                   _VP]),
    "ancka_discretize_noalloc": (C.c_int, [_VP, _VP, C.c_int32, C.c_int64, C.c_int32, C.c_int64, C.c_int32, _VP,
                                           _VP, _VP, _VP]),
    "ancka_mhc": (C.c_int, [_VP, _VP, _VP, C.c_int32, C.c_double, C.c_int32, C.POINTER(C.c_double)]),
    "ancka_cluster": (C.c_int, [_VP, C.POINTER(ancka_network), C.POINTER(ancka_params), _VP, _VP,
                                C.POINTER(ancka_report)]),
    "ancka_cluster_op": (C.c_int, [_VP, _VP, C.POINTER(ancka_params), _VP, _VP, C.POINTER(ancka_report)]),
    "ancka_ws_create": (C.c_int, [_VP, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.POINTER(_VP)]),
    "ancka_ws_destroy": (None, [_VP]),
    "ancka_ws_features": (C.c_int, [_VP, _VP, _VP, C.c_int32, C.c_int64, C.c_int64, _VP, C.c_int64]),
    "ancka_ws_forward": (C.c_int, [_VP, _VP, _VP, C.c_int64, C.c_int64, _VP, C.c_int32]),
    "ancka_ws_backward": (C.c_int, [_VP, _VP, _VP, _VP, C.c_int64, _VP]),
    "ancka_ws_step": (C.c_int, [_VP, _VP, C.c_double]),
    "ancka_ws_get_params": (C.c_int, [_VP, _VP, C.c_int32, _VP, C.POINTER(C.c_int64)]),
    "ancka_ws_set_params": (C.c_int, [_VP, _VP, _VP]),
    "ancka_ws_target": (C.c_int, [_VP, _VP, C.c_int32, C.c_int64, C.c_int32, C.c_int64, _VP, _VP, _VP]),
}
EXPORTED = sorted(_SIGS)


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot pass {type(x)} as a pointer")


class Lib:
    """The loaded library: raw C functions as attributes plus tensor-level helpers."""

    def __init__(self, path: str = LIB_PATH):
        if not os.path.exists(path):
            raise RuntimeError(f"libancka.so not found at {path}: build it with `python -m paper_2408_05459_amd.build`")
        self.path = path
        # torch first: its HIP runtime then serves this library too (the library's own reference
        # to the runtime resolves to the copy already loaded), so streams and device memory
        # handed over by torch belong to the runtime the library calls.  Loaded the other way
        # round, the process ends up with two runtimes and context creation fails.
        import torch  # noqa: F401
        self.cdll = C.CDLL(path)
        for name, (res, args) in _SIGS.items():
            f = getattr(self.cdll, name)
            f.restype = res
            f.argtypes = args
            setattr(self, name, f)
        self._ctx = {}

    # ---------------------------------------------------------------- context
    def context(self, device: int = 0):
        import torch
        stream = torch.cuda.current_stream(device).cuda_stream
        key = (device, stream)
        if key not in self._ctx:
            h = _VP()
            st = self.ancka_create(C.byref(h), device, _VP(stream))
            if st != ANCKA_OK:
                raise AnckaError(st, "ancka_create failed")
            self._ctx[key] = h
        return self._ctx[key]

    def check(self, ctx, st):
        if st != ANCKA_OK:
            raise AnckaError(st, self.ancka_last_error(ctx).decode())

    # ---------------------------------------------------------------- marshalling helpers
    @staticmethod
    def dtype_code(t) -> int:
        import torch
        return {torch.float64: ANCKA_F64, torch.float32: ANCKA_F32, torch.bfloat16: ANCKA_BF16}[t.dtype]

    def network(self, net, device="cuda"):
        """Upload a synth.Network (numpy arrays) and fill ancka_network.  Returns (struct, keep)."""
        import torch
        keep = []
        s = ancka_network()
        s.kind = net.kind
        s.L = net.L
        s.n = net.n
        s.m = net.m
        for l in range(net.L):
            p = torch.from_numpy(np.ascontiguousarray(net.ptrs[l], dtype=np.int64)).to(device)
            i = torch.from_numpy(np.ascontiguousarray(net.idxs[l], dtype=np.int32)).to(device)
            keep += [p, i]
            s.ptr[l] = p.data_ptr()
            s.idx[l] = i.data_ptr()
            s.nnz[l] = int(net.ptrs[l][-1])
        X = upload_attributes(net.X, net.x_dtype, device)
        keep.append(X)
        s.X = X.data_ptr()
        s.xdtype = DTYPE_CODE[net.x_dtype]
        s.d = X.shape[1]
        s.ldx = X.stride(0)
        return s, keep

    # ---------------------------------------------------------------- tensor-level calls
    def knn(self, X, K: int, mode: str, device=0):
        import torch
        ctx = self.context(device)
        n, d = X.shape
        idx = torch.empty((n, K), dtype=torch.int32, device=X.device)
        sim = torch.empty((n, K), dtype=torch.float64 if mode == "f64" else torch.float32, device=X.device)
        stats = ancka_knn_stats()
        self.check(ctx, self.ancka_knn(ctx, _ptr(X), self.dtype_code(X), n, d, X.stride(0), K, KNN_MODE[mode],
                                       _ptr(idx), _ptr(sim), C.byref(stats)))
        return idx, sim, stats

    def knn_ivf(self, X, K: int, nlist: int, nprobe: int, device=0):
        """Approximate KNN lists (IVF coarse quantiser, BF16 tiles, FP64 rescoring) of bf16 X."""
        import torch
        ctx = self.context(device)
        n, d = X.shape
        idx = torch.empty((n, K), dtype=torch.int32, device=X.device)
        sim = torch.empty((n, K), dtype=torch.float32, device=X.device)
        stats = ancka_knn_stats()
        self.check(ctx, self.ancka_knn_ivf(ctx, _ptr(X), self.dtype_code(X), n, d, X.stride(0), K, nlist, nprobe,
                                           _ptr(idx), _ptr(sim), C.byref(stats)))
        return idx, sim, stats

    def build_operator(self, net_struct, nbr_idx, nbr_sim, K: int, beta: float, op_dtype: str, device=0):
        ctx = self.context(device)
        h = _VP()
        self.check(ctx, self.ancka_build_operator(ctx, C.byref(net_struct), _ptr(nbr_idx), _ptr(nbr_sim),
                                                  self.dtype_code(nbr_sim), K, beta, DTYPE_CODE[op_dtype], C.byref(h)))
        return Op(self, h, net_struct.n, op_dtype)

    def discretize(self, Q, k: int, max_iter: int = 30, device=0, noalloc: bool = False):
        """Q: n x (>= k) tensor view whose first k columns are the block to discretize.
        noalloc: call ancka_discretize_noalloc (state in the library's static device array)."""
        import torch
        ctx = self.context(device)
        n = Q.shape[0]
        labels = torch.empty(n, dtype=torch.int32, device=Q.device)
        R = np.zeros((k, k))
        obj = C.c_double()
        it = C.c_int32()
        fn = self.ancka_discretize_noalloc if noalloc else self.ancka_discretize
        self.check(ctx, fn(ctx, _ptr(Q), self.dtype_code(Q), n, k, Q.stride(0), max_iter,
                           _ptr(labels), R.ctypes.data, C.addressof(obj), C.addressof(it)))
        return labels, R, obj.value, it.value

    def ws_features(self, op, X, device=0):
        """U = (X^ + P_N X^) / 2 as a float n x ldu tensor (ldu = d rounded up to 4)."""
        import torch
        ctx = self.context(device)
        n, d = X.shape
        ldu = (d + 3) // 4 * 4
        U = torch.empty((n, ldu), dtype=torch.float32, device=X.device)
        self.check(ctx, self.ancka_ws_features(ctx, op.h, _ptr(X), self.dtype_code(X), d, X.stride(0), _ptr(U), ldu))
        return U

    def ws_target(self, Qk, k: int, R, colmap, device=0):
        """Training target from the n x k view Qk (columns 1..k of the iteration block)."""
        import torch
        ctx = self.context(device)
        n = Qk.shape[0]
        T = torch.empty((n, k), dtype=torch.float32, device=Qk.device)
        R = np.ascontiguousarray(R, dtype=np.float64)
        cm = np.ascontiguousarray(colmap, dtype=np.int32)
        self.check(ctx, self.ancka_ws_target(ctx, _ptr(Qk), self.dtype_code(Qk), n, k, Qk.stride(0), R.ctypes.data,
                                             cm.ctypes.data, _ptr(T)))
        return T

    def default_params(self, **kw):
        p = self.ancka_default_params()
        for k_, v in kw.items():
            if k_ == "knn_mode" and isinstance(v, str):
                v = KNN_MODE[v]
            if k_ == "q_dtype" and isinstance(v, str):
                v = DTYPE_CODE[v]
            setattr(p, k_, v)
        return p

    def cluster(self, net_struct, params, zwarm=None, trace_capacity=1024, device=0, op=None):
        """Whole method on a network (or, with op, from a built operator).  Returns (labels, info)."""
        import torch
        ctx = self.context(device)
        n = op.n if op is not None else net_struct.n
        labels = torch.empty(n, dtype=torch.int32, device="cuda")
        rep = ancka_report()
        tt = (C.c_int32 * trace_capacity)()
        tp = (C.c_double * trace_capacity)()
        rep.trace_capacity = trace_capacity
        rep.trace_t = C.cast(tt, C.POINTER(C.c_int32))
        rep.trace_phi = C.cast(tp, C.POINTER(C.c_double))
        if op is not None:
            self.check(ctx, self.ancka_cluster_op(ctx, op.h, C.byref(params), _ptr(zwarm), _ptr(labels),
                                                  C.byref(rep)))
        else:
            self.check(ctx, self.ancka_cluster(ctx, C.byref(net_struct), C.byref(params), _ptr(zwarm),
                                               _ptr(labels), C.byref(rep)))
        m = min(rep.trace_len, trace_capacity)
        info = {
            "iterations": rep.iterations, "stop_reason": STOP_REASONS[rep.stop_reason], "best_phi": rep.best_phi,
            "best_t": rep.best_t, "init_used": "warm" if rep.init_used else "cold",
            "phi_init_cold": rep.phi_init_cold, "phi_init_warm": rep.phi_init_warm,
            "trace": [(tt[i], tp[i]) for i in range(m)],
            "phase_ms": {PHASES[i]: rep.phase_ms[i] for i in range(ANCKA_NPHASES)},
            "knn_zero_rows": rep.knn.zero_rows, "knn_uncertified_rows": rep.knn.uncertified_rows,
            "knn_tile_ms": rep.knn.tile_ms, "knn_total_ms": rep.knn.total_ms,
            "knn_sym_ms": rep.knn.sym_ms, "knn_sym_pairs": rep.knn.sym_pairs,
            "knn_handed_over": rep.knn.handed_over, "knn_window": rep.knn.window,
            "knn_rescanned": rep.knn.rescanned,
            "disc_iters_total": rep.disc_iters_total,
        }
        return labels, info


class Op:
    """Owning handle of an ancka_op."""

    def __init__(self, lib: Lib, handle, n: int, dtype: str):
        self.lib, self.h, self.n, self.dtype = lib, handle, n, dtype

    def __del__(self):
        try:
            if self.h:
                self.lib.ancka_op_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def info(self, device=0):
        ctx = self.lib.context(device)
        beta = np.zeros(self.n)
        delta = np.zeros(self.n, dtype=np.int64)
        dk = np.zeros(self.n)
        nk = C.c_int64()
        nt = C.c_int64()
        self.lib.check(ctx, self.lib.ancka_op_info(ctx, self.h, beta.ctypes.data, delta.ctypes.data, dk.ctypes.data,
                                                   C.byref(nk), C.byref(nt)))
        return {"beta": beta, "delta": delta, "dk": dk, "nnz_knn": nk.value, "nnz_topo": nt.value}

    def apply(self, Q, device=0):
        import torch
        ctx = self.lib.context(device)
        Z = torch.empty_like(Q)
        self.lib.check(ctx, self.lib.ancka_apply_p(ctx, self.h, _ptr(Q), _ptr(Z), Q.shape[1], Q.stride(0)))
        return Z

    def apply_bf16(self, Qb, device=0):
        """Z = P Q for a bf16 block Q (float Z of the same shape)."""
        import torch
        ctx = self.lib.context(device)
        Z = torch.empty(Qb.shape, dtype=torch.float32, device=Qb.device)
        self.lib.check(ctx, self.lib.ancka_apply_p_bf16(ctx, self.h, _ptr(Qb), _ptr(Z), Qb.shape[1], Qb.stride(0)))
        return Z

    def init_bcm(self, k: int, alpha: float, T_i: int, device=0):
        import torch
        ctx = self.lib.context(device)
        labels = torch.empty(self.n, dtype=torch.int32, device="cuda")
        self.lib.check(ctx, self.lib.ancka_init_bcm(ctx, self.h, k, alpha, T_i, _ptr(labels)))
        return labels

    def initial_block(self, k: int, labels=None, zwarm=None, ldq=None, device=0):
        import torch
        ctx = self.lib.context(device)
        vw = 2 if self.dtype == "f64" else 4
        ldq = ldq or (k + 1 + vw - 1) // vw * vw
        Q = torch.zeros((self.n, ldq), dtype=torch.float64 if self.dtype == "f64" else torch.float32, device="cuda")
        self.lib.check(ctx, self.lib.ancka_initial_block(ctx, self.h, _ptr(labels), _ptr(zwarm), k, _ptr(Q), ldq))
        return Q

    def orth_iter(self, Q, kp1: int, iters: int, device=0):
        ctx = self.lib.context(device)
        R = np.zeros((kp1, kp1))
        dq = C.c_double()
        self.lib.check(ctx, self.lib.ancka_orth_iter(ctx, self.h, _ptr(Q), Q.stride(0), kp1, iters, R.ctypes.data,
                                                     C.addressof(dq)))
        return R, dq.value

    def mhc(self, labels, k: int, alpha: float, gamma: int, device=0) -> float:
        ctx = self.lib.context(device)
        phi = C.c_double()
        self.lib.check(ctx, self.lib.ancka_mhc(ctx, self.h, _ptr(labels), k, alpha, gamma, C.byref(phi)))
        return phi.value


class WarmStart:
    """Owning handle of an ancka_ws model (MLP d -> h1 -> h2 -> k)."""

    def __init__(self, lib: Lib, d: int, h1: int, h2: int, k: int, seed: int = 0, device=0):
        self.lib, self.d, self.h1, self.h2, self.k, self.device = lib, d, h1, h2, k, device
        ctx = lib.context(device)
        h = _VP()
        lib.check(ctx, lib.ancka_ws_create(ctx, d, h1, h2, k, seed, C.byref(h)))
        self.h = h
        cnt = C.c_int64()
        lib.check(ctx, lib.ancka_ws_get_params(ctx, h, 2, None, C.byref(cnt)))
        self.count = cnt.value

    def __del__(self):
        try:
            if self.h:
                self.lib.ancka_ws_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def shapes(self):
        return [(self.d, self.h1), (self.h1,), (self.h1, self.h2), (self.h2,), (self.h2, self.k), (self.k,)]

    def get(self, which: int = 2):
        """Parameters as a list [W1, b1, W2, b2, W3, b3] of float32 arrays (which: 0 forward
        values, 1 gradients, 2 master weights)."""
        ctx = self.lib.context(self.device)
        flat = np.zeros(self.count, dtype=np.float32)
        cnt = C.c_int64()
        self.lib.check(ctx, self.lib.ancka_ws_get_params(ctx, self.h, which, flat.ctypes.data, C.byref(cnt)))
        out, o = [], 0
        for sh in self.shapes():
            sz = int(np.prod(sh))
            out.append(flat[o:o + sz].reshape(sh).copy())
            o += sz
        return out

    def set(self, params):
        ctx = self.lib.context(self.device)
        flat = np.ascontiguousarray(np.concatenate([np.asarray(p, np.float32).ravel() for p in params]))
        if flat.size != self.count:
            raise ValueError(f"expected {self.count} parameters, got {flat.size}")
        self.lib.check(ctx, self.lib.ancka_ws_set_params(ctx, self.h, flat.ctypes.data))

    def forward(self, U, n=None, keep_acts=False):
        import torch
        ctx = self.lib.context(self.device)
        n = U.shape[0] if n is None else n
        Z = torch.empty((n, self.k), dtype=torch.float32, device=U.device)
        self.lib.check(ctx, self.lib.ancka_ws_forward(ctx, self.h, _ptr(U), n, U.stride(0), _ptr(Z),
                                                      1 if keep_acts else 0))
        return Z

    def backward(self, Z, T, want_loss=True):
        ctx = self.lib.context(self.device)
        loss = C.c_double()
        self.lib.check(ctx, self.lib.ancka_ws_backward(ctx, self.h, _ptr(Z), _ptr(T), Z.shape[0],
                                                       C.addressof(loss) if want_loss else None))
        return loss.value if want_loss else None

    def step(self, lr: float):
        ctx = self.lib.context(self.device)
        self.lib.check(ctx, self.lib.ancka_ws_step(ctx, self.h, lr))


def upload_attributes(X: np.ndarray, x_dtype: str, device="cuda"):
    import torch
    if x_dtype == "f64":
        return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float64)).to(device)
    if x_dtype == "f32":
        return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(device)
    # values are already bf16-representable float32: the conversion is exact
    return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(device).to(torch.bfloat16)


_LIB: Optional[Lib] = None


def load(path: str = LIB_PATH) -> Lib:
    global _LIB
    if _LIB is None:
        _LIB = Lib(path)
    return _LIB
