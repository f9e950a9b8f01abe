/*
 * ancka.h -- C ABI of the MI355X (gfx950) library for KNN-augmented attributed-network
 * clustering (the ANCKA method: KNN augmentation, (alpha,beta,gamma)-random-walk
 * orthogonal iteration, Discretize, multi-hop conductance).
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Array arguments are DEVICE pointers owned by the caller (contiguous, row-major),
 *    unless a comment says "host".  k x k matrices and scalar results are host pointers.
 *  - All work is enqueued on the context's HIP stream.  Calls are asynchronous unless they
 *    return host values (those synchronise the stream before returning).
 *  - Node and hyperedge ids are int32 (n, m < 2^31); row pointers are int64.
 *  - Errors are returned as an ancka_status; nothing throws across the ABI.  A readable
 *    message of the last failure is available from ancka_last_error().  On any error the
 *    output arrays are unspecified.
 *  - Determinism: every reduction has a fixed order or is exact (integer / fixed point);
 *    two runs on the same inputs give bitwise-equal outputs.
 */
#ifndef ANCKA_H
#define ANCKA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ANCKA_OK = 0,
  ANCKA_ERR_INVALID_ARG = 1,   /* a size, pointer or parameter is outside its documented range */
  ANCKA_ERR_UNSUPPORTED = 2,   /* dtype / mode combination not provided */
  ANCKA_ERR_OOM = 3,           /* device allocation failed */
  ANCKA_ERR_HIP = 4,           /* a HIP runtime call failed */
  ANCKA_ERR_NUMERICAL = 5      /* a factorisation broke down after every fallback */
} ancka_status;

typedef enum { ANCKA_F64 = 0, ANCKA_F32 = 1, ANCKA_BF16 = 2 } ancka_dtype;

/* Network kinds of Sec. 2: attributed hypergraph, graph, multiplex graph. */
typedef enum { ANCKA_HYPERGRAPH = 0, ANCKA_GRAPH = 1, ANCKA_MULTIPLEX = 2 } ancka_kind;

/* KNN arithmetic.  EXACT_F64: FP64 tiles, top-K directly (similarities in double).
 * EXACT_F32: FP32 tiles, top-2K candidates, FP64 rescoring, certificate, exact recompute of
 * uncertified rows.  BF16_RESCORE: BF16 MFMA tiles with FP32 accumulation, then as EXACT_F32.
 * Both non-F64 modes return similarities in float. */
typedef enum { ANCKA_KNN_EXACT_F64 = 0, ANCKA_KNN_EXACT_F32 = 1, ANCKA_KNN_BF16_RESCORE = 2,
               ANCKA_KNN_IVF_BF16 = 3 /* approximate: ancka_knn_ivf (ancka_cluster only) */ } ancka_knn_mode;

#define ANCKA_MAX_LAYERS 16

typedef struct ancka_ctx ancka_ctx;
typedef struct ancka_op ancka_op;

/* Attributed network N = (V, E, X) (Sec. 2).
 *  hypergraph: L = 1, ptr[0] has m+1 entries, idx[0] lists the members of each hyperedge
 *              (repeated members are merged; an empty hyperedge is an error);
 *  graph:      L = 1, ptr[0] has n+1 entries (CSR of A; a directed input is symmetrised by
 *              adding the reverse of every edge, duplicates and self loops are dropped);
 *  multiplex:  L layers, each a CSR as for a graph.
 *  nnz[l] = ptr[l][last] (given so that no device read is needed).
 *  X: n x d attributes with leading dimension ldx, element type xdtype. */
typedef struct {
  int32_t kind;
  int32_t L;
  int64_t n;
  int64_t m;
  const int64_t* ptr[ANCKA_MAX_LAYERS];
  const int32_t* idx[ANCKA_MAX_LAYERS];
  int64_t nnz[ANCKA_MAX_LAYERS];
  const void* X;
  int32_t xdtype;
  int64_t d;
  int64_t ldx;
} ancka_network;

/* Method parameters; defaults (ancka_default_params) are the paper's experimental
 * settings of Sec. 8.1: alpha 0.2, beta 0.5, gamma 3, K 10, eps_Q 0.005, T_a 1000,
 * T_i 25, tau 5.  disc_max_iter bounds the Discretize loop of Alg. 5.  k, the number of
 * clusters of the problem statement (Sec. 2), has no default (0) and must be set. */
typedef struct {
  int32_t k;
  int32_t K;
  double alpha;
  double beta;
  int32_t gamma;
  int32_t tau;
  int32_t T_i;
  int32_t T_a;
  double eps_q;
  int32_t disc_max_iter;
  int32_t knn_mode;      /* ancka_knn_mode */
  int32_t q_dtype;       /* ANCKA_F32 or ANCKA_F64: precision of the iterated block */
  int32_t early_stop;    /* 1: apply Eqs. (tcond-1) and (tcond-2); 0: run exactly T_a iterations */
  int32_t ivf_nlist;     /* knn_mode IVF_BF16: lists of the coarse quantiser (default 1024) */
  int32_t ivf_nprobe;    /* knn_mode IVF_BF16: lists each query block scans (default 32) */
} ancka_params;

typedef struct {
  int64_t zero_rows;         /* attribute rows that are all zero */
  int64_t uncertified_rows;  /* rows whose 2K candidate list could not prove the top-K */
  int64_t recomputed_rows;   /* rows recomputed exactly (= uncertified_rows) */
  double tile_ms;            /* duration of the similarity-tile + top-K phase (HIP events on the stream);
                                for BF16_RESCORE: window pass, symmetric pass and list merge */
  double total_ms;           /* duration of the whole ancka_knn call on the stream */
  double sym_ms;             /* BF16_RESCORE: duration of the symmetric-pass kernel (0 if not run) */
  int64_t sym_pairs;         /* unordered row pairs the symmetric pass scores (padding rows included) */
  int64_t handed_over;       /* candidate pairs the symmetric pass handed to other rows' lists */
  int32_t window;            /* half-width, in blocks of rows, of the window pass; -1: whole scan */
  int32_t rescanned;         /* 1 if the hand-over buffer overflowed and the scan was redone whole */
} ancka_knn_stats;

enum { ANCKA_PHASE_KNN = 0, ANCKA_PHASE_OPERATOR = 1, ANCKA_PHASE_INIT = 2, ANCKA_PHASE_ITER = 3,
       ANCKA_PHASE_DISCRETIZE = 4, ANCKA_PHASE_MHC = 5, ANCKA_PHASE_WARM = 6, ANCKA_NPHASES = 7 };

enum { ANCKA_STOP_MAX_ITER = 0, ANCKA_STOP_CONVERGED = 1, ANCKA_STOP_EARLY = 2 };

typedef struct {
  int32_t iterations;        /* orthogonal iterations performed */
  int32_t stop_reason;       /* ANCKA_STOP_* */
  double best_phi;           /* MHC of the returned labels */
  int32_t best_t;            /* iteration that produced them (0 = initial BCM) */
  int32_t init_used;         /* 0 cold (greedy InitBCM), 1 learned warm start */
  double phi_init_cold;
  double phi_init_warm;      /* NaN when no warm block was given */
  /* phi trace: (t, phi_t) for t = 0, tau, 2 tau, ...; caller-owned host arrays */
  int32_t trace_capacity;
  int32_t trace_len;
  int32_t* trace_t;
  double* trace_phi;
  double phase_ms[ANCKA_NPHASES];
  ancka_knn_stats knn;
  int32_t disc_iters_total;
} ancka_report;

/* ---- context ------------------------------------------------------------------------- */

/* Create a context bound to HIP device `device` and stream `hip_stream` (a hipStream_t;
 * NULL means the device's null stream).  One context per host thread. */
ancka_status ancka_create(ancka_ctx** out, int32_t device, void* hip_stream);
void ancka_destroy(ancka_ctx* ctx);
const char* ancka_last_error(const ancka_ctx* ctx);
ancka_params ancka_default_params(void);
/* Number of compute units / XCD count seen by the context (host). */
ancka_status ancka_device_info(ancka_ctx* ctx, int32_t* num_cu, int32_t* warp_size);

/* ---- KNN graph (Sec. 3.1 KNN augmentation; Alg. 6, neighbour search) ------------------------------
 * For every row i of X (n x d, leading dimension ldx, element type xdtype), the K rows j != i
 * with the largest cosine similarity f(i, j) = x_i.x_j / (|x_i| |x_j|), ordered by
 * (f desc, j asc).  A zero row is never a candidate; its own list is idx -1, sim 0.  Rows
 * with fewer than K candidates are padded the same way.
 *  nbr_idx: int32 n x K (device, caller-owned).
 *  nbr_sim: n x K, double for EXACT_F64, float otherwise (device, caller-owned).
 *  stats:   host, nullable; filling it synchronises the stream.
 * Errors: INVALID_ARG unless n >= 2, d >= 1, ldx >= d and 1 <= K <= min(n-1, 64) (the candidate
 * modes keep 2K <= 128 candidates per row); UNSUPPORTED for BF16_RESCORE with a non-bf16 X or
 * d > 512. */
ancka_status ancka_knn(ancka_ctx* ctx, const void* X, int32_t xdtype, int64_t n, int64_t d,
                       int64_t ldx, int32_t K, int32_t mode, int32_t* nbr_idx, void* nbr_sim,
                       ancka_knn_stats* stats);

/* ---- approximate KNN graph: IVF coarse quantiser + exact rescoring (Alg. 6, the approximate
 * index the paper uses beyond 100k nodes; Sec. 7, KNN construction) ---------------------------
 * For n beyond the exact n^2 budget.  Coarse quantiser: nlist pivot rows (pivot c is the first
 * non-zero row at or after row c n / nlist); each row belongs to the list of its most similar
 * pivot.  Rows are grouped by list; each block of consecutive rows of a list scans, with BF16
 * MFMA tiles, the rows of its own list(s) and of the nprobe - 1 lists whose pivots are most
 * similar to its list's pivot, keeping the top 2K candidates per row by score; the candidates are
 * rescored in FP64 and the top K returned by (cosine desc, index asc).  Returned similarities are
 * exact FP64 cosines (rounded to float); the neighbour sets are approximate (a true neighbour in
 * an unprobed list is missed).  nprobe = nlist scans every row, as the exact search does.
 * X: bf16 n x d (ldx >= d), d <= 512.  nbr_idx: int32 n x K; nbr_sim: float n x K (device,
 * caller-owned).  stats: host, nullable (uncertified_rows counts rows whose 2K list could not
 * certify its top K among the scanned candidates; nothing is recomputed; sym_pairs = ordered
 * pairs scored).  Synchronises the stream.
 * Errors: INVALID_ARG unless 1 <= K <= min(n-1, 64), 1 <= nlist <= min(n, 4096) and
 * 1 <= nprobe <= min(nlist, 64); UNSUPPORTED for non-bf16 X or d > 512. */
ancka_status ancka_knn_ivf(ancka_ctx* ctx, const void* X, int32_t xdtype, int64_t n, int64_t d, int64_t ldx,
                           int32_t K, int32_t nlist, int32_t nprobe, int32_t* nbr_idx, void* nbr_sim,
                           ancka_knn_stats* stats);

/* ---- operator P = (I - B) P_N + B P_K (Eqs. AK, beta_i, p-mat-ancka, rw-hg/ag/mg) -------
 * Builds, on the device, every structure the walk needs without forming P:
 *  A_K = W + W^T with W[i,j] = f(i,j) for j in N_K(i) (mutual pairs 2f); neighbours with
 *  f <= 0 are dropped; D_K = A_K 1; P_K = D_K^-1 A_K.
 *  beta_i = 0 if D_K[i] = 0 (a zero attribute row has no KNN edge), else 1 if the node has
 *  no topology edge, else beta.  A node with beta_i = 0 and no topology edge gets P[i,i] = 1.
 *  Multiplex rows average over the layers where the node has edges.
 * nbr_idx / nbr_sim: as produced by ancka_knn (sim_dtype ANCKA_F64 or ANCKA_F32).
 * op_dtype: ANCKA_F64 or ANCKA_F32, the precision of the operator values and of every block
 * later multiplied with it.  The op owns copies of everything; the inputs may be freed after
 * the call returns (it synchronises the stream).
 * Errors: INVALID_ARG for n < 2, L outside [1, ANCKA_MAX_LAYERS], an out-of-range index or
 * an empty hyperedge (detected on the device, reported after the sync). */
ancka_status ancka_build_operator(ancka_ctx* ctx, const ancka_network* net, const int32_t* nbr_idx,
                                  const void* nbr_sim, int32_t sim_dtype, int32_t K, double beta,
                                  int32_t op_dtype, ancka_op** out);
void ancka_op_destroy(ancka_op* op);
/* Host copies of per-node operator data (for inspection; nullable outputs, host arrays of n):
 * beta_i, delta(v_i) (hypergraph degree / graph degree / summed multiplex degree), D_K[i]. */
ancka_status ancka_op_info(ancka_ctx* ctx, const ancka_op* op, double* beta, int64_t* delta,
                           double* dk, int64_t* nnz_knn, int64_t* nnz_topo);

/* ---- Z = P Q (Eq. zt, Eq. p-mat-ancka) ----------------------------------------------------
 * One application of P to an n x cols block.  Q, Z: op_dtype, leading dimension ld (>= cols).
 * Errors: INVALID_ARG if cols < 1, ld < cols or cols > 64. */
ancka_status ancka_apply_p(ancka_ctx* ctx, const ancka_op* op, const void* Q, void* Z, int32_t cols,
                           int64_t ld);

/* The same product with the block Q stored in BF16 (half the bytes of every gathered row; the
 * values are widened exactly and accumulated in FP32 as ancka_apply_p does): Q bf16 n x ld,
 * Z float n x ld.  For graph and multiplex operators of FP32 values.  Measured against the FP32
 * product on the same operator; the method itself keeps FP32 blocks (BF16 storage moves the
 * iterated subspace by more than the 1e-4 principal-angle tolerance of the path).
 * Errors: INVALID_ARG if cols < 1, cols > 64, ld < cols or ld % 4 != 0; UNSUPPORTED for a
 * hypergraph or FP64 operator. */
ancka_status ancka_apply_p_bf16(ancka_ctx* ctx, const ancka_op* op, const void* Q, float* Z, int32_t cols,
                                int64_t ld);

/* ---- greedy initial BCM (Alg. 3; Alg. 4, greedy start; Eqs. pi_c_t, argmaxlabel) ---------------
 * V_c = the k nodes of largest degree (ties: smaller index) listed by index; T_i steps of
 * Pi <- (1-alpha) Pi P_N + alpha Z_0 on the topology walk only; label of v_j = argmax_l
 * Pi[l, j], smallest l on ties.  labels: int32 n (device).
 * Errors: INVALID_ARG unless 1 <= k <= min(n, 64), 0 <= alpha <= 1, T_i >= 0. */
ancka_status ancka_init_bcm(ancka_ctx* ctx, const ancka_op* op, int32_t k, double alpha, int32_t T_i,
                            int32_t* labels);

/* ---- starting block (Alg. 4, starting block) ---------------------------------------------------
 * Q (n x (k+1), leading dimension ldq, op's dtype) = orthonormalised [1/sqrt(n) 1 | h(Y)]
 * with h(Y) of Eq. (norm-y) built from `labels`, or [1/sqrt(n) 1 | Zwarm] when `labels` is
 * NULL and `zwarm` (float n x k, leading dimension k) is given.  The block is orthonormalised
 * column by column (a Gram-Schmidt QR with positive diagonal); a zero column, and the column of
 * the last non-empty cluster (which the constant vector makes dependent), are replaced by
 * cos(pi (i + 1/2) j / n) for column j first. */
ancka_status ancka_initial_block(ancka_ctx* ctx, const ancka_op* op, const int32_t* labels,
                                 const float* zwarm, int32_t k, void* Q, int64_t ldq);

/* ---- orthogonal iteration (Eq. ortho-iter) --------------------------------------------------
 * `iters` times: Z = P Q, Q R = Z with diag(R) > 0 (Cholesky QR with an FP64 Gram and FP64
 * Cholesky; a second pass when the first is ill-conditioned or the block is FP64).
 * Q: op's dtype, n x kp1, leading dimension ldq, in/out.
 * R_last: host kp1 x kp1 (row-major, upper triangular) of the last step, nullable.
 * dq_fro: host, nullable: ||Q^(t) - Q^(t-1)||_F of the last step.
 * Errors: INVALID_ARG unless 2 <= kp1 <= 64 and ldq >= kp1; NUMERICAL if the Cholesky
 * factorisation breaks down even after a diagonal shift. */
ancka_status ancka_orth_iter(ancka_ctx* ctx, const ancka_op* op, void* Q, int64_t ldq, int32_t kp1,
                             int32_t iters, double* R_last, double* dq_fro);

/* ---- Discretize (Sec. 7: Definition 2, Eqs. updateY, svd-in-discr, Alg. 5) -------------------
 * Q: n x k block (dtype qdtype, leading dimension ldq): pass a pointer to column 1 of the
 * orthogonal-iteration block to drop the constant eigenvector.  Rows are normalised (zero
 * rows stay zero); R starts at I_k; each step: labels = row argmax of Q~ R (smallest column on
 * ties), Y~ = Y with columns divided by their sums, U Omega V^T = SVD(Y~^T Q~), R = V U^T,
 * obj = n - 2 trace(Omega); stops when |obj - obj_prev| <= 1e-12 max(1, |obj|) or after
 * max_iter steps.  labels: int32 n (device); R: host k x k row-major, nullable; obj, iters: host,
 * nullable.  Synchronises the stream.  The cluster sums are exact fixed-point integers (scale
 * 2^40, or 2^(62 - ceil(log2 n)) when n > 2^22), so they do not depend on the order of rows.
 * Errors: INVALID_ARG unless 1 <= k <= 64, 1 <= n < 2^31, ldq >= k, max_iter >= 1 and qdtype is
 * F32 or F64. */
ancka_status ancka_discretize(ancka_ctx* ctx, const void* Q, int32_t qdtype, int64_t n, int32_t k,
                              int64_t ldq, int32_t max_iter, int32_t* labels, double* R, double* obj,
                              int32_t* iters);

/* ---- Discretize without device allocation ---------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, serving loops
 * that must not call hipMalloc, harnesses that forbid it): the same computation, arguments,
 * results and errors as ancka_discretize, with its k x k state (R, the cluster sums and counts,
 * the loop state; at most 98,816 bytes) in a static device array of the library instead of a
 * context workspace.  Each GPU holds one copy of that array from ancka_create on that GPU until
 * the process ends, and every call on that GPU uses it: calls that overlap on one GPU (from any
 * context or stream) race and must be serialised by the caller.  The call clears the state it
 * needs at its start, so the contents a previous call left do not matter.  It allocates
 * nothing on the device.  Limits as ancka_discretize: 1 <= k <= 64, 1 <= n < 2^31 (no limit
 * from the state size, which does not depend on n).  Synchronises the stream. */
ancka_status ancka_discretize_noalloc(ancka_ctx* ctx, const void* Q, int32_t qdtype, int64_t n, int32_t k,
                                      int64_t ldq, int32_t max_iter, int32_t* labels, double* R, double* obj,
                                      int32_t* iters);

/* ---- multi-hop conductance (Alg. 2; Eq. mhc-comp-ancka) -------------------------------------
 * phi = 1 - (1/k) trace(Yh^T F^(gamma)), F^(0) = alpha Yh, F^(l) = (1-alpha) P F^(l-1) + F^(0),
 * Yh = h(Y) from `labels` (device int32 n, values in [0,k)).  phi: host.  Synchronises. */
ancka_status ancka_mhc(ancka_ctx* ctx, const ancka_op* op, const int32_t* labels, int32_t k,
                       double alpha, int32_t gamma, double* phi);

/* ---- whole method (Alg. 4 with Alg. 6 for the KNN graph) -------------------------------------
 * KNN graph, operator, greedy initial BCM (or the learned warm start `zwarm`, float n x k,
 * nullable; used when its labels have an MHC no larger than the greedy ones), then the
 * orthogonal iteration with Discretize and MHC every tau iterations, keeping the labels of
 * lowest MHC; stops on Eq. (tcond-1) or (tcond-2) (if params->early_stop) or after T_a.
 * labels: int32 n (device).  rep: host, nullable.  Synchronises the stream. */
ancka_status ancka_cluster(ancka_ctx* ctx, const ancka_network* net, const ancka_params* params,
                           const float* zwarm, int32_t* labels, ancka_report* rep);

/* The same method from an operator built by ancka_build_operator (Alg. 4 from the greedy start
 * on): callers that already hold the operator, e.g. to aggregate the warm-start features with
 * its walk, skip the second KNN search.  params->q_dtype must equal the operator's dtype and
 * params->K is not used.  The report's KNN and operator phases stay zero.  Synchronises.
 * Errors: as ancka_cluster. */
ancka_status ancka_cluster_op(ancka_ctx* ctx, const ancka_op* op, const ancka_params* params,
                              const float* zwarm, int32_t* labels, ancka_report* rep);

/* ---- learned warm start (not part of the paper) -------------------------------------------
 * A three-layer perceptron d_in -> h1 -> h2 -> k that predicts, for every node, its row of the
 * plain method's rotated eigenblock from its one-hop aggregated attributes; its argmax rows and
 * the block [1/sqrt(n) | Zhat] replace the greedy start of Alg. 4 (see ancka_cluster's zwarm).
 * Every matrix product takes BF16 operands (FP32 values rounded to nearest even) and
 * accumulates in FP32: the input U, the weights and both hidden activations are rounded, the
 * biases, the FP32 master weights and the Adam state are not.  Weights are laid out (in, out),
 * row-major; H1 = relu(U W1 + b1), H2 = relu(H1 W2 + b2), Zhat = H2 W3 + b3.
 * A model belongs to the device of the context that created it; calls on one model must not
 * overlap. */
typedef struct ancka_ws ancka_ws;

/* Create a model: weights uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) drawn in order W1, W2, W3
 * from the SplitMix64 stream of `seed` (53-bit uniforms), biases zero, Adam state zero.
 * Errors: INVALID_ARG unless 1 <= d_in <= 4096, 16 <= h1, h2 <= 1024 (multiples of 16) and
 * 1 <= k <= 64; OOM. */
ancka_status ancka_ws_create(ancka_ctx* ctx, int32_t d_in, int32_t h1, int32_t h2, int32_t k,
                             uint64_t seed, ancka_ws** out);
void ancka_ws_destroy(ancka_ws* ws);

/* Input features U = (X^ + P_N X^) / 2 of every node of the operator's network, X^ the rows of
 * X scaled to unit L2 norm (zero rows stay zero) and P_N the operator's topology walk (hypergraph
 * P_V P_E, graph D^-1 A, multiplex average over the layers where the node has edges; an isolated
 * node keeps U = X^ / 2).  X: device n x d, leading dimension ldx, xdtype F64 / F32 / BF16.
 * U: device float n x ldu (caller-owned; columns d..ldu-1 are left untouched).
 * Errors: INVALID_ARG unless d >= 1, ldx >= d, ldu >= d and ldu % 4 == 0. */
ancka_status ancka_ws_features(ancka_ctx* ctx, const ancka_op* op, const void* X, int32_t xdtype,
                               int64_t d, int64_t ldx, float* U, int64_t ldu);

/* Zhat = MLP(U).  U: device float n x ldu (the first d_in columns are read); zhat: device float
 * n x k, contiguous.  keep_acts = 1 keeps the rounded input and activations inside ws for
 * ancka_ws_backward (workspace grows to n rows).  Errors: INVALID_ARG unless n >= 1, ldu >= d_in. */
ancka_status ancka_ws_forward(ancka_ctx* ctx, ancka_ws* ws, const float* U, int64_t n, int64_t ldu,
                              float* zhat, int32_t keep_acts);

/* Mean squared error loss = (1/n) sum_i ||zhat_i - T_i||^2 of the last forward with
 * keep_acts = 1 (same n), and its gradients with respect to every parameter, stored inside ws
 * (read them with ancka_ws_get_params(which = 1)).  The output gradient 2 (zhat - T) / n and
 * both hidden-layer gradients are rounded to BF16 before they enter a product; the relu
 * derivative is 1 where the stored activation is positive.  zhat, T: device float n x k.
 * loss: host, nullable (synchronises when given).
 * Errors: INVALID_ARG if no activations of n rows are kept. */
ancka_status ancka_ws_backward(ancka_ctx* ctx, ancka_ws* ws, const float* zhat, const float* T,
                               int64_t n, double* loss);

/* One Adam step (Kingma and Ba 2015: beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * FP32 master weights and biases with the stored gradients; the BF16 copies used by the
 * products are refreshed.  Errors: INVALID_ARG unless lr > 0. */
ancka_status ancka_ws_step(ancka_ctx* ctx, ancka_ws* ws, double lr);

/* Host copies of the parameters, packed W1 (d_in x h1), b1, W2 (h1 x h2), b2, W3 (h2 x k), b3 as
 * float.  which: 0 the values the forward pass uses (BF16-rounded weights, FP32 biases),
 * 1 the gradients of the last backward, 2 the FP32 master weights.  host nullable (then only
 * count is written); count: host, out, number of floats.  Synchronises.
 * ancka_ws_set_params writes the master weights from the same packing, refreshes the BF16
 * copies and clears the Adam state and step count. */
ancka_status ancka_ws_get_params(ancka_ctx* ctx, ancka_ws* ws, int32_t which, float* host, int64_t* count);
ancka_status ancka_ws_set_params(ancka_ctx* ctx, ancka_ws* ws, const float* host);

/* Training target from one run of the plain method: T[:, colmap[c]] = (Q~ R)[:, c], where Q~ are
 * the rows of the n x k block Q scaled to unit L2 norm (zero rows stay zero) and R the rotation
 * of its last Discretize (ancka_discretize's R, host double k x k row-major).  Q: device, qdtype
 * F32 / F64, leading dimension ldq (a pointer to column 1 of the orthogonal-iteration block);
 * colmap: host int32 k, a permutation of 0..k-1 (the cluster-to-centre assignment); T: device
 * float n x k.  Errors: INVALID_ARG unless 1 <= k <= 64, ldq >= k and colmap is a permutation. */
ancka_status ancka_ws_target(ancka_ctx* ctx, const void* Q, int32_t qdtype, int64_t n, int32_t k,
                             int64_t ldq, const double* R, const int32_t* colmap, float* T);

#ifdef __cplusplus
}
#endif

#endif /* ANCKA_H */
