"""FP64 CPU oracle of the KNN-augmented attributed-network clustering method.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never calls it and
shares no code, tables or helpers with it.

Every function follows a passage of the paper (cited by section, equation or
algorithm) in plain numpy/scipy FP64 code.  Where the paper is silent or
ambiguous, the reading taken is stated at the function.  Pins that tie each
function to something other than itself live in ``tests/test_oracle_*.py``.

Parity status per function:
  normalize_rows, knn                          pinned (brute force, Figure 1 example)
  knn_adjacency, topology_transition, betas    pinned (Eq. AK cases, walk semantics, stochasticity)
  apply_P / transition_dense                   pinned (walk semantics, dense matrix)
  init_bcm                                     pinned (closed-form RWR power series)
  initial_q                                    pinned (QR definition properties)
  qr_pos                                       pinned (QR definition properties)
  orth_iter                                    pinned (eigh of the symmetric similar matrix)
  discretize                                   pinned (planted rotation, polar factor)
  mhc                                          pinned (escape-probability definition, offset identity)
  cluster                                      pinned (scripted conductance and step norms fix the
                                               stop, its reason and the returned labels; planted inputs)
  mlp_*                                        pinned (central finite differences)
"""
from .ancka import *  # noqa: F401,F403
from .mlp import *    # noqa: F401,F403
