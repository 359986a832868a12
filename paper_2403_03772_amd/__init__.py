"""MI355X (gfx950) DirectLiNGAM causal-ordering library: Python binding.

Argument marshalling over the C ABI of ``liblingam_mi355x.so`` (declared in
``include/lingam.h``); every step of the search runs in the library's HIP
kernels.  PyTorch supplies device memory and the current HIP stream only.
There is no CPU fallback: importing :mod:`paper_2403_03772_amd.lib` fails when
the shared library has not been built.

Functions mirror the C entry points:

* :func:`causal_order` -- ``lingam_causal_order`` (DirectLiNGAM ordering,
  Section 2.2 / Algorithm 1 of AcceleratedLiNGAM).
* :func:`causal_order_noalloc` -- ``lingam_causal_order_noalloc`` (the same
  ordering with the workspace in the library's per-GPU scratch array: the
  call allocates nothing).
* :func:`residualize` -- ``lingam_residualize`` (least-squares removal of one
  variable's effect, Section 2.2).
* :func:`varlingam_fit` -- ``varlingam_fit`` (VAR least squares, ordering of
  the residuals, instantaneous matrix B0; Section 3.2).
* :func:`adjacency` -- ``lingam_adjacency`` (least squares of every
  variable on its order predecessors: the weighted adjacency matrix).
* :func:`adjacency_pruned` -- ``lingam_adjacency_pruned`` (the adjacency
  pruned by the adaptive lasso).
* :func:`bootstrap`, :func:`bootstrap_accumulate` -- bootstrap order and
  edge probabilities (batched orderings of resamples, their adjacencies,
  ``lingam_bootstrap_accumulate``).
* :func:`total_effects` -- ``lingam_total_effects`` ((I - B)^-1, the
  total causal effects along all directed paths).
* :func:`varlingam_lagged_effects` -- ``varlingam_lagged_effects``
  (theta_tau = (I - B0) M_tau).
* :func:`batch_causal_order` -- ``lingam_batch_causal_order`` (many
  independent orderings, e.g. bootstrap resamples, in one batched run).
* :func:`workspace_size`, :func:`residualize_workspace_size`.
* learned-proposal form: ``learned=Learned(proposer, ...)`` on the ordering
  calls; :func:`proposer_scores`, :func:`proposer_grad`, :func:`proposer_adam`
  (the network's kernels: ``lingam_proposer_*``).
"""
from __future__ import annotations

from .lib import (  # noqa: F401
    LIB_PATH,
    PROPOSER_SIZE,
    Learned,
    LearnedStats,
    LingamError,
    Profile,
    adjacency,
    adjacency_pruned,
    batch_causal_order,
    bootstrap,
    bootstrap_accumulate,
    causal_order,
    causal_order_noalloc,
    last_error,
    load,
    proposer_adam,
    proposer_grad,
    proposer_scores,
    residualize,
    residualize_workspace_size,
    total_effects,
    varlingam_fit,
    varlingam_lagged_effects,
    version,
    workspace_size,
)
