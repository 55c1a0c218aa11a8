"""Seeded synthetic workloads for the IVF-PQ search path.

This package produces *inputs* only: base vectors, queries, per-query probe
counts and a trained IVF + residual-PQ index (index construction, Alg. 1).
It holds none of the search path's arithmetic (coarse scoring, LUT build,
quantisation, ADC scan, top-R, re-rank). Both the GPU path and the CPU
oracle consume what it produces; neither shares code with the other.
"""

from .synth import CONFIGS, WorkloadConfig, make_workload, scaled  # noqa: F401
from .train import spill_index, train_index  # noqa: F401
from .truth import exact_knn, recall_at_k  # noqa: F401
