"""CPU oracle for the IVF-PQ search path — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product (the HIP library and its Python binding)
never calls it; it shares no code with the GPU path.

Parity status: every function is pinned by a CPU test against the paper's
definitions (brute-force k-NN, the reconstructed-vector identity of Eq. 1,
lossless constructed cases, full sorts). The u8 LUT quantisation scheme
(per-subspace offset, one shared scale per (query, list), round half to
even, a pairwise sum of the offsets) is a reading of a passage that only
says the LUT entries are 8-bit unsigned integers, and the paper prints no
quantised values; the function is pinned to that reading by its error
bound, its invariants, lossless grid cases and two examples worked by hand
(one where the pairwise and the left-to-right sums of the offsets differ).
The adaptive nprobe/reorder stand-in (hardness, eq2) follows Eq. 2 with a
closed-form p in place of the paper's trained model; Eq. 2 itself is pinned
by hand-worked values and its limits, the choice of p is a reading.
The spilled assignment (spill_assign, SOAR) and the per-point pool of a
spilled index (top_r_unique) are pinned by a hand-worked case, the lam = 0
limit, an independent projection-matrix form and brute force.
"""

from .ivfpq import (  # noqa: F401
    adaptive_params,
    assign_lists,
    component_filter,
    eq2,
    hardness,
    brute_force_knn,
    encode,
    coarse_scores,
    lut_float,
    list_bias,
    quantize_lut,
    scan_list,
    search,
    select_probes,
    spill_assign,
    seq_sum,
    tree_sum,
    top_r,
    top_r_unique,
    rerank,
)
