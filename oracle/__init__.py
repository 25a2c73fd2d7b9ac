"""CPU oracle for the SNAPS similarity self-join.  TEST INFRASTRUCTURE ONLY.

Plain, slow, float64 brute force written from the paper's definitions
(Sec. 3.4-3.6, Tab. 2).  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import or execute anything in this
package; the product library never does.  It shares no code with the GPU
path.

Parity status: every function here is pinned by the tests in
``tests/test_oracle_pins.py`` (printed worked examples, closed forms,
textbook reductions and invariants); none is "parity unpinned".
"""
from .snaps_oracle import (  # noqa: F401
    project,
    pair_distances,
    knn,
    eps_join,
    eps_pairs,
    indegree,
    dense_rank,
    rank_keys,
    rank_metrics,
    ensemble,
    outlier_scores,
    alert_scores,
    selectivity,
    eps_exact_mean_count,
    eps_from_sample,
    top_n,
    list_similarity,
    select_tradeoff,
    eps_grid,
    eps_grid_metrics,
    eps_grid_select,
    k_grid_metrics,
    k_grid_select,
    eps_sampled_mean_count,
)
