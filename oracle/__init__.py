"""FP64 CPU oracle of the accelerated dual proximal gradient (APG) solver for
scenario-tree stochastic MPC (Sampathirao, Sopasakis, Bemporad, Patrinos,
"GPU-accelerated stochastic predictive control of drinking water networks").

TEST INFRASTRUCTURE ONLY.  It exists to check the GPU library.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it; the
library never calls it, and it shares no code with the library.
"""

from .smpc_oracle import (
    OracleProblem,
    null_space_basis,
    cost_update,
    factor_step,
    solve_step,
    prox_dist,
    prox_g,
    theta_next,
    theta_sequence,
    apg,
    primal_cost,
    stage_cost,
    soft_cost,
    support_g,
    dual_objective,
    duality_gap,
    dual_hessian_dense,
    dual_lmax_power,
    shift_map,
    shift_dual,
    plant_step,
    closed_loop_kpis,
)

__all__ = [
    "OracleProblem",
    "null_space_basis",
    "cost_update",
    "factor_step",
    "solve_step",
    "prox_dist",
    "prox_g",
    "theta_next",
    "theta_sequence",
    "apg",
    "primal_cost",
    "stage_cost",
    "soft_cost",
    "support_g",
    "dual_objective",
    "duality_gap",
    "dual_hessian_dense",
    "dual_lmax_power",
    "shift_map",
    "shift_dual",
    "plant_step",
    "closed_loop_kpis",
]
