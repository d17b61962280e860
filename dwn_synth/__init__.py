"""Seeded synthetic inputs for scenario-tree stochastic MPC of drinking water networks.

This package only *generates* problem data: linear flow models, boxes, cost
weights, scenario trees and node demands.  It holds none of the solver's
arithmetic, so both the FP64 CPU oracle and the GPU library can be fed from it
without sharing any method code.

Every generator takes an explicit seed and uses ``numpy.random.default_rng``.
"""

from .trees import uniform_tree, table1_tree, TABLE1, stage_counts
from .systems import tiny_tank_system, barcelona_shaped_system, random_dense_system
from .instances import (
    Instance,
    tiny_instance,
    barcelona_instance,
    table1_instance,
    batch_instances,
    random_small_instance,
    barcelona_demands,
    closed_loop_demands,
    serving_controllers,
    step_demands,
)

__all__ = [
    "uniform_tree",
    "table1_tree",
    "TABLE1",
    "stage_counts",
    "tiny_tank_system",
    "barcelona_shaped_system",
    "random_dense_system",
    "Instance",
    "tiny_instance",
    "barcelona_instance",
    "table1_instance",
    "batch_instances",
    "random_small_instance",
    "barcelona_demands",
    "closed_loop_demands",
    "serving_controllers",
    "step_demands",
]
