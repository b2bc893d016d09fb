"""Seeded synthetic inputs for the warehouse plan evaluator.

This package only draws random data (warehouse instances, order histories and
candidate plans).  It holds none of the plan-cost arithmetic, so both the CPU
oracle and the GPU path can consume its output without sharing any of the
method's logic.
"""
from .generators import (  # noqa: F401
    Instance,
    WORKLOADS,
    make_instance,
    make_plans,
    make_batched_instances,
    make_typed_orders,
    workload,
)
