"""Seeded synthetic input generators (no arithmetic of the method lives here)."""
from .inputs import (WORKLOADS, Workload, batch_sides, custom, initial_theta, instance, rectangles,
                     unit_noise, zero_mean_filters)

__all__ = ["WORKLOADS", "Workload", "batch_sides", "custom", "initial_theta", "instance", "rectangles",
           "unit_noise", "zero_mean_filters"]
