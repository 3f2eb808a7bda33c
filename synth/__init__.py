"""Seeded synthetic input generators (no arithmetic of the method lives here)."""
from .inputs import (SERVE_S, SERVE_SIDES, WORKLOADS, Workload, batch_set, batch_sides, custom, initial_theta,
                     instance, poisson_arrivals, rectangles, serve_samples, theta_drift, unit_noise,
                     zero_mean_filters)

__all__ = ["SERVE_S", "SERVE_SIDES", "WORKLOADS", "Workload", "batch_set", "batch_sides", "custom",
           "initial_theta", "instance", "poisson_arrivals", "rectangles", "serve_samples", "theta_drift",
           "unit_noise", "zero_mean_filters"]
