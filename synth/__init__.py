"""Seeded synthetic workloads (inputs only; no retarded-potential arithmetic)."""
from .sources import (Domain, System, Charge, config1, config2, config3_twin,
                      config4, config5, sample_sources, spatial_factors,
                      time_factors, grid_points)

__all__ = ["Domain", "System", "Charge", "config1", "config2", "config3_twin",
           "config4", "config5", "sample_sources", "spatial_factors",
           "time_factors", "grid_points"]
