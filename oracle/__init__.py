"""Oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow FP64 CPU implementation of what the retarded-potential path
computes, written from the paper: the direct quadrature of the Lorenz-gauge
retarded 4-potential over every source sub-domain with linear time
interpolation of the sources (Eqs. "4v potential", "4v potential multi" and
"space-time sampled four vector sources").

Only tests, the smoke check and the CPU-baseline leg of the benchmark may
import it.  It shares no code with the HIP path.
"""
from .ref import (self_cell_c1, contrib, potential_full, potential_points,
                  potential_at, box_distance_range, needed_sample_range,
                  load_library)

__all__ = ["self_cell_c1", "contrib", "potential_full", "potential_points",
           "potential_at", "box_distance_range", "needed_sample_range", "load_library"]
