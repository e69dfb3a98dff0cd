"""Short-range particle-particle gravity force on MI355X (gfx950).

The public functions marshal arguments to the HIP library libsr (``_sr``);
the seeded workloads live in ``synth`` and the filter fit in ``filter_fit``.
"""
from ._sr import (BatchPlan, BlocksPlan, CentresPlan, PkPlan, SRError, SRForce, batch_force, bin, bin_view, count_pairs,  # noqa: F401
                  force, force_static, force_vjp, grid, halo_centres, launch_config, momentum, new_workspace, sparse_group, sr_force, tile_balance, tile_config, timing_enable,
                  timing_read, workspace_bytes, ws_flags)
