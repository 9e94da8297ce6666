"""Seeded synthetic grids, partitions, states and noise draws (inputs only)."""
from .synth import *  # noqa: F401,F403
from .synth import CONFIGS, Grid, Batch, make_grid, make_config, make_batch, make_chains, grid_stats, measurement_set  # noqa: F401
