"""Seeded synthetic inputs for the acoustic wave-equation forward / gradient path.

This package only *generates inputs*: velocity models (layered media with a
Gaussian-smoothed random perturbation), the Ricker source wavelet, acquisition
positions, model windows and the time grid chosen from a CFL number.  It holds
none of the wave-equation arithmetic (stencil, damping profile, interpolation
weights, time stepping, adjoint, imaging condition): the CPU oracle and the HIP
library each implement that on their own, and both consume the arrays built
here, bit-identical, as float32.

Units (used throughout the repository):
  grid spacing h in m; time in ms; velocity in km/s (= m/ms);
  squared slowness m = 1/v^2 in ms^2/m^2 (= s^2/km^2); frequency in kHz.

The paper's seismic workloads (crosswell time-lapse surveys on Compass-derived
models, section "Preliminary inversion results") are not available; the
generators below stand in for them with the same kind of structure: layered
media with smooth random heterogeneity and many shots per survey.
"""
from .configs import (Shot, Workload, ricker, layered_velocity, two_layer_velocity,
                      smooth_perturbation, smooth_background, extend_edge, cfl_time_grid,
                      make_config, config_names, small_2d, small_3d, synthetic_residual, probe_table,
                      random_field, timelapse_survey, plume_mask, reservoir_rock,
                      saturation_field)

__all__ = ["Shot", "Workload", "ricker", "layered_velocity", "two_layer_velocity",
           "smooth_perturbation", "smooth_background", "extend_edge", "cfl_time_grid",
           "make_config", "config_names", "small_2d", "small_3d", "synthetic_residual", "probe_table",
           "random_field", "timelapse_survey", "plume_mask", "reservoir_rock",
           "saturation_field"]
