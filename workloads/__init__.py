"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package generates inputs only: compartment-label volumes of tissue-like
geometries, gradient waveforms sampled per time step, gradient directions and
the b-value scaling of the gradient amplitude.  It contains none of the
lattice Boltzmann arithmetic; both the CPU oracle and the HIP path consume
what it produces.

Units throughout: micrometre, millisecond.  D in um^2/ms, T2 in ms,
permeability kappa in um/ms, b in ms/um^2 (1000 s/mm^2 = 1 ms/um^2), and the
gradient is carried as gamma*G0 in rad/(um*ms).
"""
from .geometry import (Geometry, uniform, slabs, cylinders_z, cylinders_spheres,
                       ellipsoid_cells, link_delta, link_normal, tile_xy, angled_slabs_2d)
from .sequences import (pgse_waveform, ogse_cosine_waveform, gamma_g_for_b_pgse,
                        b_of_waveform, golden_spiral, axon_directions, GAMMA_H1)
from .configs import CONFIGS, make_config

__all__ = ["Geometry", "uniform", "slabs", "cylinders_z", "cylinders_spheres",
           "ellipsoid_cells", "link_delta", "link_normal", "tile_xy", "angled_slabs_2d", "pgse_waveform",
           "ogse_cosine_waveform", "gamma_g_for_b_pgse", "b_of_waveform",
           "golden_spiral", "axon_directions", "GAMMA_H1", "CONFIGS",
           "make_config"]
