"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This package draws random numbers and lays out plain real-space fields (plane
waves, Gaussian blobs, a laser pulse, macro-particle deposits).  It holds none
of the solver's arithmetic: no Fourier transforms, no modified wavenumbers, no
PSATD coefficients.  Anything that needs those (a divergence-free projection, a
charge density consistent with continuity) is done by whoever calls it.
"""

from .fields import (  # noqa: F401
    FIELD_NAMES,
    SEED_BASE,
    rng_for,
    random_fields,
    plane_wave_modes,
    plane_wave_sum,
    transverse_unit,
    gaussian_blob,
    laser_pulse,
    laser_modes,
    macro_particle_deposit,
    uneven_decomposition,
    plane_waves_and_blob,
)
from .particles import plasma_particles  # noqa: F401,E402
