"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  Draws inputs only; no retrieval arithmetic lives here."""
from .cubes import (Cube, pixel_cube, tissue_cube, tissue_703k, frame, lowrank_log_cube, components,
                    paper_sim_cube, paper_sim_shape, PAPER_SIM_SCALES,
                    wavenumbers, envelope, reference, lorentz_chi, rng_for)

__all__ = ["Cube", "pixel_cube", "tissue_cube", "tissue_703k", "frame", "lowrank_log_cube", "components", "paper_sim_cube",
           "paper_sim_shape", "PAPER_SIM_SCALES",
           "wavenumbers", "envelope", "reference", "lorentz_chi", "rng_for"]
