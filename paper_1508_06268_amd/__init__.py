"""MI355X-native Exchange Monte Carlo (parallel tempering) for the 3D random
field Ising model (arXiv:1508.06268): HIP kernels for gfx950 behind the C ABI
of include/rfim.h, with a thin ctypes binding."""
from .rfim import (EXPORTS, Batch, Pool, FIELDS_AUTO, FIELDS_BIMODAL, FIELDS_CONTINUOUS, MEASURE_FOURIER,
                   MODE_BITS, Rfim, RfimError, load_library, rfim_adapt_temps, rfim_create, rfim_create_ex,
                   rfim_destroy, rfim_energies, rfim_sweep)

__all__ = ["EXPORTS", "Batch", "Pool", "FIELDS_AUTO", "FIELDS_BIMODAL", "FIELDS_CONTINUOUS", "MEASURE_FOURIER",
           "MODE_BITS", "Rfim", "RfimError", "load_library", "rfim_adapt_temps", "rfim_create", "rfim_create_ex",
           "rfim_destroy", "rfim_energies", "rfim_sweep"]
