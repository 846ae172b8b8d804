"""MI355X-native geometric-energy correlation (skeletal densities, 3D FFT).

The compute path lives in libga.so (HIP kernels for gfx950 behind the C ABI of
include/ga.h); ``paper_1711_05017_amd.ga`` is its ctypes binding.
"""

from . import ga  # noqa: F401
from .ga import (  # noqa: F401
    GA_C2R,
    GA_FIELDS,
    GA_LOWPASS_COARSE,
    GA_LOWPASS_ZEROPAD,
    GA_PLAN_AXIS_PASSES,
    GA_R2C,
    GA_SCORE_IM,
    GA_SCORE_RE,
    GA_SERVE_LOCAL,
    GA_SERVE_SPECTRAL,
    GA_SINGLE,
    Batch,
    GaError,
    Plan,
    Server,
    ga_correlate,
    ga_energy_fields,
    ga_fft3d,
    ga_field_table,
    ga_field_table_query,
    ga_field_grad,
    ga_force_torque,
    ga_force_torque_noalloc,
    ga_lowpass,
    ga_spectral_pack4,
    ga_spectral_rotate,
    ga_spectral_rotate_packed,
    ga_pose_local,
    ga_pose_prepare,
    ga_pose_spectral,
    ga_score,
    ga_splat,
    ga_supported_n,
)
from .spectra import load_spectrum, save_spectrum, skeleton_key  # noqa: F401


def lib():
    """The loaded libga.so (raises when it has not been built)."""
    return ga.load()
