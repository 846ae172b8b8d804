"""FP64 CPU oracle for the skeletal-density cross-correlation.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
link this package: only the tests, the smoke check and the benchmark's CPU
baseline leg use it. It shares no code with the HIP library; the only module
both sides consume is the seeded input generator package ``synth``.

Every function is a plain, slow, obviously correct restatement of what the
paper defines, in float64. See ``oracle.core`` for the citations.
"""

from .core import (  # noqa: F401
    place,
    kernel_value,
    splat,
    moment_channels,
    min_image_coord,
    dft_direct3,
    dft_axis,
    fft_axis,
    fft3,
    ifft3,
    rfft3,
    irfft3,
    omega,
    grad_spectral,
    correlate_direct,
    correlate_brute_field,
    correlate_fft,
    energy_field,
    force_field_spectral,
    force_field_physical,
    torque_field_moment,
    torque_field_cross,
    single_pose_sum,
    local_pose_sum,
    spectral_rotate,
    spectral_rotate4,
    lowpass_mask,
    lowpass_coarse,
    lowpass_energy,
    affinity_weights,
    reflect_spectrum,
    score_direct,
    score_fft,
    lattice_read,
    trilinear_read,
    pair_fields,
    rel_l2,
)
