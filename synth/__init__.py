"""Seeded synthetic interferometer data (array layouts, uvw tracks, sky models).

This package produces the inputs that both the GPU imager and the oracle
consume.  It holds none of the imaging arithmetic (no gridding, no FFT, no
w-stacking): it only builds baselines, samples a sky, and predicts
visibilities with the forward measurement equation (Eq. 1 of the paper).
"""

from .interferometer import (  # noqa: F401
    C_LIGHT,
    ARCSEC,
    Dataset,
    CONFIGS,
    config_spec,
    make_config,
    make_channels,
    stack_channels,
    sky_image,
    antenna_layout,
    baselines_xyz,
    uvw_track,
    predict_point_sources,
)
