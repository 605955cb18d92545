"""Seeded synthetic inputs for the plane-wave beamformer.

This package generates scatterer phantoms and the channel RF they produce under
plane-wave insonification. It is the only code shared by the FP64 oracle tests
and the GPU path: it contains the forward acoustic model (echo arrival times and
the transmitted pulse) and no receive-beamforming step (no interpolation,
apodization, summation, compression or FFT post-processing).
"""

from .configs import (  # noqa: F401
    Geometry,
    config_c1,
    config_c2,
    config_c3,
    config_c4_frames,
    config_c5_probes,
    paper_geometry,
)
from .phantom import (  # noqa: F401
    Phantom,
    phantom_c1,
    phantom_c3,
    phantom_scaled,
    point_phantom,
    simulate_rf,
    make_frame,
)
