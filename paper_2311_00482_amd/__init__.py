"""MI355X plane-wave receive beamformer: HIP kernels behind a C ABI (libpwbf.so).

    from paper_2311_00482_amd import compound, beamform_das, beamform_dmas
    planes = compound(geometry, rf_tensor, "das", want=("rf", "env", "log"))
"""

from ._abi import PwbfError, lib  # noqa: F401
from .api import (  # noqa: F401
    Batch,
    FrameSpec,
    Completed,
    GeometryArg,
    ProbeSpec,
    Server,
    Tile,
    alloc_outputs,
    beamform,
    beamform_das,
    beamform_dmas,
    beamform_bbdmas,
    beamform_iqdas,
    beamform_pdas,
    compound,
    compound_noalloc,
    contrast_metrics,
    describe_plan,
    fk_migrate,
    fk_workspace_bytes,
    iq_demodulate,
    resolution_metrics,
    tune,
    tune_clear,
    tune_load,
    tune_save,
    workspace_bytes,
)
