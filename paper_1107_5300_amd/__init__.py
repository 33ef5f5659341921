"""MI355X-native RGF conductance of armchair graphene nanoribbons.

HIP kernels for gfx950 behind the C ABI in include/rgf.h (librgf.so in this
directory), with a thin torch binding. Build with
`python -m paper_1107_5300_amd.build`.
"""

from .rgf import (  # noqa: F401
    Ribbon,
    PRECISIONS,
    Workspace,
    conductance,
    conductance_batched,
    conductance_noalloc,
    conductance_segments,
    grad,
    ldos,
    RGFConductance,
    lead_self_energy,
    lead_modes,
    channel_transmission,
    workspace_bytes,
    version,
    autotune,
    refine_stats,
)
