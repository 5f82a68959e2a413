"""MI355X (gfx950) adaptive ray-tracing radiative transfer.

Thin Python binding of the C ABI in include/rt.h (librtmi.so, built from
csrc/ by build.py).  Every step of the computation runs in the library's HIP
kernels; this module only marshals torch device tensors (memory and streams)
into the C calls.  There is no CPU fallback: if the library is not built, or
no GPU is present, the calls raise.
"""
from .binding import (  # noqa: F401
    RT_F32,
    RT_F64,
    REDUCTION_PARAMS,
    SCHED_BINNED,
    SCHED_DIRECT,
    SCHED_SPATIAL,
    SCHEME_FEAUTRIER2,
    SCHEME_HERMITE,
    WALK_EXACT,
    WALK_PADDED,
    WALK_TWO_PASS,
    MLP,
    Batch,
    DirSet,
    Model,
    Plan,
    RtError,
    autotune,
    cached_memory,
    plan_memory,
    closure_apply,
    closure_feature_stats,
    closure_features,
    closure_merge,
    closure_normalize,
    closure_targets,
    release_cached_memory,
    compute_J,
    compute_J_batched,
    compute_J_direct,
    compute_J_workspace,
    closure_J,
    closure_J_ws,
    opts_dict,
    healpix_vec2pix,
    load,
    mesh_indicators,
    mlp_nll,
    solve,
    spatial_order,
    sync_status,
    trace,
    validate_host,
    version,
)
