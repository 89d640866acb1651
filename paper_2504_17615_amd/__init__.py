"""MI355X-native multilevel graph partitioning with edge sparsification.

Python binding of ``liblmgp.so`` (C ABI in ``include/lmgp.h``).  This module
only marshals arguments: every step of coarsening, sparsification,
partitioning and refinement runs in the library's HIP kernels and host
engine.  Importing the package does not load the library; the first call does,
and raises if it has not been built (``paper_2504_17615_amd.build``).
"""
from ._binding import (  # noqa: F401
    NOALLOC_MAX_ENTRIES,
    NOALLOC_MAX_NODES,
    NOALLOC_SCRATCH_BYTES,
    LmgpError,
    Params,
    LevelInfo,
    Result,
    ServerConfig,
    ServerStats,
    DeviceGraph,
    Hierarchy,
    Server,
    create_graph,
    default_params,
    library,
    partition_batch,
    profile_enable,
    profile_filter,
    profile_read,
    tuner_clear,
    tuner_info,
)
