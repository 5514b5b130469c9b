"""paper_2604_01356_amd -- divide-and-conquer multinomial resampling on MI355X.

A thin Python binding over libdcr.so (include/dcr.h).  The functions carry
the C names and only marshal arguments: torch tensors supply device memory and
the current HIP stream; every step of the computation runs in the library's
HIP kernels.  Importing this package does not load the library; the first call
does, and fails loudly if the library has not been built.
"""
from ._binding import (  # noqa: F401
    DCR_FP32_COMP,
    DCR_FP64,
    DCR_MULTINOMIAL,
    DCR_STRATIFIED,
    DCR_SYSTEMATIC,
    DcrError,
    dcr_batched_autotune,
    dcr_batched_workspace_bytes,
    dcr_cumulative_weights,
    dcr_inverse_cmf,
    dcr_plan_autotune,
    dcr_plan_create_batched,
    dcr_plan_destroy,
    dcr_plan_map_chunk,
    dcr_plan_resample_batched,
    dcr_profile_begin,
    dcr_profile_end,
    dcr_resample,
    dcr_resample_batched,
    dcr_resample_batched_ex,
    dcr_resample_noalloc,
    dcr_resample_outer,
    dcr_resample_scheme,
    dcr_scheme_uniforms,
    dcr_sorted_uniforms,
    dcr_status_string,
    dcr_stream_probe,
    dcr_workspace_bytes,
    library,
    library_path,
    precision_of,
    STATUS,
)
