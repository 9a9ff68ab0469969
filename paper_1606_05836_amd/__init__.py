"""MI355X (gfx950) permanents: Gray-code BB/FG (Glynn) and Ryser sweeps in HIP.

The computation lives in libpermhip.so (C ABI: include/permhip.h); this
package is its Python binding plus a torch.autograd.Function wrapper.
"""
from .permhip import (  # noqa: F401
    PH_CHUNK_LOG2_MAX,
    PH_NMAX,
    PH_NMAX_GRAD,
    PermhipError,
    Plan,
    boson_probs,
    boson_probs_grad,
    boson_sample,
    sample_inputs,
    fp64_peak,
    lib,
    perm,
    perm_batched,
    perm_noalloc,
    perm_chunk_log2,
    perm_combine,
    perm_partial,
    gray_terms,
    perm_grad,
    perm_row_minors,
    perm_ryser_paired,
    version,
)
from .autograd import BosonProbsFn, PermFn, boson_probabilities, permanent  # noqa: F401


def __getattr__(name):
    # the segment runner is also a command line (python -m ...segments), so it
    # is imported on first use rather than with the package
    if name == "segments":
        import importlib

        return importlib.import_module(".segments", __name__)
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")
