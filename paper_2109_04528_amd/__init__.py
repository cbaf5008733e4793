"""MI355X Torontonian: the recursive Cholesky-reuse evaluation of Eq. 2 of
Kaposi et al. (arXiv 2109.04528) as HIP kernels for gfx950 behind a C ABI.

    from paper_2109_04528_amd import Context
    with Context() as ctx:
        r = ctx.eval(O)            # O: 2n x 2n complex128 (numpy or torch)
        r.value, r.cancellation   # Tor(O) and R = sum|t| / |Tor|
    with Context(flags=TOR_FACTOR_DD) as ctx:
        ctx.eval(O)                # the same with a double-double factor

The binding only marshals arguments; the library must be built (see build.py)
and there is no CPU fallback.
"""
from ._lib import (  # noqa: F401
    Context, TorError, TorResult, load, workspace_size,
    TOR_OK, TOR_PENDING, TOR_E_INVAL, TOR_E_NOT_PD, TOR_E_NUMERIC, TOR_E_BUSY,
    TOR_E_NOMEM, TOR_E_DEVICE, TOR_E_TIMEOUT, TOR_E_UNKNOWN, TOR_E_SCRATCH,
    TOR_ACCUM_DD, TOR_ACCUM_FP64, TOR_INPUT_DEVICE, TOR_CHECK_HERMITIAN, TOR_FORCE_COMPLEX,
    TOR_FACTOR_DD, TOR_OUTPUT_DEVICE, TOR_TUNE_REAL, TOR_TUNE_COMPLEX, TOR_TUNE_QUAD,
    TOR_CLICK_ALL_MAX_M,
)


def tor(O, **ctx_kwargs) -> float:
    """Torontonian of one matrix with a throw-away context.  A torch CUDA
    tensor is read in place (TOR_INPUT_DEVICE); anything else is copied
    from host memory."""
    if getattr(getattr(O, "device", None), "type", None) == "cuda":
        ctx_kwargs["flags"] = ctx_kwargs.get("flags", 0) | TOR_INPUT_DEVICE
    with Context(**ctx_kwargs) as ctx:
        return ctx.eval(O).value
