"""MI355X (gfx950) truncated FFT library: Python binding of ``include/tft.h``.

Argument marshalling only: every step of the transforms and products runs in
the HIP kernels of ``libtft.so``.  PyTorch provides device memory and streams.
The binding never computes a result itself; if the shared library is missing
it raises instead of falling back to anything else.
"""

from ._binding import (  # noqa: F401
    FERMAT,
    MLP,
    NEGA,
    POLICY_GIVEN,
    POLICY_MODEL,
    POLICY_RULE,
    PRIME,
    PRIME_P,
    SPLIT_DC,
    SS_FEATURES,
    STATIC_SCRATCH_BYTES,
    BatchPlan,
    Plan,
    SSParams,
    Split,
    TFTError,
    alu_rate,
    array_bytes,
    debug_base_cases,
    elem_bytes,
    fermat_ring,
    itft_inverse,
    lib,
    lib_path,
    nega_ring,
    pointwise_mul,
    prime_ring,
    requests_array,
    ring_check,
    ss_candidates,
    ss_default_params,
    ss_features,
    ss_time,
    status_string,
    tft_forward,
    transform_workspace,
    zmx_mul_nussbaumer,
    zmx_mul_nussbaumer_workspace,
    zx_mul_ss,
    zx_mul_ss_static,
    zx_mul_ss_timed,
    zx_mul_ss_workspace,
    zx_request,
    zpx_mul_ntt,
    ZXRequest,
)

__all__ = [
    "FERMAT", "NEGA", "Plan", "SSParams", "Split", "TFTError", "array_bytes", "elem_bytes", "fermat_ring",
    "itft_inverse", "lib", "lib_path", "nega_ring", "pointwise_mul", "ring_check", "status_string", "tft_forward",
    "zmx_mul_nussbaumer", "zmx_mul_nussbaumer_workspace", "zx_mul_ss", "zx_mul_ss_timed", "zx_mul_ss_workspace",
    "BatchPlan", "MLP", "SPLIT_DC", "SS_FEATURES", "ZXRequest", "requests_array", "ss_candidates", "ss_default_params",
    "ss_features", "ss_time", "zx_request", "POLICY_GIVEN", "POLICY_RULE", "POLICY_MODEL", "transform_workspace",
    "STATIC_SCRATCH_BYTES", "zx_mul_ss_static", "alu_rate",
    "PRIME", "PRIME_P", "prime_ring", "zpx_mul_ntt",
]
