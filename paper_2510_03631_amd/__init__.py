"""MI355X (gfx950) PIR Answer engine.

The server step of single-server LWE private information retrieval over a
byte database resident in HBM: ``a = D q mod 2^32``, its batched form and the
offline hint ``H = D A``, as hand-written HIP kernels behind the C ABI in
``include/qpir.h``.  This package is the thin Python binding; it never
computes on the host.
"""
from ._lib import (Database, PirError, lib, LIB_PATH, SIGNATURES,  # noqa: F401
                   chor_answer, client_decode, client_query, variant_names)

__all__ = ["Database", "PirError", "lib", "LIB_PATH", "SIGNATURES", "client_query",
           "client_decode", "variant_names", "chor_answer"]
