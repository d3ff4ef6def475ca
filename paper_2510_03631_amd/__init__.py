"""MI355X (gfx950) PIR Answer engine.

The server step of private information retrieval over a database resident in
HBM, as hand-written HIP kernels behind the C ABI in ``include/qpir.h``:
single-server LWE (``a = D q mod 2^32``, its batched form, the offline hint
``H = D A``), Goldberg's field form (``D Q mod p``), Chor XOR PIR and the
CIP-PIR offline/online split.  This package is the thin Python binding; it never
computes on the host.
"""
from ._lib import (ClientMatrix, Database, PirError, lib, LIB_PATH, SIGNATURES,  # noqa: F401
                   chor_answer, client_decode, client_query, oop_answer, oop_offline,
                   prg_expand, variant_names)

__all__ = ["ClientMatrix", "Database", "PirError", "lib", "LIB_PATH", "SIGNATURES",
           "client_query", "client_decode", "variant_names", "chor_answer", "prg_expand",
           "oop_offline", "oop_answer"]
