"""MI355X (gfx950) library for the NSHEDB equality-mask hot path.

BFV ciphertext arithmetic over batch-encoded columns - subtraction,
multiplication with relinearization, and the Fermat equality mask
EQ(x, y) = 1 - (x - y)^(p-1) - as hand-written HIP kernels behind a C ABI
(include/nshe.h), with this package as the thin Python binding.
"""
from .context import Context  # noqa: F401
from .params import paper_params, modulus_chain  # noqa: F401
from . import _lib  # noqa: F401
