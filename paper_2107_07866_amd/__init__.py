"""MI355X EAM lattice molecular dynamics (the MISA-MD hot path) on hand-written HIP kernels.

``misa`` is the ctypes binding of the C ABI in ``include/misa.h``;
``Lattice`` owns one handle and its torch-allocated state buffer; ``Batch`` owns
many boxes stepped together (batched replicas).
"""
from . import misa  # noqa: F401  (fails loudly when libmisa.so is missing)
from .lattice import Batch, Lattice  # noqa: F401
