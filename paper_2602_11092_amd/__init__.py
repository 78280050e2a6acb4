"""MI355X (gfx950) strong simulation of linear-optical interferometers.

Python face of libslos_hip.so: Fock amplitudes and probabilities of n
photons through an m-mode interferometer by the photon-by-photon recursion
of arXiv 2602.11092 (Sec. II-A), its adjoint, and the phase-shifter /
beam-splitter mesh U(x, theta).  All arithmetic runs in the library's HIP
kernels; importing this package does not load the library until first use.
"""
from ._binding import (  # noqa: F401
    OP_AMPLITUDES, OP_AMPLITUDES_BACKWARD, OP_PROBS, OP_PROBS_BACKWARD,
    VARIANT_AUTO, VARIANT_FUSED, VARIANT_LAYERED,
    Batch, Plan, SlosError,
    fock_amplitudes, fock_amplitudes_backward, fock_probs, fock_probs_backward,
    mesh_to_unitary, mesh_to_unitary_backward,
    slos_fock_dim, slos_fock_rank, slos_fock_unrank,
)
from . import autograd  # noqa: F401
from .layer import QuantumLayer  # noqa: F401
