"""MI355X (gfx950) strong simulation of linear-optical interferometers.

Python face of libslos_hip.so: Fock amplitudes and probabilities of n
photons through an m-mode interferometer by the photon-by-photon recursion
of arXiv 2602.11092 (Sec. II-A), its adjoint, and the phase-shifter /
beam-splitter mesh U(x, theta); restricted computation spaces, measurement
strategies (per-mode expectations, threshold detectors, shot sampling),
amplitude-encoded inputs and the fidelity kernel.  All arithmetic runs in
the library's HIP kernels; importing this package does not load the
library until first use.
"""
from ._binding import (  # noqa: F401
    OP_AMPLITUDES, OP_AMPLITUDES_BACKWARD, OP_PROBS, OP_PROBS_BACKWARD,
    OP_MODE_EXPECTATIONS, OP_MODE_EXPECTATIONS_BACKWARD, OP_THRESHOLD_PROBS, OP_THRESHOLD_PROBS_BACKWARD,
    OP_SAMPLE, PLAN_DEFAULT, PLAN_FORWARD_ONLY, PLAN_UNBUNCHED, PLAN_DUAL_RAIL, PLAN_THRESHOLD,
    VARIANT_AUTO, VARIANT_FUSED, VARIANT_LAYERED,
    Batch, Plan, SharedSuperposition, SlosError, Superposition,
    fock_amplitudes, fock_amplitudes_backward, fock_probs, fock_probs_backward,
    fock_mode_expectations, fock_mode_expectations_backward,
    fock_threshold_probs, fock_threshold_probs_backward, fock_sample,
    fock_superposition_amplitudes, fock_superposition_amplitudes_backward,
    fock_shared_superposition_amplitudes, fock_shared_superposition_amplitudes_backward,
    fock_fidelity_kernel,
    mesh_to_unitary, mesh_to_unitary_backward,
    slos_fock_dim, slos_fock_rank, slos_fock_unrank, slos_space_dim, slos_threshold_dim, slos_unbunched_dim,
)
from . import autograd  # noqa: F401
from .layer import AmplitudeEncodedLayer, FidelityKernel, QuantumLayer  # noqa: F401
