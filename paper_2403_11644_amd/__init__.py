"""MI355X-native Pauli decomposition (arXiv 2403.11644 hot path).

c_P = 2^-n Tr(P A) for all 4^n Pauli strings of a 2^n x 2^n complex matrix,
computed by hand-written gfx950 HIP kernels behind a C ABI (include/ptd.h).
"""
from .api import (  # noqa: F401
    ADJOINT, ANTIDIAGONAL, BANDED, BANDS_IN, C64, C128, COMPACT, COMPENSATED, DIAGONAL, HERMITIAN, LOW_RANK,
    PURE_STATE, TOEPLITZ, BatchPlan,
    block_diagonal, decompose, decompose_batched, decompose_csr, decompose_sparse, direct_sum, hermitian_augment,
    lcu_amplitudes, linear_combination, nonempty_x, num_nonempty_x, pad_to_power_of_two, parseval, reconstruct,
)
from .labels import flat_index, index, label, to_dict  # noqa: F401
from .host_tree import host_tree_decompose  # noqa: F401
from .autograd import PauliDecompose, PauliReconstruct, pauli_decompose, pauli_reconstruct  # noqa: F401
from . import tuning  # noqa: F401

if __import__("os").environ.get("PTD_AUTOTUNE", "1") != "0":
    try:
        tuning.load()
    except Exception:  # a missing or damaged cache only means default settings
        pass
