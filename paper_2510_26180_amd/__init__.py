"""KLE-CGC on AMD Instinct MI355X (gfx950): parareal with a diagonalised coarse grid
correction and a KL/gPC initial guess (arXiv 2510.26180), as hand-written HIP kernels
behind a C ABI (include/klecgc.h), with a thin ctypes binding.

Importing the package does not touch the GPU; `Context()` loads libklecgc.so and
fails loudly if it has not been built.
"""
from ._lib import (KC_BATCH_GRAPH, KC_BATCH_PERSISTENT, KC_GPC_HERMITE, KC_GPC_LEGENDRE, KC_MODEL_ADE_P1,  # noqa: F401
                   KC_MODEL_ALLEN_CAHN, KC_MODEL_BURGERS, KC_INIT_COARSE, KC_INIT_GIVEN, KC_INIT_GPC, KC_INIT_MLP,  # noqa: F401
                   KC_INIT_MLP_GPC_FALLBACK, KC_INIT_RANDOM, KC_INIT_ZERO, KC_KLE_FIELD_EXP,
                   KC_KLE_SNAPSHOT, KC_PREC_F32_REFINED, KC_PREC_F64, KC_SAMPLE_CONVERGED,
                   KC_SAMPLE_MAXITER, KC_SAMPLE_NONFINITE, LIB_PATH, load)
from .api import Context, Handle, KlecgcError, ModelSpec, ProblemSpec  # noqa: F401

__all__ = ["Context", "Handle", "KlecgcError", "ModelSpec", "ProblemSpec", "load", "LIB_PATH"]
