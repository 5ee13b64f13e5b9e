"""MI355X (gfx950) two-material finite-volume library -- Python binding.

A thin ctypes layer over the C ABI in ``include/m2c.h`` (``libm2c.so``, built
in-tree by ``paper_2508_16387_amd.build``).  Every step of the method runs in
the library's HIP kernels; this package only marshals arguments.  PyTorch is
used, where a caller wants it, for device memory and streams (``torch.cuda``
tensors and streams can be passed to the ``*_device`` calls and the
kernel-level entry points).

Importing the package does not load the library; :func:`lib` does, and it
raises if ``libm2c.so`` has not been built -- there is no fallback path.
"""
from ._binding import (  # noqa: F401
    M2C_OK, M2C_ERR_ARG, M2C_ERR_NONPHYSICAL, M2C_ERR_RIEMANN, M2C_ERR_DEVICE, M2C_ERR_STATE,
    M2C_ERR_UNIMPLEMENTED, M2C_ERR_NOMEM, M2C_BC_TRANSMISSIVE, M2C_BC_WALL, M2C_BC_PERIODIC,
    M2C_PREC_FP64, M2C_PREC_MIXED, M2C_GUESS_ACOUSTIC, M2C_GUESS_MLP,
    M2C_LIM_MC, M2C_LIM_VAN_ALBADA, M2C_LIM_VAN_ALBADA_MOD, M2C_FLUX_HLLC, M2C_FLUX_LLF,
    Config, Stats, M2CError, lib, lib_path, exported_symbols, config_default, config_for, Sim, Batch,
    eval_hllc, riemann_solve, Mlp, TrainOpts, mlp_features, riemann_solve_learned, NPARAM,
    M2C_EOS_NASG, M2C_EOS_MG, M2C_EOS_JWL, M2C_EOS_MAX, Eos, eos_table, riemann_solve_eos, eos_eval,
    reinit_field, riemann_solve_learned_async, NOALLOC_MAX_PROBLEMS, riemann_solve_eos_learned, mlp_features_eos,
)
