"""lbnlm: MI355X-native lattice-Boltzmann solver for channel flow of the
instantaneous nonlinear generalised Maxwell fluid (Papenkort & Voigtmann,
arXiv:1310.7450).

The solver is the C-ABI library ``liblbnlm.so`` (``include/lb.h``) built from
the gfx950 HIP sources in ``csrc/``; :mod:`.lbnlm` is its Python binding.
Channels are driven by a body force, by a pressure drop (generalised
periodic boundaries) or by a moving top wall (planar Couette flow).

Other modules: :mod:`.workloads` (seeded inputs), :mod:`.protocol`
(start-up/cessation driver), :mod:`.autotune` (strip height),
:mod:`.mlp` (the warm-start network, ``include/lbml.h``) and
:mod:`.warmstart` (training on solver steady states, warm-started runs).
"""
from .lbnlm import (ABI_FUNCTIONS, FP32_SHIFTED, FP64, PROFILES, SCALARS, ChannelSpec, LbError,
                    Solver, load_library, options, workspace_bytes)

__all__ = ["ABI_FUNCTIONS", "FP32_SHIFTED", "FP64", "PROFILES", "SCALARS", "ChannelSpec", "LbError",
           "Solver", "load_library", "options", "workspace_bytes"]
