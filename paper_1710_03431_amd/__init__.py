"""MI355X engine for quantum-jump trajectories of the adiabatic master equation.

The computation lives in the HIP library libaqt.so (C ABI in include/aqt.h);
`paper_1710_03431_amd.binding.Engine` is its Python binding.
"""

__all__ = ["binding", "build"]
