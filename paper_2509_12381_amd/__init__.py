"""Ensemble Dormand-Prince 5(4) integration of atom + trapped-ion trajectories
on AMD Instinct MI355X (gfx950).

The integrator runs in hand-written HIP kernels behind the C ABI declared in
``include/ai.h`` (``libai.so``); ``binding`` marshals arguments to it and
``workload`` builds seeded synthetic inputs.  Importing the package loads
nothing; the HIP library is opened on first use and a missing build is an
error, never a fallback.
"""
__all__ = ["workload", "binding"]
