"""MI355X (gfx950) library for the dynamical symplectic reduced model of the
parametric particle-based Vlasov-Poisson system (arXiv:2201.05555) and the
particle-in-cell full-order model.

The compute path is the HIP library ``lib/libsymrom.so`` behind the C ABI of
``include/symrom.h``; ``paper_2201_05555_amd.binding`` marshals arguments to
it.  PyTorch provides device memory and streams only.
"""
__all__ = ["binding"]
