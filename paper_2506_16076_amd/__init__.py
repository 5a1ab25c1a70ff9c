"""MI355X-native FC-SDNN hot path: FC-Gram derivatives, curvilinear Euler
right-hand side with smooth artificial viscosity, network classifier and
SSPRK(5,4) stages as hand-written HIP kernels behind a C ABI
(include/fcsdnn.h, libfcsdnn.so).

``paper_2506_16076_amd.api`` holds the torch-facing wrappers; importing it
requires the built library and torch.
"""
__all__ = ["api", "build"]
