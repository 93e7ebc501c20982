"""MI355X (gfx950) qubit lattice algorithm for 2D Maxwell scattering in an inhomogeneous
dielectric: hand-written HIP kernels behind the C ABI of include/qla.h, with a thin
ctypes binding (`paper_2604_21128_amd.qla`)."""

__all__ = ["qla", "build"]
