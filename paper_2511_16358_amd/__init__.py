"""iFCTN tensor completion by PAM on MI355X (gfx950): HIP kernels behind a
C ABI (include/ifctn.h), a ctypes binding (ifctn) and seeded synthetic
workloads (workloads)."""
