"""MI355X (gfx950) entropic lattice Boltzmann step with the closed-form
relaxation parameter, behind the C ABI of include/elbm.h.

`elbm` is the ctypes binding of libelbm.so (built by `build`); `workloads`
holds the seeded synthetic initial fields.
"""
