"""MI355X-native hydro packet step: PLM-minmod + HLLC + SSP-RK2 on packets of
mesh blocks, computed by hand-written HIP kernels for gfx950 behind a C ABI.

Importing the package loads nothing native; ``paper_2507_09337_amd.hydro``
loads ``libhydro.so`` on first use and raises if it is missing.
"""
