"""MI355X-native unsplit hydrodynamic solver (MHM, VL, CTU) for patch groups.

Importing the package loads nothing; ``paper_1103_3373_amd.hydro`` binds the
HIP library ``libhydro.so`` on first use and fails loudly if it is missing.
"""
