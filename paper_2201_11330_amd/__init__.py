"""MI355X-native hot path of the IMEXLBM lattice Boltzmann method.

The compute path is the HIP library ``liblbm.so`` built from ``csrc/``; this
package only marshals arguments to it (``paper_2201_11330_amd.lbm``).  The
library is loaded on first use and its absence is an error.
"""
