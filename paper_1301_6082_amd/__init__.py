"""MI355X-native multispin Monte Carlo sweep of 1+1-dimensional
reaction-diffusion models (DP, PCPD, TCPD), after Schram, arXiv:1301.6082.

The compute path is the HIP library libpcpd.so behind include/pcpd.h; the
Python module `pcpd` is its ctypes binding. Importing this package loads
nothing; import `paper_1301_6082_amd.pcpd` to load the library.
"""
