"""MI355X-native self-adaptive Ising machine (SAIM) hot path.

Import of this package is light: the HIP library is loaded on first use of
``paper_2501_04971_amd.binding``.
"""
