"""MI355X (gfx950) implementation of the enthalpy-based MRT lattice Boltzmann
method for solid-liquid phase change in metal foams under local thermal
non-equilibrium (arXiv:1701.00702).

The compute path is the shared library ``liblbmpcm.so`` built from
``csrc/`` (C ABI in ``include/lbmpcm.h``); ``lbm`` is its ctypes binding and
``build`` compiles it.
"""
