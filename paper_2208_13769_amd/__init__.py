"""MI355X (gfx950) implementation of the per-time-step lattice update of the
Lagrangian lattice Boltzmann method for nonlinear solids (Faust, Schlueter,
Mueller & Mueller, 2022).

The native library is loaded lazily by :mod:`paper_2208_13769_amd.lbm`, so
importing the package (for example for :mod:`.inputs`) needs no GPU.
"""
