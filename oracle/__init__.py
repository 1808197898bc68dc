"""Plain FP64 CPU oracle for the hybrid low-Mach lattice-Boltzmann / finite-difference
time step (Hosseini, Darabiha, Thevenin, "Low Mach number lattice Boltzmann model for
turbulent combustion: flow in confined geometries", arXiv 2207.11567).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its Python
binding) may import, call or link this package; only ``tests/``, ``__graft_entry__.smoke``
and the ``cpu_baseline`` leg of ``bench.py`` use it, to check and to time the GPU path.

It is written for a reader holding the paper: every function follows one equation or one
stated step of Sec. 2 (Eqs. 1-14) in the paper's notation, in float64, vectorised over
cells with plain torch/numpy operations and no blocking, fusion or reordering.  Where the
paper is silent or garbled the reading taken is stated in the function's docstring.

Shares no code with the HIP path: its own lattice tables, equilibria, moment transforms,
cumulant relations, stencils, chemistry and noise generator.

Pins: every function is checked in ``tests/test_oracle_*.py`` against closed forms,
invariants, brute force or special cases fixed by the paper or by mathematics.
Parity unpinned: the paper's own cumulant realisation (its transforms are in a
supplement that is not available), which is why the reading here is the specification.
"""
