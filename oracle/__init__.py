"""Plain FP64 CPU oracle of the pseudospectral phase-field ImEx-ARK method.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (no kernels, headers, tables or helpers) and never consumes anything the
HIP path produced; both sides only share the seeded input generators in
``pfinputs``.

Modules
-------
spectral     grid, wavevectors, real 3D DFT conventions, brute-force DFT
model        free energy terms, Khachaturyan elasticity, split right-hand side
ark          ImEx additive Runge-Kutta tables, step, embedded error, WRMS,
             step-size controller, time loop
diagnostics  mass, free energy, precipitate volume fraction
fno          Fourier neural operator forward/backward in FP64

Parity status: every function here is pinned by the ``-m "not gpu"`` tests
against closed forms, brute force, invariants or library routines; see the
per-module headers.  Functions without such a pin say "parity unpinned".
"""
