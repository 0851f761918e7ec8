"""CPU oracle for the quantics-tensor-train (QTT) Navier-Stokes RK4 step.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
float64 NumPy implementation of what the GPU library computes, written from the
paper (arXiv 2406.17823, "Quantum-Inspired Fluid Simulation of 2D Turbulence
with GPU Acceleration").  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
HIP path: no kernels, headers, helpers, tables or constant generators.

Modules
-------
mps     quantics encoding, TT-SVD, MPS add / Hadamard / MPO apply, TT-rounding
mpo     finite-difference MPOs built from the carry table of App. A
sweep   environments, local linear systems, CG, the one-site variational sweep
        (App. B) and the RK4 step as four Euler minimisations
dense   brute-force full-grid step: circulant finite differences, the penalty
        solve in closed form per Fourier mode, RK4
mlp     float64 forward/backward of the learned block preconditioner
schmidt Schmidt spectra per bipartition and the bond dimension chi_l(eps)
dns     dense DNS reference (App. D), fidelity and TKE spectrum

Parity status of each function is stated in its docstring; a function without
an independent pin says "parity unpinned".
"""
