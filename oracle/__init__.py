"""Plain CPU FP64 oracle for the Gaussian-state -> MPS conversion.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (different algorithms are used on purpose wherever one exists: NumPy
``eigh`` instead of Jacobi sweeps, a heap instead of the sibling enumeration,
the paper's sequential PCO algorithms instead of the level gather).

Modules, each following the paper (arXiv 2512.10643):

* ``hafnian``   -- brute-force hafnians and Fock amplitudes of paired-form
                   states (the definition the tensors must reproduce, Sec. II.C).
* ``gaussian``  -- covariance checks, Williamson form, Bogoliubov matrices,
                   paired forms and the iterative Gaussian SVD (Sec. II.A-B,
                   App. A).
* ``kept``      -- entanglement energies, kept virtual bases and truncation
                   errors (Sec. II.C.1, Sec. III.A).
* ``pco``       -- Algorithms 1-5 of App. B plus the physical-mode PCOs.
* ``recurrence``-- an independent per-element route to the same tensors
                   (annihilation-operator recursion; used only as a pin).
* ``mps``       -- assembly, normalisation, amplitudes, exact marginals,
                   sampling, fidelity and SVD truncation of the MPS.
* ``build``     -- the whole pipeline, step by step.

Parity status of each function is stated in its module header.
"""
