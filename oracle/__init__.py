"""FP64 CPU oracle for the confined polar-active-fluid (TTSH) solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the GPU path: its transforms are
``scipy.fft``/``numpy.fft`` (checked against a brute-force O(N^4) DFT), its
arithmetic is written from the paper's equations, and it reads nothing the GPU
path produces.

Modules
-------
ttsh  the time step (Alg. 1 literally, and an independent velocity/Leray form),
      the masks (tanh and Alg. 2), projections, norms, diagnostics.
fno   the Fourier-neural-operator surrogate, forward and hand-written backward.
"""
