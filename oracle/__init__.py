"""CPU FP64 oracle for resistance distance by Lanczos iteration.

TEST INFRASTRUCTURE, NOT PRODUCT CODE. Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import, call, link or run anything in this package. The GPU library and its
Python binding never do, and share no code with it.

Modules:

* ``dense``   - r(s,t), potentials and edge gradients from the dense
                pseudoinverse (the plain definition), plus grounded-Laplacian and
                shifted-inverse cross-checks.
* ``lanczos`` - a literal numpy transcription of the paper's Algorithm 3 in
                FP64, with the tolerance stopping rule this implementation reads
                into it.
* ``cpu``     - the same Algorithm 3 and a Jacobi-preconditioned conjugate
                gradient solve in C (OpenMP), for graphs with millions of nodes.
"""
