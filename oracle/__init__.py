"""FP64 CPU oracle for the one-reduction DCGS2 Arnoldi-QR expansion.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the GPU path: it receives plain
arrays (the seeded inputs) and builds its own operators from the PDE
definitions.

Everything here is plain NumPy/SciPy in float64, written to be checked against
the paper by eye (Bielich, Langou, Thomas, Swirydowicz, Yamazaki, Boman,
"Low-Synch Gram-Schmidt with Delayed Reorthogonalization for Krylov Solvers",
arXiv 2104.01253):

* ``gram_schmidt``  -- CGS, CGS2 (Alg. cgs2), MGS and DCGS2 (Alg. qr) for QR.
* ``arnoldi``       -- CGS2 (Alg. cgs2_arnoldi), MGS and DCGS2 (Alg. arnoldi)
                       Arnoldi-QR expansions, plus the Krylov-Schur
                       continuation step.
* ``operators``     -- convection-diffusion / Manteuffel matrices (Sec. 6.1)
                       and their closed-form eigenvalues.
* ``gmres``         -- restarted GMRES on the DCGS2 basis.
* ``krylov_schur``  -- Krylov-Schur eigensolver on the DCGS2 basis.
* ``metrics``       -- loss of orthogonality and representation error (Sec. 6).

Pins (what fixes each function independently of itself) live in
``tests/test_oracle_*.py``.  Parity unpinned: none of the functions above is
left without a pin.
"""
