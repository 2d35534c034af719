"""CPU oracle for the constrained-realization (CR) operator and its solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or call anything here.
The product path (``paper_1308_5299_amd``) never imports it, and the oracle
never imports the product path: the two share no code.  The only common
module is ``workloads`` (seeded synthetic inputs, no arithmetic of the
method).

What the oracle computes, all in float64 with numpy/scipy, written from the
definitions in Seljebotn et al. (2013):

* ``geometry``  HEALPix RING rings (Sec. 2.1; Gorski et al. 2005).
* ``legendre``  normalized associated Legendre functions P~_lm(cos theta)
                (Sec. 3.2, eq. for P~_lm beside eq. Ni-dense) by the
                three-term recurrence, in extended-exponent form.
* ``sht``       synthesis Y (eq. sh-synthesis) and its literal transpose Y^T
                (Sec. 2.1), in a real orthonormal basis; plus a brute-force
                dense Y for tiny grids built from ``scipy.special``.
* ``operator``  A = S^-1 + B Y^T N^-1 Y B (eq. system-explicit) and the level
                operators A_h = D_h + B_h Y^T N^-1 Y B_h (eq. A_h); dense
                Y^T N^-1 Y by brute force and by the ring-DFT formula
                (eq. Ni-dense).
* ``solve``     the exact solution x* = A^-1 b (dense Cholesky, or
                Jacobi-preconditioned CG), the CR right-hand side (eq.
                cr-system plus fluctuation terms), manufactured solutions
                (Sec. 4.1) and an a-posteriori max-pixel-error certificate.

Every function here is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against closed forms, library routines, brute
force or invariants of the mathematics.
"""
