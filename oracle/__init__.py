"""Plain, slow, obviously-correct FP64 CPU oracle for REXI time stepping of the
shallow-water equations on the rotating sphere (Schreiber, Schaeffer & Loft,
arXiv:1805.06557).

TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product library: only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP path (no kernels,
headers, tables or helpers) and deliberately uses different algorithms:

* ``oracle.rexi``      -- Cauchy-contour REXI coefficients in mpmath (40 digits),
                          rounded once to complex128.
* ``oracle.operator``  -- the linear operator L = L_g + L_c per zonal order m as a
                          dense matrix over (h, zeta, delta) interleaved by degree.
* ``oracle.linear``    -- REXI linear step by pivoted LAPACK banded solves of the
                          full 3-field system per (pole, m); dense expm reference.
* ``oracle.sht``       -- Gauss nodes by its own Newton iteration, normalised
                          associated Legendre functions by recurrence, numpy FFT.
* ``oracle.nonlinear`` -- N(U) on the grid, Heun RK2, Strang splitting.

Every function cites the passage of the paper it follows.  Readings of passages
that are silent or ambiguous are listed in the repository's design notes.
"""
