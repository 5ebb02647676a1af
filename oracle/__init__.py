"""CPU FP64 oracle for the FlashMP hot path (test infrastructure only).

This package is a plain, slow, obviously correct NumPy/SciPy reference of what
the GPU library computes.  It exists to check the GPU path, never to run it:
only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import it.  It shares no code with the HIP library and
does not import the product package.

Modules
-------
yee        Yee-grid unknown sets, the sparse curl C and double-curl K = C^T C,
           the operator A = I + c diag(1/eps_e) K (Section II-A, eq. (4);
           Section III-A, curl and double-curl displays).
transforms Orthonormal DCT-II / DST-I matrices and the discrete transform
           box solve: forward transform, per-wavenumber 3x3 block solve,
           inverse transform (Section III-A, Steps 1-3, eq. (6), Alg. 1
           exact_solve), restated for a PEC box.
ras        Restricted additive Schwarz preconditioner built from exact box
           solves (Section II-B, the M_RAS^{-1} display).
woodbury   The paper's index-block subdomain: compact differences and their
           SVD (eq. (8)), exact_solve with that basis, the boundary term
           Lambda = Q W Q^T / alpha and Algorithm 1's Woodbury correction
           (Section III-A Step 4), and RAS over index blocks (overlap >= 0).
krylov     Right-preconditioned BiCGSTAB and flexible GMRES(m) (Section IV-A
           workloads; Table III operation counts).
coarse     Learned coarse correction reference: subdomain averaging R0,
           piecewise-constant prolongation P0, and an FP64 MLP with a
           hand-written backward pass.
"""
