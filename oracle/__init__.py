"""Plain FP64 CPU oracle of the spectral-multigrid Poisson path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library under
``paper_2606_17636_amd/``) may import, link or call anything in this package;
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the GPU path: geometry, operator
coefficients, Fourier transforms, multigrid, screening masses and discrete
Green's functions are all written here independently, in numpy/scipy, from
the paper (Mandal, Gressel, Ziegler, Mignone, "A fast spectral-multigrid
Poisson solver in non-Cartesian geometries").

Modules
-------
geometry   finite-volume grid: faces, centroids, volumes, 1D stencil factors
           (Sec. 2.1.1 spherical, Sec. 2.1.2 cylindrical)
operator   per-mode 2D Helmholtz operator (Sec. 2.2, Eqs. helmholz_sph/cyl)
fourier    azimuthal DFT with Hermitian reduction (Sec. 2.2)
omega      WKB over-relaxation parameter (Appendix A)
multigrid  the paper's V-cycle: zebra-line even-odd SOR smoother,
           area-weighted transfers, red-black SOR coarsest solve (Sec. 3)
james      screening masses, discrete Green's functions, boundary
           convolution (Sec. 4)
solve      the seven-step workflow (Sec. 5.1)
net        the learned initial guess of the low-m planes (a U-Net with BF16
           weights and activations), forward and backward

Parity status of every function is stated in its docstring; the DGF tables
(``james.dgf_tables``) are "parity unpinned" beyond the physics checks listed
there (no closed form exists for the truncated-domain DGF).
"""
