"""Plain FP64 CPU oracle for the two-flavour Wilson-fermion HMC hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything here.  The product
path (the HIP library and its Python binding) never imports, links or calls
this package, and this package imports nothing from the product path: the two
share only the seeded input generators in ``lattice_inputs``.

Everything is NumPy complex128 / float64, vectorised over lattice sites with
``np.roll`` shifts so that each function reads like its defining formula.  No
blocking, fusion or reordering beyond what each definition states.

Paper reference: Haar, Kamleh, Zanotti, Nakamura, "Improving
Polynomial-filtered Hybrid Monte Carlo With Hasenbusch" (INPC 2016,
arXiv:1702.00124).  Each function cites the section / equation it follows.

Modules
-------
lattice     geometry, boundary phases, gamma matrices, su(3) generators
wilson      Wilson hopping operator D, M = 1 - kappa D, even-odd M-hat,
            K = M^dag M, K-hat, J = K-hat + mu^2
solver      conjugate gradient (Sec. 2: inversion of K)
poly        Chebyshev filter polynomial P approximating 1/x (Sec. 2)
su3         exp(i eps P), reunitarisation, coefficient <-> matrix maps
gauge       Wilson plaquette action and its force
force       the link-derivative bilinear of Re(A^dag D C)
action      the pseudofermion action terms, heatbaths and forces
            (two-flavour, mass-preconditioned, polynomial-filtered)
integrator  the generalised multi-time-scale integrator (Sec. 3.2)
hmc         one HMC trajectory with Metropolis (Sec. 2)

Pins (what ties each part to something other than itself) are the
``-m "not gpu"`` tests in ``tests/test_oracle_*.py``.  Parity is pinned for
every function here; the paper's cost values C = N_mat/P_acc (Sec. 3.3) are
the only quantity that stays unpinned, since they need an ensemble that is not
available.
"""
