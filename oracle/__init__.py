"""FP64 CPU oracle for the chi0 -> Dyson -> S(q,w) -> F(q,tau) path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call or link anything in this package.  Only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it.

The oracle is a plain, slow, obviously-correct NumPy implementation of the
quantities the GPU path computes, written from their definitions:

  * Adler-Wiser Kohn-Sham response chi0_GG'(q,w) (textbook linear-response
    TDDFT; the paper names linear-response TDDFT in Sec. 1 and the
    Lorentzian broadening eta there),
  * Dyson equation chi = (1 - chi0 K)^-1 chi0 with K = v + f_xc (the
    adiabatic kernel of Sec. A.1),
  * fluctuation-dissipation theorem, Eq. (8), with detailed balance,
  * two-sided Laplace transform to the ITCF, Eq. (1).

and, on top of S and F: the eta-convergence metrics and reference eta
(Sec. 2, Eq. 2; ``eta``), the constraints-based attenuation of narrow-band
fluctuations (Sec. 3, Eqs. 3-7; ``attenuation``), the dielectric properties
from S (Eqs. A-1, A-2; ``dielectric``) and the Kubo-Greenwood route
(Sec. A.3; ``kubo_greenwood``).

It shares no code with the HIP path; only ``workloads`` (seeded problem
definitions) serves both.  Library primitives used as single steps: dense
matrix products, ``numpy.linalg.eigh``/``solve``/``qr``, ``numpy.polyfit``
and ``numpy.fft``.

Each function's pins (closed forms, sum rules, symmetries, brute force) live
in ``tests/test_oracle_*.py``.  Functions with no independent pin say
"parity unpinned" in their docstring.
"""
from .lattice import (reciprocal, mp_kpoints, gsphere, kq_map,
                      response_basis)
from .states import (build_states, fermi, find_mu, States)
from .response import (transitions, pair_densities, chi0, coulomb, dyson,
                       dsf, itcf, Transitions)
from .xc import fxc_alda, exc_pw92, density_on_grid, fxc_matrix
from .pipeline import run_q, run_workload, QResult
