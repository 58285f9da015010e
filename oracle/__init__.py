"""Plain FP64 CPU oracle for the hyperspectral DOT Born hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.
The product path (the HIP library and its Python binding) never imports,
calls or links it, and this package never imports the product.

What it computes, each from its plain definition (Saibaba, Kilmer, Miller,
Fantini, "Fast algorithms for hyperspectral diffuse optical tomography"):

* ``model``   - optical model (Sec. 2.1, eqs. for D and the chromophore
                perturbation) and the matrix-free operator's matrices
                written out as sparse matrices (Sec. 2.2 / Sec. 3.1 shifted form);
* ``fields``  - phi = A(lambda)^-1 b for every right-hand side and wavelength:
                dense LU, banded LU, fast diagonalisation (exact on the box),
                and textbook unrecycled restarted GMRES(m);
* ``born``    - the Born operator J_lambda[s,d,k] = -h^3 phi_s(k) phi_d(k)
                (Sec. 2.1 integral equation; rows of H, Sec. 2.2 measurement
                model) and its products J v and J^H w;
* ``pals``    - the parametric level-set shape (Sec. 5, eq. pals), its
                derivative, the data misfit (Sec. 5, eq. minimization) and its
                gradient;
* ``compress``    - the recursive randomized compression of an explicit H
                    (Sec. 4 and its appendix);
* ``reconstruct`` - Alg. opt on an explicit H: contrast least squares and
                    Levenberg-Marquardt steps on the PaLS parameters with
                    discrepancy-principle stopping (Sec. 5).

Every pin against the paper and the mathematics lives in ``tests/``.
"""
from . import model, fields, born, pals  # noqa: F401
