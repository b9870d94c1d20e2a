"""FP64 CPU oracle for the lattice ES-BGK model (Meng, Zhang, Hadjiconstantinou,
Radtke and Shan, "Lattice ellipsoidal statistical BGK model for thermal
non-equilibrium flows").

THIS PACKAGE IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it. The product path (the HIP
library and its Python binding) never imports, calls or links anything here,
and nothing here imports the product path.

The oracle is written in plain numpy, in float64, directly from the paper:

* ``quadrature`` - the 1-D Gauss-Hermite rule (Sec. 2.2, eq. weight) and the
  two on-lattice velocity sets D2Q37 / D3Q39 derived by moment matching to the
  Gaussian weight function (the quadrature-degree requirement of Sec. 2.2).
* ``hermite``    - Grad's tensor Hermite polynomials chi^(n) (Sec. 2.2,
  eqs. approxf, an).
* ``model``      - the ES-BGK pieces: the tensor lambda (Sec. 2.1, eq. cfeq),
  the closed-form coefficients a_ES^(n) (Sec. 2.2), the Hermite projection
  (eq. approxfeq), the body-force expansion (Sec. 2.2), the truncated
  Maxwellian S(T,u) (Sec. 3.2, eq. feq0), the relaxation time (Sec. 2.2) and
  the macroscopic moments (Sec. 2.1, eq. mac).
* ``lattice``    - the space-time scheme: exact on-lattice streaming with the
  diffuse (Maxwell, gamma = 1) wall of Sec. 3.2, collision and force with a
  forward-Euler or trapezoidal time discretisation of eq. lbgk, macroscopic
  output and FP64 reductions.
* ``offlattice`` - the paper's own scheme (Sec. 3.1) on its own velocity set:
  the 6-point Gauss-Hermite product set, forward Euler in time and TVD minmod
  finite-volume fluxes in space, periodic boundaries.

Where the paper is silent or ambiguous, the reading taken is stated in the
docstring of the function that depends on it.
"""

import importlib as _il

for _m in ("quadrature", "hermite", "model", "lattice", "offlattice"):
    try:
        _il.import_module(f"{__name__}.{_m}")
    except ModuleNotFoundError:
        pass
