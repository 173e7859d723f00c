"""FP64 CPU oracle for the RoadRunner transit model (Parviainen 2020).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct reference that the HIP implementation is checked against.  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  The product library never imports, links or calls it, and it
shares no code with the HIP path (no kernels, headers, helpers, tables or
constants).

Modules
-------
roadrunner  Oracle-A: the method step by step, in the order of Sects. 2-3
            (z-grid, annulus weights over (k, g), LD tables, k- and
            g-interpolation, Eq. 5), plus the orbit and supersampling that
            Sect. 4 describes; also the per-row LD, direct-model
            (Sect. 3.1.1) and small-planet (Sect. 3.4.2) forms.  This is the
            GPU parity target.
exact       Oracle-B: the plain definition of the transit signal (Eq. 1-2)
            integrated with adaptive quadrature, and a 2-D brute-force
            integral over the planet disk for tiny inputs.  It pins Oracle-A's
            discretisation error.
orbit       Keplerian orbit -> projected separation, plus an independent
            bisection Kepler solver used as a pin.
gradient    Analytic gradient of the Gaussian log-likelihood of Oracle-A's
            light curve, and a central finite-difference driver.
analytic    The analytic quadratic limb-darkening transit model of Mandel &
            Agol (2002), which the paper uses to measure its accuracy; a pin
            for both oracles.
"""

from . import orbit, roadrunner, exact, analytic  # noqa: F401
