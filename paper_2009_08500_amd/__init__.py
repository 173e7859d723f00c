"""MI355X-native RoadRunner transit light curves (Parviainen 2020).

The light-curve path runs in hand-written HIP kernels for gfx950 behind the C
ABI of ``librr.so`` (declared in ``include/rr.h``); this package is the thin
Python binding over it.  Importing it loads the library and fails loudly if
the library has not been built.
"""

from ._lib import (RR_FP64, RR_MIXED, RRError, lib)  # noqa: F401
from .api import (DEFAULT_GRID, NUM_VARIANTS, Evaluator, RRLogLik, RRLogLikLD, Tables,  # noqa: F401
                  TimeSeries, evaluate, evaluate_direct, evaluate_ld, evaluate_small_planet,
                  evaluate_unregistered,
                  flux_at_z, loglik_grad, loglik_grad_ld, loglik_grad_small_planet,
                  make_grid, select_variant)
from . import ldlaws  # noqa: F401,E402
from .tuning import tune_grid  # noqa: F401,E402

from .serving import Server  # noqa: F401,E402

lib()  # load now: a missing build is an import error, never a fallback
