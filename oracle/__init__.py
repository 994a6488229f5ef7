"""FP64 CPU oracle for AR-BC preconditioned Landweber deblurring.

Test infrastructure only: imported by the test-suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the product library."""
from .ar_oracle import *  # noqa: F401,F403
from .ar_oracle import __all__  # noqa: F401
from . import learned_oracle as learned  # noqa: F401,E402
from . import bc_oracle as bc  # noqa: F401,E402
