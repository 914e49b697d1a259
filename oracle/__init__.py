"""FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It shares no code with the GPU path.
"""

from .fill_oracle import *  # noqa: F401,F403
from . import dense  # noqa: F401
from . import lanczos  # noqa: F401
from . import strips  # noqa: F401
from . import laplace  # noqa: F401
from . import block_precond  # noqa: F401
