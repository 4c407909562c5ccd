"""Plain FP64 CPU oracle of the Whittaker-Henderson smoother.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library and its Python binding never import it, and it imports nothing from
them: the two sides share no code.
"""

from . import whs_ref  # noqa: F401
