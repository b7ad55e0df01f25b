"""Reference typemap walker (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does.
"""
from .oracle import OracleError, OType, build, build_type, load  # noqa: F401
