"""CPU oracle for Stone's SIP (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The library path never does.
"""
from .oracle import (  # noqa: F401
    build, factor, residual, residual_f32, forward, backward, forward_f32, backward_f32,
    iterate, solve, norm2, blocks,
)
