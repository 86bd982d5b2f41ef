"""CPU oracle of the view-tied Gaussian splatting renderer.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the CPU
baseline of ``bench.py``; the product path never imports it.  The C source
(``oracle.c``) is compiled by :func:`build` with gcc (no FMA contraction, no
fast-math) into ``liboracle.so`` beside it.
"""
from .api import *  # noqa: F401,F403
from .api import build, lib  # noqa: F401
