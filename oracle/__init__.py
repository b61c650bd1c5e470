"""CPU oracle for homogeneous diffusion inpainting (Kaemper, Chizhov, Weickert).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything here; only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP library: it never imports ``paper_2401_06744_amd`` (the seeded input
generators in ``paper_2401_06744_amd.synth`` are passed in by the caller as
plain arrays).

All arithmetic is float64.  See ``oracle.inpaint`` for the functions and the
passage of the paper each one follows.
"""
from .inpaint import *  # noqa: F401,F403
from .inpaint import __all__  # noqa: F401
