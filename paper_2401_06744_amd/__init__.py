"""MI355X (gfx950) homogeneous diffusion inpainting: reduced full multigrid with an
optimized restricted additive Schwarz smoother, behind the C ABI of
``include/inpaint.h``.  ``binding`` is the ctypes layer over ``libinpaint.so``;
``synth`` draws seeded synthetic inputs."""
from . import binding  # noqa: F401
from .binding import (  # noqa: F401
    inpaint_solve, inpaint_solve_ex, inpaint_rel_res, inpaint_last_error, inpaint_version,
    inpaint_hierarchy_size, make_opts,
)
