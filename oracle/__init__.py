"""FP64 CPU oracle for the splattable-neural-primitive rasterizer.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product path (the HIP
library and its Python binding) never calls it and shares no code with it.

It is a plain, slow, direct reading of the paper (Splat the Net, ICLR 2026):
ellipsoid-bounded primitives (Sec. 3.1), the cosine density MLP (Eq. 5-6), the
exact line integral of that density through its antiderivative (Eq. 7-8), the
clamped splatting kernel (Eq. 9) and front-to-back alpha blending of the
depth-sorted primitives (Eq. 3-4).  Everything is float64.  Readings of points
the paper leaves open are documented per function.
"""
from .geometry import quat_to_rotmat, pixel_rays, intersect_ellipsoid  # noqa: F401
from .density import (antiderivative, chord_integral, chord_integral_literal,  # noqa: F401
                      chord_integral_quadrature)
from .keys import project_all, tile_lists, sorted_instances, tile_ranges  # noqa: F401
from .render import render_view, render_views, l1_loss, RenderOptions  # noqa: F401
