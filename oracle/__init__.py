"""FP64 CPU oracle of the SG-Splatting rasteriser.

TEST INFRASTRUCTURE ONLY: imported by `tests/`, the package smoke check and
the benchmark's CPU-baseline leg, never by the product path.  It shares no
code with the HIP path.  See `forward.py` for the forward definition and the
readings taken where the paper is silent, `backward.py` for the analytic
backward and finite differences, `sh.py` for the SH basis.
"""
from .forward import (Pre, Image, preprocess, emit_pairs, sort_pairs, tile_ranges,
                     render, render_batch, render_pixel, pixel_list, blend_image,
                     ALPHA_BAND, T_BAND)
from .backward import (blend_backward, preprocess_backward, l1_loss, render_and_grad,
                       fd_grad, signature, pixel_backward)
from .sh import sh_basis, sh_basis_grad

__all__ = ["Pre", "Image", "preprocess", "emit_pairs", "sort_pairs", "tile_ranges",
           "render", "render_batch", "render_pixel", "pixel_list", "blend_image",
           "ALPHA_BAND", "T_BAND", "blend_backward", "preprocess_backward", "l1_loss",
           "render_and_grad", "fd_grad", "signature", "pixel_backward", "sh_basis",
           "sh_basis_grad"]
