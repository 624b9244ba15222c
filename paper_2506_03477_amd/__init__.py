"""MI355X (gfx950) implementation of the imaginary-axis polarization chi0 and
the dielectric step of quasiparticle self-consistent GW (arXiv 2506.03477),
with the exchange self-energy and the imaginary-axis part of the correlation
self-energy on the same matrix-core machinery.

The computation lives in libchi0.so (hand-written HIP kernels behind the C ABI
of include/chi0.h); this package is its ctypes binding.
"""
from ._lib import (Block, Problem, SigxBlock, SigxProblem, SigcBlock, SigcProblem, HistSpec, Context, Chi0Error, load, header_functions, tile_choice, PREC, ZTYPE,
                   CHI0_OK, CHI0_EINVAL, CHI0_ENOMEM, CHI0_EDEVICE, CHI0_ENOTHPD,
                   CHI0_ESINGULAR, CHI0_EUNSUPPORTED)

__all__ = ["Block", "Problem", "SigxBlock", "SigxProblem", "SigcBlock", "SigcProblem", "HistSpec", "Context", "Chi0Error", "load", "header_functions", "tile_choice", "PREC",
           "ZTYPE", "CHI0_OK", "CHI0_EINVAL", "CHI0_ENOMEM", "CHI0_EDEVICE",
           "CHI0_ENOTHPD", "CHI0_ESINGULAR", "CHI0_EUNSUPPORTED"]
