"""dpx: multi-wavelength diffractive propagation through cascaded dielectric phase layers and
its gradient, as hand-written HIP for AMD Instinct MI355X (gfx950) behind a C ABI
(include/dpx.h).  Importing the package loads nothing; ``paper_2604_02624_amd.dpx`` loads the
library on first use and raises if it is missing."""

__all__ = ["dpx", "workloads", "build"]
