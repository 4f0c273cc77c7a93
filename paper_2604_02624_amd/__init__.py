"""dpx: multi-wavelength diffractive propagation through cascaded dielectric phase layers and
its gradient, as hand-written HIP for AMD Instinct MI355X (gfx950) behind a C ABI
(include/dpx.h).  Importing the package loads nothing; ``paper_2604_02624_amd.dpx`` loads the
library on first use and raises if it is missing.

Modules: ``dpx`` (binding of every C call, ``Plan``), ``train`` (Adam training loop with
minibatches, channel swapping, vaccination and quantised heights), ``robustness``
(misalignment and detuning tools), ``layer_models`` (phase-only layers of Eq. 3),
``workloads`` (seeded synthetic inputs), ``build`` (compiles libdpx.so), ``profiling``
(summaries of rocprofv3 output)."""

__all__ = ["dpx", "workloads", "build", "train", "robustness", "layer_models", "profiling"]
