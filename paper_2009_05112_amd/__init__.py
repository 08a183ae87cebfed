"""MI355X (gfx950) implementation of the per-iteration hot path of vegas+
(G. P. Lepage, arXiv:2009.05112): HIP kernels behind the C ABI in
include/vegasp.h, with a thin ctypes binding.

    from paper_2009_05112_amd import Context, Problem, workloads
"""
from . import workloads  # noqa: F401  (seeded inputs; no method arithmetic)


def __getattr__(name):
    # the binding loads libvegasp.so on first use and raises if it is missing
    if name in ("Context", "Problem", "Server", "integrate", "VegaspError", "lib", "declared_symbols"):
        from . import _binding
        return getattr(_binding, name)
    raise AttributeError(name)
