"""MI355X-native 3D-RISM initialisation: solute-solvent potential, long-range
asymptotics and their adjoint, as hand-written HIP kernels for gfx950 behind
the C-ABI library ``librism.so``.

The HIP binding is imported lazily so that ``workloads`` can be used without
loading the shared library."""

__all__ = ["workloads"]


def __getattr__(name):
    if name in ("potential", "asymptotics", "initialize", "potential_backward",
                "RismPotential", "Opts", "lib"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
