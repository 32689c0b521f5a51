"""GPAIR direct forward/adjoint operators for MI355X (gfx950).

``paper_2602_03893_amd.inputs`` (seeded synthetic workloads) imports without
the native library.  Everything else (``Plan``, ``GpairForward``, the update
helpers) loads ``libgpair.so`` on first use and raises ``ImportError`` when it
has not been built: there is no CPU fallback.
"""

__version__ = "0.1.0"

_LAZY = {
    "Plan": ("api", "Plan"),
    "pgd_update": ("api", "pgd_update"),
    "adam_update": ("api", "adam_update"),
    "npc_map": ("api", "npc_map"),
    "npc_grad": ("api", "npc_grad"),
    "vcr": ("api", "vcr"),
    "cawr_rate": ("api", "cawr_rate"),
    "peak_probe": ("api", "peak_probe"),
    "GpairError": ("_lib", "GpairError"),
    "GpairForward": ("autograd", "GpairForward"),
    "gpair_forward": ("autograd", "gpair_forward"),
    "AssaForward": ("autograd", "AssaForward"),
    "assa_forward": ("autograd", "assa_forward"),
    "AnisoForward": ("autograd", "AnisoForward"),
    "aniso_forward": ("autograd", "aniso_forward"),
}


def __getattr__(name):
    if name in _LAZY:
        import importlib
        mod, attr = _LAZY[name]
        return getattr(importlib.import_module(f".{mod}", __name__), attr)
    raise AttributeError(name)
