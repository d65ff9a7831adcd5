"""List-based D3Q19 TRT lattice Boltzmann for AMD Instinct MI355X (gfx950).

A sparse representation (fluid cells only, 1-D list + 18-entry adjacency with
implicit bounce-back) is assembled on the GPU from a flag field in a chosen
cell ordering, and the two-relaxation-time pull sweep runs over it -- the
method of Wittmann, Zeiser, Hager, Wellein, "Domain decomposition and
locality optimization for large-scale lattice Boltzmann simulations".

All computation runs in the HIP library ``liblbm.so`` (C ABI in
include/lbm.h); this package marshals torch tensors to it.  Importing the
package does not load the library; the first call does, and raises if it has
not been built.
"""
from .inputs import Geometry  # noqa: F401  (seeded synthetic inputs)


def __getattr__(name):
    # lazy: keep `import paper_1111_1129_amd.inputs` free of torch and HIP
    if name in ("build", "init", "step", "moments", "params", "set_state", "count_fluid",
                "partition_stats", "aligned_stride", "Lattice", "State", "Batch",
                "compress", "step_c16", "narrow", "step_c8", "Compressed", "StepGraph", "InplaceState",
                "init_inplace", "step_inplace"):
        from . import lattice
        return getattr(lattice, name)
    if name in ("PermeabilityFn", "adjoint_gradient", "forward_states"):
        from . import adjoint
        return getattr(adjoint, name)
    if name in ("tune_layout", "tune_ordering"):
        from . import tune
        return getattr(tune, name)
    if name in ("lbm_build_adjacency", "lbm_init", "lbm_step", "lbm_step_adjoint", "lbm_moments",
                "lbm_partition_stats", "lbm_compress_adjacency", "lbm_step_c16",
                "lbm_step_inplace", "lbm_step_adjoint_c16", "lbm_step_adjoint_c8",
                "lbm_narrow_codes", "lbm_step_c8", "lbm_check_adjacency",
                "lbm_step_inplace_c8", "lbm_version",
                "LbmError"):
        from . import _native
        return getattr(_native, name)
    raise AttributeError(name)
